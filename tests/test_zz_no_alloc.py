"""The allocation-free scene entry point (pbdr_scene_create_static): a scene in
the library's static device workspace, for callers that cannot allocate.

Its results must equal those of the same scene in a caller workspace
(pbdr_scene_create) bit for bit, on two calls in a row, the second with a
smaller scene, and one of its substeps must match the FP64 reference.
"""
import os

import numpy as np
import pytest

from paper_2603_14634_amd import binding as B
from paper_2603_14634_amd import scenes

from scene_helpers import touching_bodies

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load_library()


def _check_against_reference(orc, sc, s):
    """One substep of `s` from the scene's initial state against the reference."""
    s.set_state(sc.x, sc.v)
    s.substep(1)
    dg = s.read_debug(B.DEBUG_DELTA).astype(np.float64)
    info = s.info()
    p = orc.params_for(sc, hash_bits=info.hash_bits, nbr_cap=info.nbr_cap, threads=THREADS)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    xo, _, _ = orc.substep(p, rest, sc.x, sc.v)
    err = float(np.abs(dg - (xo - sc.x.astype(np.float64))).max())
    print("[static] %s: displacement error %.3g m (tolerance %.3g)" % (sc.name, err, 1e-5 * sc.radius), flush=True)
    assert err <= 1e-5 * sc.radius


def test_static_scene_equals_a_workspace_scene_on_two_calls(orc):
    first = scenes.drop_cubes(0)                         # 512 particles
    second = touching_bodies([27, 64, 8], seed=5)        # 99 particles
    second.name = "touching [27, 64, 8]"
    assert second.n < first.n
    for sc, frames in ((first, 60), (second, 12)):
        p = B.params_for(sc)
        ref = B.Solver(p, sc.x, sc.v, sc.mass, sc.body_start)
        st = B.Solver(p, sc.x, sc.v, sc.mass, sc.body_start, static_workspace=True)
        assert st.workspace is None
        ref.step(frames)
        st.step(frames)
        xr, vr = ref.read_state()
        xs, vs = st.read_state()
        print("[static] %s (%d particles): %d frames, states equal: %s" % (sc.name, sc.n, frames,
              bool(np.array_equal(xs, xr) and np.array_equal(vs, vr))), flush=True)
        np.testing.assert_array_equal(xs, xr)
        np.testing.assert_array_equal(vs, vr)
        _check_against_reference(orc, sc, st)
        ref.close()
        st.close()


def test_static_scene_rejects_a_scene_beyond_its_workspace():
    sc = scenes.dense_pile(0, n_bodies=3000)              # about 300k particles, well over the static workspace
    with pytest.raises(B.PbdrError) as e:
        B.Solver(B.params_for(sc), sc.x, sc.v, sc.mass, sc.body_start, static_workspace=True)
    assert e.value.status == B.ERR_WORKSPACE
    assert "static workspace" in str(e.value)
