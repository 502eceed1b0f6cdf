/*
 * pbdr.h -- C ABI of the MI355X (gfx950) PBD-R rigid-body solver.
 *
 * PBD-R is the position-based dynamics formulation of "Physically Accurate
 * Rigid-Body Dynamics in Particle-Based Simulation" (arXiv 2603.14634): rigid
 * bodies are groups of equal-radius spheres ("object groups", Sec. III-A);
 * each substep predicts positions, then runs K Jacobi iterations of ground
 * contact, particle-particle contact between different groups, and shape
 * matching (Alg. 1), with the paper's incremental velocity update (Sec. III-B,
 * Eqs. (1)-(3)) and momentum conservation constraint (Sec. III-C, Eqs. (4)-(5)).
 *
 * Conventions
 *  - Units are SI.  Particle arrays are structure-of-arrays FP32: a "[3][N]"
 *    array holds all x components, then all y, then all z.
 *  - Particles are grouped by body: body b owns particles
 *    body_start[b] .. body_start[b+1]-1 (bodies contiguous and non-empty).
 *  - Device memory is owned by the caller.  A scene lives entirely inside one
 *    device workspace of pbdr_scene_bytes() bytes handed to pbdr_scene_create;
 *    the library never allocates or frees device memory.  The library owns only
 *    the opaque host-side pbdr_scene, freed by pbdr_scene_destroy (which does
 *    not touch the workspace).
 *  - All device work is enqueued on the hipStream_t given at creation (NULL
 *    means the null stream).  Calls that return results to the host
 *    synchronise that stream.
 *  - Every call returns a pbdr_status.  Invalid arguments are rejected before
 *    any device work is enqueued.  Conditions found on the device (a neighbour
 *    list over capacity, a non-finite state, a device-side wait that gave up)
 *    are latched in the workspace and reported by the next call that
 *    synchronises (pbdr_scene_read_*, pbdr_scene_check).  The frame in which
 *    one is raised is discarded: the scene's state (x, v) is committed only at
 *    the end of a frame with no latched condition, so it stays at the last
 *    frame completed before the condition, and later pbdr_scene_step calls
 *    leave it there until pbdr_scene_set_state clears the latch.
 *    pbdr_last_error() gives a message for the calling thread's last failure.
 *  - A scene is not thread-safe; distinct scenes may be used from distinct
 *    threads.
 */
#ifndef PBDR_H
#define PBDR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBDR_ABI_VERSION 1
#define PBDR_MAX_PLANES 8
#define PBDR_MAX_BODY_PARTICLES 1024

typedef enum {
    PBDR_OK = 0,
    PBDR_ERR_INVALID_ARG = -1, /* bad pointer, size, body partition or parameter   */
    PBDR_ERR_WORKSPACE = -2,   /* workspace too small or misaligned (256 B)         */
    PBDR_ERR_DEVICE = -3,      /* a HIP runtime call failed, or a device-side wait
                                  gave up (the frame was discarded)                 */
    PBDR_ERR_CAPACITY = -4,    /* a neighbour list exceeded nbr_cap (the frame was
                                  discarded; recreate the scene with a larger cap)  */
    PBDR_ERR_NONFINITE = -5,   /* a position or velocity became NaN/Inf (the frame
                                  was discarded)                                    */
    PBDR_ERR_STATE = -6        /* call not valid in the scene's current state        */
} pbdr_status;

/* pbdr_params.flags */
#define PBDR_FLAG_STD_VELOCITY 0x1u  /* standard PBD velocity (X_{i+1}-X_init)/dt, Sec. III-A */
#define PBDR_FLAG_NO_LIN_MOM 0x2u    /* drop the linear momentum correction, Eq. (4)   */
#define PBDR_FLAG_NO_ANG_MOM 0x4u    /* drop the angular momentum correction, Eq. (5)  */
#define PBDR_FLAG_NO_GRAPH 0x10u     /* enqueue kernels directly instead of replaying a
                                        captured HIP graph per frame                    */
#define PBDR_FLAG_ITERATION_LAUNCHES 0x20u  /* one launch per solver iteration even when the
                                        scene's iteration grid fits the GPU at once (the
                                        one-launch form needs every workgroup resident:
                                        scenes stepped concurrently on other streams
                                        should set this)                                */
#define PBDR_PP_AVG_MAX (0u << 8)    /* pair correction / max(n_p, n_q)  (default)      */
#define PBDR_PP_AVG_OWN (1u << 8)    /* pair correction / n_p                           */
#define PBDR_PP_AVG_NONE (2u << 8)   /* pair corrections summed                         */
#define PBDR_PP_AVG_MASK (3u << 8)

/*
 * Solver parameters.  Zero in a field marked "0 = default" selects the default.
 *  dt_frame, substeps  the substep length of Alg. 1 is h = dt_frame / substeps
 *                      (Sec. IV-B runs 100 Hz frames with 10 substeps).
 *  iterations          solver iterations K per substep (Alg. 1 while loop).
 *  gravity             uniform acceleration, part of f_ext (Alg. 1, first loop).
 *  friction_mu         Coulomb coefficient, static = kinetic (Tables I, II).
 *  radius              common particle radius r; spheres touch at 2r.
 *  search_radius       neighbour predicate radius R_s, 0 = 2r.
 *  cell_size           hash-grid cell edge a >= R_s, 0 = R_s * (1 + 2^-10).
 *  grid_origin         hash-grid origin o.
 *  hash_bits           key bits k in [6, 28], 0 = max(10, ceil(log2(8N))).
 *  planes              half-spaces n.x >= d + r, rows (nx, ny, nz, d), |n| = 1.
 *  nbr_cap             neighbour-list capacity per particle, 0 = 32, max 64.
 */
typedef struct {
    double dt_frame;
    int32_t substeps;
    int32_t iterations;
    double gravity[3];
    double friction_mu;
    double radius;
    double search_radius;
    double cell_size;
    double grid_origin[3];
    int32_t hash_bits;
    int32_t n_planes;
    double planes[PBDR_MAX_PLANES][4];
    uint32_t flags;
    int32_t nbr_cap;
} pbdr_params;

/*
 * Initial scene, in HOST memory; copied during pbdr_scene_create, so the
 * caller may free it on return.
 *  x, v        [3][N] positions (m) and velocities (m/s).
 *  mass        [N] particle masses (kg), finite and > 0.
 *  body_start  [B+1] body partition, body_start[0] = 0, body_start[B] = N,
 *              strictly increasing; at most PBDR_MAX_BODY_PARTICLES per body.
 *  rest_q      optional [3][N] rest offsets q_p of shape matching (to resume a
 *              saved scene); NULL derives them from x as x - (mass-weighted
 *              body centre), in FP64 (Sec. III-C).
 */
typedef struct {
    int32_t n_particles;
    int32_t n_bodies;
    const float* x;
    const float* v;
    const float* mass;
    const int32_t* body_start;
    const float* rest_q;
} pbdr_scene_desc;

/* Values the scene derived from its parameters (defaults resolved). */
typedef struct {
    int32_t n_particles;
    int32_t n_bodies;
    int32_t hash_bits;
    int32_t nbr_cap;
    double substep_h;
    double search_radius;
    double cell_size;
    int32_t waves_per_block;      /* iteration kernel: 64-lane waves per workgroup */
    int32_t iteration_blocks;     /* iteration kernel: workgroups per launch */
    int32_t max_body_particles;
    int32_t iteration_kernel;     /* 0: register-rich variant, one launch per iteration;
                                     1: 80-VGPR variant, taken when the grid
                                     oversubscribes the GPU; 2: all K iterations of a
                                     substep in one launch (the grid is resident at
                                     once, K < 64) */
    size_t workspace_bytes;
} pbdr_scene_info;

typedef struct pbdr_scene pbdr_scene;

/* ABI version this library implements (PBDR_ABI_VERSION). */
int32_t pbdr_abi_version(void);

/* Device conditions a workspace latches (bits).  A frame that raises any of
 * them is discarded (see Conventions). */
#define PBDR_COND_CAPACITY 0x1u      /* a neighbour list exceeded nbr_cap            */
#define PBDR_COND_NONFINITE 0x2u     /* a position or velocity became NaN/Inf        */
#define PBDR_COND_INTERNAL 0x4u      /* an internal consistency check failed (a key
                                        sort position out of range, a pool scene
                                        that did not fit its launch shape)          */
#define PBDR_COND_PARTNER_WAIT 0x8u  /* a one-launch iteration's wait for a contact
                                        partner gave up (its workgroups were not all
                                        resident together)                           */

/* The status that the synchronising calls return for a set of latched
 * conditions, and the message they leave for pbdr_last_error: PBDR_OK for
 * none; PBDR_ERR_CAPACITY before PBDR_ERR_NONFINITE before PBDR_ERR_DEVICE
 * (the waits), since an overflowing list can make partner waits give up.
 * Host only; no device work. */
pbdr_status pbdr_condition_status(uint32_t conditions);

/* Message describing the calling thread's last failed call ("" if none). */
const char* pbdr_last_error(void);

/* Device workspace bytes a scene of this size needs; 0 if the parameters are
 * invalid (see pbdr_last_error). */
size_t pbdr_scene_bytes(const pbdr_params* params, int32_t n_particles, int32_t n_bodies);

/* Creates a scene in dev_workspace (device pointer, 256-byte aligned,
 * ws_bytes >= pbdr_scene_bytes).  Copies desc into the workspace on
 * hip_stream (a hipStream_t, or NULL) and synchronises it.  On success *out
 * receives the handle. */
pbdr_status pbdr_scene_create(const pbdr_params* params, const pbdr_scene_desc* desc,
                              void* dev_workspace, size_t ws_bytes, void* hip_stream,
                              pbdr_scene** out);

/* Per-particle external acceleration a_p = w_p f_ext,p (Alg. 1, first loop),
 * added to gravity: a DEVICE pointer to [3][N] floats that the scene reads at
 * every substep until replaced, or NULL for none.  The caller keeps it alive. */
pbdr_status pbdr_scene_set_accel(pbdr_scene* scene, const float* accel_dev);

/* Moves the scene's work to another stream (hipStream_t or NULL for the
 * default stream): waits for the work already enqueued on the current one,
 * then enqueues every later call on hip_stream.  Lets a scene be created on a
 * stream of its own (creation synchronises that stream) and then join a
 * stream that other work keeps busy.  PBDR_ERR_DEVICE if the wait fails. */
pbdr_status pbdr_scene_set_stream(pbdr_scene* scene, void* hip_stream);

/* Advances n_frames frames (asynchronous).  A frame is `substeps` substeps of
 * Alg. 1, each the integration step, the neighbour search and `iterations`
 * Jacobi iterations of ground and particle contact and shape matching with
 * the velocity update of Sec. III-B and the momentum constraint of Sec. III-C
 * (frames of substeps as in Sec. IV-B).  The state is committed at the end of
 * every frame that latched no device condition; see Conventions.  Frames are
 * replayed from a captured HIP graph unless PBDR_FLAG_NO_GRAPH.
 * PBDR_ERR_INVALID_ARG for n_frames < 0; PBDR_ERR_DEVICE if a launch fails. */
pbdr_status pbdr_scene_step(pbdr_scene* scene, int32_t n_frames);

/* Advances n_substeps substeps of Alg. 1 as one frame (asynchronous; the
 * state is committed after the last of them); for substep-level checks. */
pbdr_status pbdr_scene_substep(pbdr_scene* scene, int32_t n_substeps);

/* Replaces positions and velocities ([3][N] each; host pointers if
 * on_device == 0, device pointers otherwise) and clears the latched device
 * conditions.  Bodies and rest pose are kept. */
pbdr_status pbdr_scene_set_state(pbdr_scene* scene, const float* x, const float* v, int32_t on_device);

/* Copies positions and velocities out ([3][N] each, either may be NULL) and
 * synchronises; returns any latched device condition. */
pbdr_status pbdr_scene_read_state(pbdr_scene* scene, float* x, float* v, int32_t on_device);

/* Per-body state of the current x, v, to HOST arrays (any may be NULL; B =
 * n_bodies), computed on the device with FP64 sums over each body:
 *   com  [B][3]  centre of mass c = sum m x / M;
 *   rot9 [B][9]  row-major rotation of shape matching for this pose (Sec.
 *                III-C): the proper rotation maximising tr(R^T A) with
 *                A = sum m (x - c) q^T against the rest offsets q, so that
 *                x - c ~ R q (evaluated in FP32 from the normalised A;
 *                identity for A = 0, unspecified for bodies on a line);
 *   P    [B][3]  linear momentum sum m v;
 *   L    [B][3]  angular momentum about the centre, sum m (x - c) x v.
 * Synchronises; returns any latched device condition. */
pbdr_status pbdr_scene_read_bodies(pbdr_scene* scene, double* com, double* rot9, double* P, double* L);

/* Rest offsets q [3][N] (host), for checkpoints: a scene created from a saved
 * state with these offsets continues identically. */
pbdr_status pbdr_scene_read_rest(pbdr_scene* scene, float* rest_q);

/* Synchronises and returns any latched device condition; *max_neighbours (if
 * not NULL) receives the largest neighbour count seen since creation. */
pbdr_status pbdr_scene_check(pbdr_scene* scene, int32_t* max_neighbours);

/* Neighbour-list statistics since creation (or the last set_state):
 * largest length and mean length over all particle-substeps (synchronises). */
pbdr_status pbdr_scene_neighbour_stats(pbdr_scene* scene, int32_t* max_neighbours, double* mean_neighbours);

/* Debug buffers of the last substep, copied to HOST memory (synchronises):
 *  PBDR_DEBUG_XT          float [3][N] FP32 predicted positions (index input)
 *  PBDR_DEBUG_KEYS        uint32 [N]   cell key of each particle
 *  PBDR_DEBUG_SORTED      uint32 [N]   particle ids sorted by (key, id): the
 *                                      order of the substep's radix sort
 *  PBDR_DEBUG_CELL_START  uint32 [2^k] first sorted slot of each key (for an
 *                                      empty key, that of the next occupied
 *                                      key, or N)
 *  PBDR_DEBUG_CELL_COUNT  uint32 [2^k] particles per key
 *  PBDR_DEBUG_NBR_COUNT   uint32 [N]   neighbour-list lengths
 *  PBDR_DEBUG_NBR         uint32 [nbr_cap][N] lists, slot-major, ascending
 *  PBDR_DEBUG_DELTA       float [3][N] X_K - X_init of the last substep, before
 *                                      the final FP32 rounding of the positions */
enum {
    PBDR_DEBUG_XT = 1,
    PBDR_DEBUG_KEYS = 2,
    PBDR_DEBUG_SORTED = 3,
    PBDR_DEBUG_CELL_START = 4,
    PBDR_DEBUG_CELL_COUNT = 5,
    PBDR_DEBUG_NBR_COUNT = 6,
    PBDR_DEBUG_NBR = 7,
    PBDR_DEBUG_DELTA = 8
};
pbdr_status pbdr_scene_read_debug(pbdr_scene* scene, int32_t what, void* dst_host);

/* Measurement aid: enqueues n_launches back-to-back launches of the solver
 * iteration kernel on the buffers of the last substep.  A launch is one Jacobi
 * iteration of Alg. 1 over all bodies, as the substep itself does K times; for
 * a scene whose substep runs all K iterations as one launch (iteration_kernel
 * 2 in pbdr_scene_info), it is that launch (preceded by a small kernel that
 * resets the launch's synchronisation flags).  The state (x, v) is unchanged;
 * the next substep overwrites the iteration buffers.  Requires at least one
 * completed substep (else PBDR_ERR_STATE). */
pbdr_status pbdr_scene_launch_iterations(pbdr_scene* scene, int32_t n_launches);

/* Measurement aid: as pbdr_scene_launch_iterations, with a pair of HIP events
 * bound to each launch's own dispatch (begin and end timestamps of the kernel,
 * no marker packets in between); waits for the last launch and writes the
 * duration of launch i, in microseconds, to out_us[i] (host array of
 * n_launches floats, owned by the caller).  1 <= n_launches <=
 * PBDR_MAX_TIMED_LAUNCHES, else PBDR_ERR_INVALID_ARG; PBDR_ERR_STATE before the
 * first substep; PBDR_ERR_DEVICE if an event or a launch fails.  Blocks the
 * calling thread until the launches have finished. */
#define PBDR_MAX_TIMED_LAUNCHES 4096
pbdr_status pbdr_scene_time_iterations(pbdr_scene* scene, int32_t n_launches, float* out_us);

/* Resolved parameters and sizes. */
pbdr_status pbdr_scene_info_get(const pbdr_scene* scene, pbdr_scene_info* out);

/* Frees the host handle (and any captured graph).  The workspace is untouched. */
void pbdr_scene_destroy(pbdr_scene* scene);

/* Size of the static device workspace of pbdr_scene_create_static. */
#define PBDR_STATIC_WORKSPACE_BYTES (128u << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): a scene as
 * pbdr_scene_create makes it, placed in the library's own static device
 * workspace of PBDR_STATIC_WORKSPACE_BYTES bytes instead of a caller
 * workspace.  Every device the library runs on holds that workspace until the
 * process ends.
 *  - A scene whose pbdr_scene_bytes exceeds PBDR_STATIC_WORKSPACE_BYTES is
 *    rejected with PBDR_ERR_WORKSPACE before any device work.
 *  - Nothing is allocated: no hipMalloc or hipFree, no allocating library
 *    routine, and the scene's host record is one of the library's own (one
 *    per device).  The scene steps by direct kernel launches (pbdr_scene_step
 *    never captures a graph for it, which would allocate).
 *  - One static scene per device at a time: a later call on the same device
 *    waits for the earlier static scene's work and then replaces it in the
 *    same workspace and host record, so the earlier handle refers to the new
 *    scene.  Calls that overlap on one device race.
 *  - The inputs (desc, host memory) are as for pbdr_scene_create; every state
 *    in the workspace that must start cleared is cleared by this call.  Every
 *    other pbdr_scene_* call works on the returned handle as on any scene;
 *    pbdr_scene_destroy releases it.
 */
pbdr_status pbdr_scene_create_static(const pbdr_params* params, const pbdr_scene_desc* desc,
                                     void* hip_stream, pbdr_scene** out);

/* ------------------------------------------------------------------------
 * Scene pools: many independent small scenes stepped together.
 *
 * A pool holds up to max_scenes scenes of at most PBDR_POOL_MAX_PARTICLES
 * particles and PBDR_POOL_MAX_BODIES bodies each, in arenas of max_particles
 * particles and max_bodies bodies, all inside one device workspace owned by
 * the caller (pbdr_pool_bytes).  Each scene is one workgroup that runs every
 * substep of a step call on its own (Alg. 1 as for a single scene), so a
 * call is a handful of launches however many scenes are resident.  Scenes of
 * up to 8192 particles, 64 bodies and 128 slots of 64 lanes (see
 * pbdr_pool_set_tuning) keep their particles in registers, in 7 size classes
 * whose launch shape is tunable; larger ones run a kernel that keeps them in
 * global memory.  Scenes
 * share the pool's pbdr_params (time step, substeps, iterations, radius,
 * planes, flags, nbr_cap; hash_bits and PBDR_FLAG_NO_GRAPH are ignored) and
 * bring their own gravity and friction coefficient.
 *
 * A scene's result depends only on the scene: it is bitwise the same alone
 * or among others and for every launch shape the tuner may choose.
 * Admission: pbdr_pool_add fails with PBDR_ERR_CAPACITY when no slot, no
 * contiguous particle range or no body range is free; pbdr_pool_info reports
 * what is free.  Slots are reused after pbdr_pool_remove.
 * ------------------------------------------------------------------------ */
#define PBDR_POOL_MAX_PARTICLES 65535
#define PBDR_POOL_MAX_BODIES 256
#define PBDR_POOL_CLASSES 7      /* register-resident size classes: class c holds scenes of n <= 128 << c */
#define PBDR_POOL_LANES 4        /* independent launch lanes (see pbdr_pool_step_slots_on) */

typedef struct pbdr_pool pbdr_pool;

/* One scene for a pool, in HOST memory (copied by pbdr_pool_add; the caller
 * may free it on return).  x, v [3][N], mass [N], body_start [B+1] as in
 * pbdr_scene_desc; rest offsets are derived from x in FP64. */
typedef struct {
    int32_t n_particles;
    int32_t n_bodies;
    const float* x;
    const float* v;
    const float* mass;
    const int32_t* body_start;
    double gravity[3];
    double friction_mu;
} pbdr_pool_scene_desc;

typedef struct {
    int32_t max_scenes, scenes_used;
    int32_t max_particles, particles_used, largest_free_particles;
    int32_t max_bodies, bodies_used, largest_free_bodies;
    int32_t max_scene_particles;   /* largest scene this device can hold (LDS of its class) */
    size_t workspace_bytes;
} pbdr_pool_info;

/* Device workspace bytes of a pool; 0 if invalid (see pbdr_last_error). */
size_t pbdr_pool_bytes(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies);

/* Creates an empty pool in dev_workspace (256-byte aligned, >= pbdr_pool_bytes)
 * working on hip_stream (hipStream_t or NULL); synchronises it. */
pbdr_status pbdr_pool_create(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies,
                             void* dev_workspace, size_t ws_bytes, void* hip_stream, pbdr_pool** out);

/* Adds a scene; *slot receives its slot.  The upload is enqueued on the pool's
 * stream (asynchronous).  PBDR_ERR_CAPACITY if it does not fit now. */
pbdr_status pbdr_pool_add(pbdr_pool* pool, const pbdr_pool_scene_desc* desc, int32_t* slot);

/* Frees a slot and its arena ranges (its data is no longer readable). */
pbdr_status pbdr_pool_remove(pbdr_pool* pool, int32_t slot);

/* Advances every resident scene by n_frames frames (asynchronous). */
pbdr_status pbdr_pool_step(pbdr_pool* pool, int32_t n_frames);

/* Advances the listed slots by frames[j] frames each (0 = stays); the others
 * stay.  For continuous batching, where scenes have different horizons. */
pbdr_status pbdr_pool_step_slots(pbdr_pool* pool, int32_t count, const int32_t* slots, const int32_t* frames);

/* As pbdr_pool_step_slots, but enqueued on hip_stream (a hipStream_t) through
 * launch lane `lane` (0 .. PBDR_POOL_LANES-1).  Launches on different lanes
 * may be in flight together; each lane's calls must be ordered on one stream.
 * Lane 0 runs the size classes of a call side by side on internal streams,
 * the other lanes run them one after another on hip_stream.
 * The work waits for every pbdr_pool_add before the call.  Synchronise that
 * stream before reading or removing the listed slots, and list no slot on two
 * lanes at once.  The pool's own calls use lane 0. */
pbdr_status pbdr_pool_step_slots_on(pbdr_pool* pool, int32_t lane, void* hip_stream, int32_t count,
                                    const int32_t* slots, const int32_t* frames);

/* Launch class of a resident scene: 0 .. PBDR_POOL_CLASSES-1 for the
 * register-resident size classes, PBDR_POOL_CLASSES for the large-scene
 * kernel. */
pbdr_status pbdr_pool_slot_class(const pbdr_pool* pool, int32_t slot, int32_t* cls);

/* Launch class, as pbdr_pool_slot_class reports it, that a scene of this shape
 * would get in this pool, without adding it (host only: body_start [B+1] in
 * host memory).  PBDR_ERR_INVALID_ARG if the shape is malformed or could
 * never be added to this pool. */
pbdr_status pbdr_pool_class_for(const pbdr_pool* pool, int32_t n_particles, int32_t n_bodies,
                                const int32_t* body_start, int32_t* cls);

/* Advances every resident scene by n_substeps substeps (for substep checks). */
pbdr_status pbdr_pool_substep(pbdr_pool* pool, int32_t n_substeps);

/* Copies a scene's positions and velocities ([3][N] each; host or device
 * pointers; either may be NULL), synchronises, and returns the scene's latched
 * device condition (PBDR_ERR_CAPACITY, PBDR_ERR_NONFINITE) if any. */
pbdr_status pbdr_pool_read_state(pbdr_pool* pool, int32_t slot, float* x, float* v, int32_t on_device);

/* Debug buffers of a scene's last substep, to HOST memory (synchronises):
 * PBDR_DEBUG_XT, PBDR_DEBUG_NBR_COUNT, PBDR_DEBUG_NBR ([nbr_cap][N], ascending
 * scene-local ids) and PBDR_DEBUG_DELTA, with the layouts of
 * pbdr_scene_read_debug. */
pbdr_status pbdr_pool_read_debug(pbdr_pool* pool, int32_t slot, int32_t what, void* dst_host);

/* Synchronises; returns the scene's latched device condition and (if not
 * NULL) its largest neighbour count so far. */
pbdr_status pbdr_pool_check(pbdr_pool* pool, int32_t slot, int32_t* max_neighbours);

/* Launch shape of each size class ([PBDR_POOL_CLASSES] arrays): waves per
 * workgroup, 1, 2, 4, 8 or 16.  Bodies are laid out wave-aligned: body b
 * fills ceil(n_b / 64) slots of 64 lanes, and a pooled scene may fill at most
 * 128 slots.  Each launch gives every lane the fewest register sets (1-6 or 8)
 * that cover the class's largest stepped scene; a class whose scenes need more
 * than 8 sets at the set width is widened for that launch. */
pbdr_status pbdr_pool_get_tuning(const pbdr_pool* pool, int32_t* waves);
pbdr_status pbdr_pool_set_tuning(pbdr_pool* pool, const int32_t* waves);

/* Tuner: for every register-resident size class with resident scenes, times each admissible
 * launch shape over n_frames frames of the class's scenes (best of `repeats`)
 * and keeps the fastest.  Scene states are restored afterwards; synchronises.
 * ms_out (may be NULL) receives [PBDR_POOL_CLASSES] the chosen shape's time. */
pbdr_status pbdr_pool_autotune(pbdr_pool* pool, int32_t n_frames, int32_t repeats, double* ms_out);

pbdr_status pbdr_pool_info_get(const pbdr_pool* pool, pbdr_pool_info* out);

/* Frees the host handle; the workspace is untouched. */
void pbdr_pool_destroy(pbdr_pool* pool);

/* ------------------------------------------------------------------------
 * Scene batches: many independent scenes stepped together by the kernels of
 * the single-scene path, every substep of Alg. 1 spread over the whole GPU.
 * For scenes too large for a pool's register-resident classes: a call is one
 * set of launches per frame for all the scenes it steps, where stepping them
 * one by one pays the launches of every scene.
 *
 * The batch holds up to max_scenes scenes, max_particles particles and
 * max_bodies bodies (bodies of at most 1024 particles) in one device
 * workspace owned by the caller (pbdr_batch_bytes).  Each scene has its own
 * hash table in the batch's key arena (4 to 8 keys per particle), so scenes
 * never interact; they share the batch's pbdr_params (time step, substeps,
 * iterations, radius, planes, flags, nbr_cap; gravity, friction_mu and
 * hash_bits are ignored) and bring their own gravity and friction
 * coefficient.  A scene's result depends only on the scene: it is bitwise
 * the same alone or among others.  Calls are enqueued on the batch's stream
 * (asynchronous) and stepped with direct launches (no graph).  Device
 * conditions (capacity, non-finite state) are latched for the whole batch.
 * ------------------------------------------------------------------------ */
typedef struct pbdr_batch pbdr_batch;

typedef struct {
    int32_t max_scenes, scenes_used;
    int32_t max_particles, particles_used, largest_free_particles;
    int32_t max_bodies, bodies_used;
    int32_t max_keys, largest_free_keys;
    size_t workspace_bytes;
} pbdr_batch_info;

/* Device workspace bytes of a batch; 0 if invalid (1 <= max_bodies <=
 * max_particles <= 2^24, 1 <= max_scenes <= 65536, valid params). */
size_t pbdr_batch_bytes(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies);

/* Creates an empty batch in dev_workspace (256-byte aligned, >=
 * pbdr_batch_bytes) working on hip_stream (hipStream_t or NULL); synchronises it. */
pbdr_status pbdr_batch_create(const pbdr_params* params, int32_t max_scenes, int32_t max_particles,
                              int32_t max_bodies, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                              pbdr_batch** out);

/* Adds a scene (desc in host memory, as for pools); *slot receives its slot.
 * Uploads on a stream of the batch's own (waits only for that upload); the
 * next call waits for it.  PBDR_ERR_CAPACITY if no slot, particle, body or
 * key range is free now; PBDR_ERR_INVALID_ARG for a malformed scene or a body
 * of more than 1024 particles. */
pbdr_status pbdr_batch_add(pbdr_batch* batch, const pbdr_pool_scene_desc* desc, int32_t* slot);

/* Frees a slot and its ranges; later calls no longer step it, and a scene
 * added later may reuse the ranges.  Synchronise the batch's stream before
 * removing a scene that a pending call steps. */
pbdr_status pbdr_batch_remove(pbdr_batch* batch, int32_t slot);

/* Advances every resident scene by n_frames frames (asynchronous). */
pbdr_status pbdr_batch_step(pbdr_batch* batch, int32_t n_frames);

/* Advances the listed slots by frames[j] frames each (0 = stays; each slot
 * listed at most once); the others stay.  Scenes with equal remaining frames
 * are stepped together, in as many launch sequences as there are distinct
 * frame counts. */
pbdr_status pbdr_batch_step_slots(pbdr_batch* batch, int32_t count, const int32_t* slots, const int32_t* frames);

/* Advances every resident scene by n_substeps substeps (for substep checks). */
pbdr_status pbdr_batch_substep(pbdr_batch* batch, int32_t n_substeps);

/* Copies a scene's positions and velocities ([3][N] each; host or device
 * pointers; either may be NULL), synchronises, and returns the batch's
 * latched device condition, if any. */
pbdr_status pbdr_batch_read_state(pbdr_batch* batch, int32_t slot, float* x, float* v, int32_t on_device);

/* Debug buffers of a scene's last substep to HOST memory (synchronises):
 * PBDR_DEBUG_XT, PBDR_DEBUG_NBR_COUNT, PBDR_DEBUG_NBR ([nbr_cap][N], scene-local
 * ids ascending) and PBDR_DEBUG_DELTA, with the layouts of pbdr_scene_read_debug. */
pbdr_status pbdr_batch_read_debug(pbdr_batch* batch, int32_t slot, int32_t what, void* dst_host);

/* Synchronises; returns the latched device condition and (if not NULL) the
 * largest neighbour count seen since the batch was created. */
pbdr_status pbdr_batch_check(pbdr_batch* batch, int32_t* max_neighbours);

pbdr_status pbdr_batch_info_get(const pbdr_batch* batch, pbdr_batch_info* out);

/* Synchronises the batch's stream and frees the host handle; the workspace is untouched. */
void pbdr_batch_destroy(pbdr_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* PBDR_H */
