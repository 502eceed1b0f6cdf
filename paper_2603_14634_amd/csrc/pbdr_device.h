// Internal device-side layout shared by the PBD-R kernels and the C-ABI host
// code of libpbdr.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbdr {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kMaxWaves = 16;    // iteration kernel: waves per workgroup (bodies <= 1024 particles)
constexpr int kMaxPlanes = 8;
constexpr int kMaxCap = 64;      // largest supported neighbour-list capacity
constexpr int kScanItems = 16;   // cell-table scan: counts per thread
constexpr int kScanTile = kBlock * kScanItems;

// kErrInternal: the cell-table scan's look-back (or a pool launch shape) gave
// up; kErrWait: a one-launch iteration's wait for a contact partner gave up.
enum : uint32_t { kErrCapacity = 1u, kErrNonFinite = 2u, kErrInternal = 4u, kErrWait = 8u };
// Any of these discards the frame in which it is raised: the committed state
// keeps the last frame completed without one.
constexpr uint32_t kErrDiscard = kErrCapacity | kErrNonFinite | kErrInternal | kErrWait;

enum : uint32_t {
    kFlagStdVelocity = 0x1u,
    kFlagNoLinMom = 0x2u,
    kFlagNoAngMom = 0x4u,
    kAvgShift = 8u,
};

// Device-side error bits, latched until read by the host.
struct Counters {
    uint32_t err;                  // kErr* bits (latched until cleared by the host)
    uint32_t epoch;                // substeps begun (one-launch iterations tag their data with it)
};

// Neighbour-list statistics, one slot per neighbour-kernel workgroup (no
// contended atomics); the host reduces them when asked.
struct NbrStats {
    uint32_t max_nbr;              // largest list length seen
    uint32_t pad;
    unsigned long long sum;        // sum of list lengths
    unsigned long long rows;       // particles counted in sum
};

// FP32 constants of one substep.
struct StepConsts {
    float h, inv_h;
    float g[3];
    float mu, radius, two_r;
    float search_r2;      // fl32(R_s^2)
    float inv_cell;       // fl32(1 / a)
    float origin[3];
    uint32_t key_mask;    // 2^k - 1
    int32_t nbr_cap;
    uint32_t flags;
    int32_t n_planes;
    float plane_n[kMaxPlanes][3];
    float plane_d[kMaxPlanes];
};

// Several independent scenes stepped as one (multi-scene mode): per scene,
// its gravity, friction coefficient, hash-table range and whether it takes
// part in the current launches.
struct MultiScene {
    float g[3];
    float mu;
    uint32_t key_base;        // first key of the scene's table
    uint32_t key_mask;        // table size - 1 (power of two)
    uint32_t active;          // 1: stepped by the current launches
    uint32_t pad;
};

// Device pointers into a scene's workspace.
struct Scene {
    int32_t n, nb;
    uint32_t T;               // 2^k cells
    uint32_t n_scan_tiles;    // ceil(T / kScanTile)
    float* x;                 // [3][N] committed positions: the state after the last clean frame
    float* v;                 // [3][N] committed velocities
    float* x0;                // [3][N] X_init of the current substep (the working state)
    const float* mass;        // [N]
    const int32_t* body;      // [N] body of each particle
    const float* q;           // [3][N] rest offsets
    const int32_t* body_start;// [B+1]
    const float* body_mass;   // [B]
    const int32_t* wave_body; // [n_iter_blocks * waves_per_block] body of each wave, -1 = idle
    const int32_t* body_wave0;// [B] first (global) wave of each body
    const int32_t* block_body;// [2 * n_iter_blocks] first body and body count of each workgroup
    const float* body_mq;     // [B][3] sum of m q over the body (rest frame, ~0)
    int32_t waves_per_block;  // W: iteration workgroup = 64 W threads
    int32_t n_iter_blocks;
    int32_t dense_iterate;    // 1: the iteration grid oversubscribes the GPU (80-VGPR kernel)
    float* dl[2];             // [3][N] X_i - X_init, double buffered
    float* vel[2];            // [3][N] V_i, double buffered
    float* xt;                // [3][N] FP32 predicted positions
    float4* sxt4;             // [N] predicted position and body id (bits) in raw sorted order
    uint32_t* key;            // [N]
    uint32_t* rank;           // [N] slot within the key from the counting pass
    uint32_t* sorted_raw;     // [N] ids grouped by key, arbitrary order within a key
    uint32_t* sorted;         // [N] ids sorted by (key, id), written on demand
    uint32_t* nbr_n;          // [N] neighbour-list length
    uint32_t* nbr;            // [cap][N] neighbour ids, slot-major, ascending
    uint32_t* cell_count;     // [T] per-key counts (zero outside a substep)
    uint2* cells;             // [T + 1] per key: first sorted slot, body signature (the one
                              //     body of all its particles, -1 empty, -2 mixed); the count of
                              //     key k is cells[k + 1].x - cells[k].x, cells[T].x = N
    unsigned long long* tile_state;  // [n_scan_tiles] scan look-back: (status << 32) | value

    float* body_rot;          // [B][9] last rotation of shape matching
    Counters* counters;
    NbrStats* nbr_stats;      // [ceil(N / kBlock)]
    const float* accel;       // [3][N] external acceleration or nullptr
    // multi-scene mode (nullptr otherwise): scene slot of each particle (-1:
    // none) and the scenes.  Particles of scenes not stepped take no key, so
    // the key grouping holds the stepped particles only (cells[T].x of them).
    const int32_t* pscene;    // [N]
    const MultiScene* mscene; // [S]
    int32_t n_extent;         // launch extent: particles 0 .. n_extent - 1 may be stepped
    int32_t n_active;         // particles stepped by the current launches
    // one-launch iterations (single scene whose iteration grid is resident at
    // once): X_i - X_init of particles with contact partners, each component
    // with the tag of its iteration, (tag << 32) | float bits, double buffered
    unsigned long long* tagged = nullptr;   // [2][3][N]
    int32_t resident_iterate = 0;           // 1: the K iterations run as one launch
};

// Enqueues `count` substeps of K = iterations solver iterations.  s2 (or
// NULL) is the same scene with the wave tables of a second iteration launch
// (bodies of more than 4 waves, when s packs the others into 4-wave
// workgroups); both launches make one Jacobi iteration.
hipError_t enqueue_substeps(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
                            hipStream_t stream);

// Workgroups of the one-launch iteration kernel (64 waves_per_block threads)
// that the GPU holds at once; 0 if it cannot be queried.
int resident_iterate_capacity(int waves_per_block);

// Enqueues `count` launches of the iteration kernel(s) alone (measurement):
// one Jacobi iteration each (all but the first continue from the rotation of
// the one before), or, for a scene whose substep runs its `iterations`
// iterations as one launch, that launch.
hipError_t enqueue_iterations(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
                              hipStream_t stream);

// As enqueue_iterations, launch `k` bound to the events t0[k] (begin of its
// first kernel) and t1[k] (end of its last).
hipError_t enqueue_iterations_timed(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
                                    hipStream_t stream, const hipEvent_t* t0, const hipEvent_t* t1);

// Writes the canonical (key, id) order of the last substep into `sorted`.
hipError_t enqueue_canonical_order(const Scene& s, hipStream_t stream);

// Clears the latched counters.
hipError_t enqueue_clear_counters(const Scene& s, hipStream_t stream);

// Zeroes the per-key counts and writes the end sentinel cells[T] (once, at creation).
hipError_t enqueue_init_tables(const Scene& s, hipStream_t stream);

}  // namespace pbdr
