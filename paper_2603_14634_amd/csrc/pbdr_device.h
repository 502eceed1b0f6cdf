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
// Shape matching's sums over a body of many particles lose precision in FP32
// (ten rounding levels over about 1000 terms of one sign): a body of more
// than kWideBodyWaves waves (64 particles each) accumulates them in FP64.
// Bodies of up to 512 particles keep FP32 sums, which meet the per-substep
// tolerance in every mode.
constexpr int kWideBodyWaves = 8;
constexpr int kRadixBits = 8;                   // key sort: digit width
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kMaxRadixPasses = 4;               // keys of up to 32 bits
// A sort tile is kBlock threads of `items` keys each: 16 from kRadixLargeFrom
// keys on (longer runs of one digit per tile, so longer runs of writes), 4
// below (more tiles to fill the GPU).
constexpr size_t kRadixLargeFrom = size_t(1) << 20;
inline uint32_t radix_items_for(size_t n) { return n >= kRadixLargeFrom ? 16u : 4u; }
// The digit histogram takes 16 keys per thread, in workgroups of 1024 threads
// from kRadixLargeFrom keys on (fewer workgroups adding to the counts), 256
// below (more workgroups for a small sort); a workgroup's keys are whole tiles.
inline int radix_hist_threads_for(size_t n) { return n >= kRadixLargeFrom ? 1024 : 256; }
inline size_t radix_tiles_for(size_t n)
{
    const size_t t = (size_t)kBlock * radix_items_for(n);
    return (n + t - 1) / t;
}
// the most tiles of any key count up to n
inline size_t radix_tiles_capacity(size_t n)
{
    const size_t a = radix_tiles_for(n), b = radix_tiles_for(n < kRadixLargeFrom ? n : kRadixLargeFrom - 1);
    return a > b ? a : b;
}

// kErrInternal: an internal consistency check failed (a sort position out of
// range, a pool scene that does not fit its launch shape);
// kErrWait: a one-launch iteration's wait for a contact partner gave up.
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
    // contact geometry in FP64 (penetration depths are differences of
    // centimetre-sized lengths, formed before any rounding to FP32)
    double radius_d, two_r_d;
    double plane_d_d[kMaxPlanes];
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
    uint32_t T;               // keys in use: 2^k (one scene), or the key arena's high water
                              //     (multi-scene mode; T is also the key of particles not stepped)
    int32_t n_sort;           // particles taking part in the key sort (0 .. n_sort - 1)
    int32_t radix_passes;     // ceil(key bits / 8)
    uint32_t radix_items;     // keys per thread of a sort tile: radix_items_for(n_sort)
    uint32_t n_radix_tiles;   // radix_tiles_for(n_sort)
    float* x;                 // [3][N] committed positions: the state after the last clean frame
    float* v;                 // [3][N] committed velocities
    float* x0;                // [3][N] X_init of the current substep (the working state)
    const float* mass;        // [N]
    const int32_t* body;      // [N] body of each particle
    const float* q;           // [3][N] rest offsets
    const int32_t* body_start;// [B+1]
    const float* body_mass;   // [B]
    const double* body_mass64;// [B] the same in FP64 (sum of the FP32 particle masses)
    const int32_t* wave_body; // [n_iter_blocks * waves_per_block] body of each wave, -1 = idle
    const int32_t* body_wave0;// [B] first (global) wave of each body
    const int32_t* block_body;// [2 * n_iter_blocks] first body and body count of each workgroup
    const float* body_mq;     // [B][3] sum of m q over the body (rest frame, ~0)
    int32_t waves_per_block;  // W: iteration workgroup = 64 W threads
    int32_t n_iter_blocks;
    int32_t dense_iterate;    // 1: the iteration grid oversubscribes the GPU (80-VGPR kernel)
    int32_t n_chunked = 0;    // 80-VGPR kernel: its first n_chunked workgroups (4 waves) take one body
                              //     of more than 4 waves each (block_body holds (body, 1) for them)
    int32_t wide_bodies;      // 1: some body of the iteration launch spans more than kWideBodyWaves waves
    float* dl[2];             // [3][N] X_i - X_init, double buffered
    float* vel[2];            // [3][N] V_i, double buffered
    float* xt;                // [3][N] FP32 predicted positions
    float4* sxt4;             // [N] predicted position and body id (bits) in (key, id) order
    uint32_t* key;            // [N] cell key of each particle (by id)
    uint32_t* kbuf[2];        // [N] keys between sort passes (ping-pong)
    uint32_t* ibuf[2];        // [N] ids between sort passes (ping-pong)
    const uint32_t* skey;     // keys in (key, id) order: kbuf[(radix_passes - 1) & 1]
    const uint32_t* sorted;   // ids in (key, id) order: ibuf[(radix_passes - 1) & 1]
    uint32_t* nbr_n;          // [N] neighbour-list length
    uint32_t* nbr;            // [cap][N] neighbour ids, slot-major, ascending
    uint32_t* hist;           // [kMaxRadixPasses][kRadixBins] digit counts of the substep's keys
    uint32_t* tile_off;       // [kRadixBins][n_radix_tiles] sort pass: a tile's count of each
                              //     digit, then the digit's first output position in the tile
    uint4* cells;             // [T] per key, written for occupied keys only: first sorted slot,
                              //     end slot, body signature (the one body of all its particles,
                              //     or -2 mixed), and the substep (epoch) that wrote it; an entry
                              //     of an earlier substep marks an empty key

    float* body_rot;          // [B][9] last rotation of shape matching
    Counters* counters;
    NbrStats* nbr_stats;      // [ceil(N / kBlock)]
    const float* accel;       // [3][N] external acceleration or nullptr
    // multi-scene mode (nullptr otherwise): scene slot of each particle (-1:
    // none) and the scenes.  Particles of scenes not stepped take key T, so the
    // sorted order holds the stepped particles first (n_active of them).
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

// Enqueues `count` substeps of K = iterations solver iterations.
hipError_t enqueue_substeps(const Scene& s, const StepConsts& c, int iterations, int count, hipStream_t stream);

// Workgroups of the one-launch iteration kernel (64 waves_per_block threads)
// that the GPU holds at once; 0 if it cannot be queried.
int resident_iterate_capacity(int waves_per_block);

// Enqueues `count` launches of the iteration kernel(s) alone (measurement):
// one Jacobi iteration each (all but the first continue from the rotation of
// the one before), or, for a scene whose substep runs its `iterations`
// iterations as one launch, that launch.
hipError_t enqueue_iterations(const Scene& s, const StepConsts& c, int iterations, int count, hipStream_t stream);

// As enqueue_iterations, launch `k` bound to the events t0[k] (begin) and
// t1[k] (end).
hipError_t enqueue_iterations_timed(const Scene& s, const StepConsts& c, int iterations, int count,
                                    hipStream_t stream, const hipEvent_t* t0, const hipEvent_t* t1);

// Zeroes `bytes` (a multiple of 4) at `p` with a fill kernel (no memset node
// when the caller captures the stream).
hipError_t enqueue_zero(void* p, size_t bytes, hipStream_t stream);

// Clears the latched counters.
hipError_t enqueue_clear_counters(const Scene& s, hipStream_t stream);

// Clears the key table, the digit counts and the substep epoch (once, at
// creation; `cells` holds `table` entries).
hipError_t enqueue_init_tables(const Scene& s, size_t table, hipStream_t stream);

}  // namespace pbdr
