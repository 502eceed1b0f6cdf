// Internal device-side layout of scene pools (many independent small scenes
// stepped together, one workgroup per scene).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbdr_device.h"

namespace pbdr {

constexpr int kPoolClasses = 7;            // register-resident size classes: n <= 128 << c
constexpr int kPoolMaxParticles = 8192;    // 128 << (kPoolClasses - 1)
constexpr int kPoolMaxBodies = 64;         // bodies of a register-resident scene
constexpr int kPoolBigClass = kPoolClasses;   // launch class of the large scenes
constexpr int kPoolBigMaxParticles = 65535;   // scene-local ids fit 16 bits
constexpr int kPoolBigMaxBodies = 256;
constexpr int kPoolBigMaxSlots = kPoolBigMaxParticles / 64 + 1 + kPoolBigMaxBodies;
constexpr int kPoolBigKeyBits = 13;
constexpr int kPoolMaxWaves = 16;          // waves per workgroup
constexpr int kPoolBodyFloats = 48;        // per-body LDS record
constexpr int kPoolMaxSlots = 128;         // 64-lane slots per scene (bodies wave-aligned) = 16 waves x 8

inline int pool_class_bound(int cls) { return 128 << cls; }
// key bits of a class's workgroup-local hash table (about one key per particle)
inline int pool_class_key_bits(int cls) { return cls + 7 < 8 ? 8 : (cls + 7 > 13 ? 13 : cls + 7); }

// One pooled scene (indexed by slot), written by the host when it is added.
struct PoolScene {
    int32_t p0, n;      // first particle in the particle arena, particle count
    int32_t b0, nb;     // first body in the body arena, body count
    int32_t s_base;     // large scenes: first slot of its range in the slot-sum arena
    int32_t pad[3];
    float g[3];         // gravity
    float mu;           // friction coefficient
};

// Device-side conditions of a pooled scene, latched until the host clears them.
struct PoolStat {
    uint32_t err;       // kErr* bits
    uint32_t max_nbr;   // largest neighbour-list length seen
};

struct PoolDev {
    int32_t P;                 // particle capacity = component stride of [3][P] arrays
    float* x;                  // [3][P] committed positions (after the last clean frame)
    float* v;                  // [3][P] committed velocities
    float* x0;                 // [3][P] X_init of the running substep (read by contact partners)
    const float* mass;         // [P]
    const float* q;            // [3][P] rest offsets
    const uint16_t* pbody;     // [P] scene-local body of each particle
    float* dl;                 // [3][P] X_i - X_init of the running iteration
    float* xt;                 // [3][P] FP32 predicted positions of the last substep
    float4* sxt4;              // [P] predicted position and body (bits), grouped by key per scene
    uint32_t* nbr_n;           // [P] neighbour-list lengths
    uint32_t* nbr;             // per scene: [cap][n] at cap * p0, scene-local ids, ascending
    const int32_t* body_first; // [Bc] first particle of each body (scene-local)
    const float* body_mass;    // [Bc]
    const float* body_mq;      // [Bc][3] sum of m q over the body
    float* part;               // large scenes: [slot arena][24] slot sums and boxes
    uint32_t* sid;             // large scenes: [P] key-grouped (id | body << 16)
    uint32_t* rank;            // large scenes: [P] slot within the key
    float* vel;                // large scenes: [3][P] V_i while a substep runs
    float* cd;                 // large scenes: [3][P] contact displacement of the iteration
    const PoolScene* scenes;   // [S]
    PoolStat* stats;           // [S]
    const int2* order;         // per launch: (slot, frames or substeps), grouped by size class
};

// FP32 constants shared by every scene of a pool.
struct PoolConsts {
    float h, inv_h;
    float radius, two_r;
    float search_r2;           // fl32(R_s^2)
    float search_r;            // R_s
    float box_margin;          // 2 R_s: growth of the body boxes in the broad phase
    float inv_cell;            // fl32(1 / a)
    float origin[3];
    int32_t nbr_cap;
    uint32_t flags;
    int32_t n_planes;
    float plane_n[kMaxPlanes][3];
    float plane_d[kMaxPlanes];
    int32_t iterations;
    double radius_d, two_r_d;            // contact geometry in FP64
    double plane_d_d[kMaxPlanes];
};

// Dynamic LDS bytes of the pool kernel for a size class (or kPoolBigClass).
size_t pool_lds_bytes(int cls);

// Allows every pool kernel variant up to max_lds bytes of dynamic LDS.
hipError_t pool_prepare(size_t max_lds);

// Particle slots per lane with a kernel variant: 1-6 and 8.
inline bool pool_slots_supported(int s) { return (s >= 1 && s <= 6) || s == 8; }

// Launches the pool kernel over `count` scenes of class `cls` listed at
// order[first ..]: each listed (slot, units) advances units * subs_per_unit substeps.
// `waves` (1, 2, 4, 8 or 16) and `slots` (register sets per lane, see
// pool_slots_supported) must satisfy waves * slots >= the largest slot count
// (sum over bodies of ceil(n_b / 64)) of the listed scenes.
hipError_t enqueue_pool_class(const PoolDev& d, const PoolConsts& c, int cls, int waves, int slots, int first,
                              int count, int subs_per_unit, hipStream_t stream);

}  // namespace pbdr
