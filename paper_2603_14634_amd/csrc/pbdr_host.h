// Host-side helpers shared by the C-ABI sources of libpbdr (scenes and scene
// pools): error reporting and parameter resolution.  Not part of the public
// interface.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

#include "pbdr.h"

namespace pbdr {
struct StepConsts;
namespace host {

constexpr uint32_t kKnownFlags = PBDR_FLAG_STD_VELOCITY | PBDR_FLAG_NO_LIN_MOM | PBDR_FLAG_NO_ANG_MOM |
                                 PBDR_FLAG_NO_GRAPH | PBDR_FLAG_ITERATION_LAUNCHES | PBDR_PP_AVG_MASK;
constexpr int32_t kMaxParticles = 1 << 28;
constexpr int kMinHashBits = 6, kMaxHashBits = 28;

// First-fit allocator of integer ranges [start, start + len) (arena admission).
class RangeAlloc {
public:
    void init(int32_t capacity)
    {
        free_.clear();
        if (capacity > 0) free_[0] = capacity;
    }
    int32_t alloc(int32_t len)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const int32_t start = it->first, rest = it->second - len;
            free_.erase(it);
            if (rest > 0) free_[start + len] = rest;
            return start;
        }
        return -1;
    }
    void release(int32_t start, int32_t len)
    {
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                prev->second += len;
                return;
            }
        }
        free_[start] = len;
    }
    // end of the highest range in use (0 if none) for an allocator of `capacity`
    int32_t high_water(int32_t capacity) const
    {
        if (free_.empty()) return capacity;
        const auto last = std::prev(free_.end());
        return last->first + last->second == capacity ? last->first : capacity;
    }
    int32_t largest() const
    {
        int32_t m = 0;
        for (const auto& e : free_) m = std::max(m, e.second);
        return m;
    }

private:
    std::map<int32_t, int32_t> free_;
};

// Parameters with defaults filled in.
struct Resolved {
    pbdr_params p;
    double h, rs, a;   // substep, search radius, cell edge
    int k, cap;        // key bits, neighbour-list capacity
};

// Records a printf-style message for pbdr_last_error() and returns st.
pbdr_status fail(pbdr_status st, const char* fmt, ...);
void clear_error();
bool finite3(const double* v);
// Status for latched device error bits (pbdr::kErr*): PBDR_OK if none; a list
// over capacity before a non-finite state before a wait that gave up.
pbdr_status latched_status(uint32_t err, uint32_t max_nbr, int cap);
// Validates params for a scene of n particles and resolves the defaults.
pbdr_status resolve(const pbdr_params* in, int32_t n, Resolved* out);
// FP32 constants of one substep from resolved parameters.
void fill_step_consts(const Resolved& r, StepConsts* out);
// pbdr_scene_create into `dev_workspace`, filling `record` (one of the reused
// host records, or NULL for a new one).  A scene in a reused record steps by
// direct launches only (no graph capture, which allocates), and
// pbdr_scene_destroy releases the record without freeing it.
pbdr_status create_scene_in(const pbdr_params* params, const pbdr_scene_desc* desc, void* dev_workspace,
                            size_t ws_bytes, void* hip_stream, pbdr_scene* record, pbdr_scene** out);
// Reused host record `index` (0 .. 63), or NULL.
pbdr_scene* fixed_scene_record(int index);
// Waits for the work of the scene in a reused record, if it holds one, and
// releases the record.
void release_fixed_record(pbdr_scene* record);

}  // namespace host
}  // namespace pbdr

#define HIP_TRY(expr)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) return pbdr::host::fail(PBDR_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
