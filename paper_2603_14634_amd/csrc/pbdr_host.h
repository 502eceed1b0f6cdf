// Host-side helpers shared by the C-ABI sources of libpbdr (scenes and scene
// pools): error reporting and parameter resolution.  Not part of the public
// interface.
#pragma once
#include <stdint.h>

#include "pbdr.h"

namespace pbdr {
namespace host {

constexpr uint32_t kKnownFlags = PBDR_FLAG_STD_VELOCITY | PBDR_FLAG_NO_LIN_MOM | PBDR_FLAG_NO_ANG_MOM |
                                 PBDR_FLAG_NO_GRAPH | PBDR_PP_AVG_MASK;
constexpr int32_t kMaxParticles = 1 << 28;
constexpr int kMinHashBits = 6, kMaxHashBits = 28;

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
// Validates params for a scene of n particles and resolves the defaults.
pbdr_status resolve(const pbdr_params* in, int32_t n, Resolved* out);

}  // namespace host
}  // namespace pbdr

#define HIP_TRY(expr)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) return pbdr::host::fail(PBDR_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
