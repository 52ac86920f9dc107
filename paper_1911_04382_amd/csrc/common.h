// Internal declarations of the GRASS gfx950 library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/grass.h"

namespace grass {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    grass_status code;
    Error(grass_status c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

#define GR_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            throw ::grass::Error(GRASS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GR_CHECK_LAUNCH() GR_HIP(hipGetLastError())

inline void require(bool ok, grass_status code, const std::string &msg) {
    if (!ok) throw Error(code, msg);
}

// ------------------------------------------------------------- workspace
// Bump allocator over caller-provided device memory. `dry` mode only counts
// bytes (used by grass_workspace_bytes), so the plan and the footprint can
// never disagree.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    bool dry = false;
    template <typename X>
    X *take(size_t count) {
        size_t bytes = ((count * sizeof(X)) + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        size_t at = off;
        off += bytes;
        if (dry) return nullptr;
        if (off > cap)
            throw Error(GRASS_ERR_OOM, "workspace too small: need more than " + std::to_string(cap) + " bytes");
        return reinterpret_cast<X *>(base + at);
    }
};

// ------------------------------------------------------ device helpers
// Cross-workgroup communication uses agent-scope relaxed atomics (coherent
// across the XCDs' L2 caches) plus explicit waits for ordering.
__device__ __forceinline__ int ld_acq_i32(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_agent_u32(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u32(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent_i32(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_i32(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until every outstanding memory operation of this wave has completed
__device__ __forceinline__ unsigned long long ld_agent_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

// order-preserving bit images of non-negative floating point values
__device__ __forceinline__ unsigned fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ unsigned long long fbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// Spin limit of every bounded wait (a guard: a correct run never reaches it).
constexpr long long kSpinLimit = 1ll << 28;

// device error flag bits
enum : unsigned {
    DEVERR_SPIN = 1u,      // a bounded wait expired
    DEVERR_NONFINITE = 2u, // NaN/Inf met in a vector
    DEVERR_TREE = 4u,      // tree edges do not span the graph
};

inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }
inline int kpad(int k) {
    int p = 1;
    while (p < k) p <<= 1;
    return p;
}

// ------------------------------------------------------------- primitives
// (prim.hip) integer scans, stream compaction, stable LSD radix sort.
struct ScanTmp {
    int *bsum = nullptr;
    int nblk_cap = 0;
};
void plan_scan(Arena &a, long long n, ScanTmp &t);
// out[i] = sum_{j<i} in[j] (exclusive); *total (device, optional) = sum of all.
void scan_excl_i32(const int *in, int *out, long long n, int *total, const ScanTmp &t, hipStream_t s);
// inclusive variant
void scan_incl_i32(const int *in, int *out, long long n, const ScanTmp &t, hipStream_t s);

struct SortTmp {
    unsigned long long *k2 = nullptr;
    int *v2 = nullptr;
    int *hist = nullptr;
    ScanTmp scan;
    long long cap = 0;
    int nblk = 0;
};
void plan_sort(Arena &a, long long n, SortTmp &t);
// Stable ascending sort of (key, value) pairs by bits [0, key_bits) of key, in
// place (keys/vals hold the result when the call returns).
void radix_sort_pairs(unsigned long long *keys, int *vals, long long n, int key_bits, const SortTmp &t,
                      hipStream_t s);

// fill helpers
void fill_i32(int *p, long long n, int v, hipStream_t s);
void fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s);
void fill_u32(unsigned *p, long long n, unsigned v, hipStream_t s);
void fill_f64(double *p, long long n, double v, hipStream_t s);
void fill_f32(float *p, long long n, float v, hipStream_t s);
inline void fill_T(float *p, long long n, float v, hipStream_t s) { fill_f32(p, n, v, s); }
inline void fill_T(double *p, long long n, double v, hipStream_t s) { fill_f64(p, n, v, s); }
// synchronous read of one device int (stream-ordered)
int read_i32(const int *p, hipStream_t s);

}  // namespace grass
