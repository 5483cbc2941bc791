// Internal declarations shared by the translation units of libneuphys.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "neuphys.h"

namespace np {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

// ---------------------------------------------------- learned correction
// Attached network (cnn.hip): log2 of its grid per axis (-1 when none), and
// its prediction xc = rms * N(fc / rms) on a coarse level of that size.
int cnn_attached_lg();
np_status cnn_coarse_guess(int lg, const double *fc, double *xc, hipStream_t s, bool *used);

#define NP_HIP_TRY(expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::np::set_error("%s:%d: %s -> %s", __FILE__, __LINE__, #expr,                  \
                            hipGetErrorString(e_));                                        \
            return NP_EHIP;                                                                \
        }                                                                                  \
    } while (0)

#define NP_TRY(expr)                                                                       \
    do {                                                                                   \
        np_status s_ = (expr);                                                             \
        if (s_ != NP_OK) return s_;                                                        \
    } while (0)

// Checks the launch that was just enqueued.
#define NP_LAUNCH_CHECK() NP_HIP_TRY(hipGetLastError())

// --------------------------------------------------------- storage types
// BF16 is kept as raw 16-bit patterns.  float -> bf16 rounds to nearest, ties
// to even, NaN stays NaN: gfx950's packed conversion (v_cvt_pk_bf16_f32), one
// instruction for two values.  It matches the integer rounding
// u + 0x7fff + (bit 16 of u), then the high half, bit for bit on every
// non-NaN float (all 2^32 inputs compared on the device).
struct bf16 {
    uint16_t u;
};

typedef __bf16 np_bf16x2 __attribute__((ext_vector_type(2)));
typedef float np_f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_to_float(uint16_t u) { return __uint_as_float(uint32_t(u) << 16); }

// a in the low half, b in the high half
__device__ __forceinline__ uint32_t float2_to_bf16x2(float a, float b) {
    const np_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, np_bf16x2));
}

__device__ __forceinline__ uint16_t float_to_bf16(float f) { return uint16_t(float2_to_bf16x2(f, 0.0f)); }

// Storage traits: C is the arithmetic type for fields stored as S.
template <class S> struct St;
template <> struct St<double> {
    typedef double C;
    static __device__ __forceinline__ double ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, double v) { *p = v; }
};
template <> struct St<float> {
    typedef float C;
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
};
template <> struct St<bf16> {
    typedef float C;
    static __device__ __forceinline__ float ld(const bf16 *p) { return bf16_to_float(p->u); }
    static __device__ __forceinline__ void st(bf16 *p, float v) { p->u = float_to_bf16(v); }
};

// Explicit fused multiply-add (one rounding): kernels that must round alike
// (a fused kernel and the pair it replaces) spell their products this way, so
// that the compiler's contraction choices cannot differ between them.
__device__ __forceinline__ float np_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double np_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Round trip of a value through storage S (BF16: nearest even; identity otherwise).
template <class S>
__device__ __forceinline__ typename St<S>::C st_round(typename St<S>::C v) {
    S t;
    St<S>::st(&t, v);
    return St<S>::ld(&t);
}

inline size_t prec_bytes(np_prec p) { return p == NP_FP64 ? 8 : (p == NP_FP32 ? 4 : 2); }

// ------------------------------------------------------------ reductions
constexpr int kRedBlocks = 1024;  // fixed partial count: deterministic reduction order
constexpr int kBlock = 256;

// Sum over a 64-wide wavefront (xor butterfly), then over the NT / 64 waves of
// the block (blockDim.x == NT) through LDS; the result is valid in thread 0.
// Fixed order: deterministic.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v) {
    __shared__ double wsum[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += wsum[i];
    __syncthreads();
    return s;
}
__device__ __forceinline__ double block_sum(double v) { return block_sum_n<kBlock>(v); }

// XCD-aware workgroup order.  The dispatcher hands workgroup i to XCD i mod 8;
// remapping ids so that XCD x runs the contiguous range [x G/8, (x+1) G/8)
// keeps neighbouring rows and planes of a stencil in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned g) {
    return (g & 7u) == 0u ? (b & 7u) * (g >> 3) + (b >> 3) : b;
}

// -------------------------------------------------------------- profiling
// Event bracketing of finest-level launches (np_prof_*).  prof_on() returns
// the mask of kernel kinds being timed.
enum ProfKind {
    kProfDown = 1,      // smoothing + residual + restriction (iterate read)
    kProfDownZero = 2,  // the same from a zero iterate
    kProfUp = 4,        // prolongation + correction + smoothing
    kProfJacobi = 8,    // single Jacobi sweep
    kProfRestrict = 16, // residual + restriction
    kProfProlong = 32,  // prolongation + correction
    kProfRefine = 64,   // FP64 update + residual of the mixed-precision refinement
    kProfSweepZero = 128,  // Jacobi sweep from a zero iterate
};
int prof_on();
np_status prof_begin(hipStream_t s, void **tok);
np_status prof_end(hipStream_t s, void *tok, double bytes);

// ----------------------------------------------------------------- helpers
inline bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }
inline int ilog2(int64_t n) {
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}
inline unsigned blocks_for(int64_t m, int per = kBlock) { return unsigned((m + per - 1) / per); }

// Validates a grid for the multigrid entry points; returns log2(n) or -1.
int check_grid(const np_dims &dims);

// Workspace cache lifetime.
void release_mg_cache();
void release_ns_cache();
void release_batched_cache();
extern int g_batched_graphs;
extern int g_batched_autotune;
extern int g_batched_rm;
extern int g_batched_wg;
extern int g_zmarch_explicit;
extern int g_mom_rows;
extern int g_mom_ring;
extern int g_conv3z;
extern int g_wgrad_mfma;
extern int g_zc3;  // planes per workgroup of the 3D z-marching solver kernels (0: automatic)

}  // namespace np
