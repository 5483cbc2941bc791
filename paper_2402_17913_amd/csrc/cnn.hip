// Learned warm start: a small periodic 3D U-Net (16 channels, BF16 storage,
// FP32 accumulation) with its own forward, backward and Adam kernels.
//
// Activations are channels-last BF16 tensors [z][y][x][16].  A 3x3x3
// convolution is an implicit GEMM per 16-voxel row segment: output channel
// (M = 16) x voxel (N = 16) x (tap, input channel) (K = 27 x 16, two taps
// per 16x16x32 MFMA step, 14 steps).  The workgroup stages its input halo
// tile (x: row + 2, y: 4 rows + 2, z: 3 planes) and the weights in LDS.
// The data gradient is the same kernel on the flipped, transposed filter; the
// weight gradient is an FP32 reduction over voxels.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "mg_kernels.h"
#include "np_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace np {
namespace {

constexpr int kC = 16;                 // channels
constexpr int kTaps = 27;
constexpr int kWsz = kTaps * kC * kC;  // weights per conv ([tap][out][in])
constexpr int kPsz = kWsz + kC;        // + bias
constexpr int kWgBlocks = 768;         // workgroups of a weight-gradient reduction (three per CU)
}  // namespace
int g_wgrad_mfma = 1;  // tuning knob "wgrad_mfma": weight gradients on the matrix cores
int g_conv3z = 1;  // tuning knob "conv3z": z-marching convolution tiles (0 off, 1 automatic, else planes)
namespace {

__device__ __forceinline__ float b2f(uint16_t u) { return __uint_as_float(uint32_t(u) << 16); }
__device__ __forceinline__ uint16_t f2b(float f) { return float_to_bf16(f); }

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------------ conv
// Y = conv(X, W) (+ bias, ReLU) on an n^3 periodic grid, n = 2^lg >= 16.
// Workgroup: TXV = min(64, n) voxels along x, 4 rows along y, one plane.
template <bool RELU, bool OUT32>
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ X, const uint16_t *__restrict__ W,
                                              const float *__restrict__ bias, void *__restrict__ Y, int lg) {
    __shared__ uint4 xs[(64 + 2) * 6 * 3 * 2];  // halo voxels x 32 B
    __shared__ uint4 ws[kTaps * kC * 2];         // 27 x 16 rows x 32 B
    const int n = 1 << lg, txv = n < 64 ? n : 64, hx = txv + 2;
    const int tiles_x = n / txv;
    const int b = blockIdx.x;
    const int tx = b % tiles_x, y4 = (b / tiles_x) % (n / 4), z = b / (tiles_x * (n / 4));
    const int x0 = tx * txv, y0 = 4 * y4, tid = threadIdx.x;
    const uint4 *W4 = reinterpret_cast<const uint4 *>(W);
    for (int q = tid; q < kTaps * kC * 2; q += 256) ws[q] = W4[q];
    const int nh = hx * 6 * 3;
    const uint4 *X4 = reinterpret_cast<const uint4 *>(X);
    for (int q = tid; q < nh * 2; q += 256) {
        const int v = q >> 1, half = q & 1;
        const int lx = v % hx, ly = (v / hx) % 6, lz = v / (hx * 6);
        const int gx = wrapi(x0 + lx - 1, n), gy = wrapi(y0 + ly - 1, n), gz = wrapi(z + lz - 1, n);
        xs[q] = X4[((((int64_t(gz) << lg) + gy) << lg) + gx) * 2 + half];
    }
    __syncthreads();
    const int w = tid >> 6, l = tid & 63;
    const int col = l & 15, grp = l >> 4;
    const int tsel = grp >> 1, cb = grp & 1;
    for (int tt = 0; tt < txv / 16; ++tt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 14; ++s) {
            const int tap = 2 * s + tsel;
            bf16x8 av, bv;
            if (tap < kTaps) {
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const uint4 a4 = ws[(tap * kC + col) * 2 + cb];
                const int hv = ((1 + dz) * 6 + (w + 1 + dy)) * hx + (tt * 16 + col + 1 + dx);
                const uint4 b4 = xs[hv * 2 + cb];
                av = *reinterpret_cast<const bf16x8 *>(&a4);
                bv = *reinterpret_cast<const bf16x8 *>(&b4);
            } else {
                const uint4 zz = make_uint4(0, 0, 0, 0);
                av = *reinterpret_cast<const bf16x8 *>(&zz);
                bv = av;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
        // lane holds output channels 4*grp .. +3 of voxel `col`
        const int gx = x0 + tt * 16 + col, gy = y0 + w;
        const int64_t v = (((int64_t(z) << lg) + gy) << lg) + gx;
        float o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float t = acc[r] + (bias ? bias[4 * grp + r] : 0.f);
            if (RELU) t = t > 0.f ? t : 0.f;
            o[r] = t;
        }
        if (OUT32) {
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(Y) + v * kC + 4 * grp) = make_float4(o[0], o[1], o[2], o[3]);
        } else {
            uint2 pk;
            pk.x = float2_to_bf16x2(o[0], o[1]);
            pk.y = float2_to_bf16x2(o[2], o[3]);
            *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(Y) + v * kC + 4 * grp) = pk;
        }
    }
}

// Z-marching form of the same convolution (same MFMA sequence per output, so
// the same bits): a workgroup of 256 threads (4 waves, one row each) owns a
// TXV x 4 tile of the plane (TXV = min(64, n)) and zc consecutive planes.
// Input planes z - 1, z, z + 1 with their one-voxel halo sit in a ring of
// three LDS buffers, the weights are staged once per workgroup, and plane
// z + 2 replaces plane z - 1 after plane z is computed, so each input plane is
// read about once per workgroup instead of three times.
constexpr int kCzT = 256, kCzY = 4;
constexpr int kCzSlots = (64 + 2) * (kCzY + 2) * 2;  // uint4 per plane buffer (halo tile, two per voxel)

// This thread's share of an input plane of k_conv3z, loaded straight into
// its ring buffer: slot q holds half (q & 1) of voxel (q >> 1) of the halo tile.
__device__ __forceinline__ void cz_fill(uint4 *__restrict__ dst, const uint4 *__restrict__ X4, int64_t base, int tid,
                                        int hx, int x0, int y0, int lg) {
    const int n = 1 << lg, nslot = hx * (kCzY + 2) * 2;
    for (int q = tid; q < nslot; q += kCzT) {
        const int v = q >> 1, half = q & 1, lx = v % hx, ly = v / hx;
        dst[q] = X4[base + ((int64_t(wrapi(y0 + ly - 1, n)) << lg) + wrapi(x0 + lx - 1, n)) * 2 + half];
    }
}

template <bool RELU, bool OUT32>
__global__ __launch_bounds__(kCzT) void k_conv3z(const uint16_t *__restrict__ X, const uint16_t *__restrict__ W,
                                                 const float *__restrict__ bias, void *__restrict__ Y, int lg, int zc) {
    __shared__ uint4 xs[3][kCzSlots];
    const int n = 1 << lg, txv = n < 64 ? n : 64, hx = txv + 2;
    const int tiles_x = n / txv, tiles_y = n / kCzY;
    const int b = blockIdx.x;
    const int x0 = (b % tiles_x) * txv, y0 = ((b / tiles_x) % tiles_y) * kCzY, z0 = (b / (tiles_x * tiles_y)) * zc;
    const int tid = threadIdx.x;
    const uint4 *W4 = reinterpret_cast<const uint4 *>(W);
    const uint4 *X4 = reinterpret_cast<const uint4 *>(X);
    auto plane = [&](int z) { return int64_t(wrapi(z, n)) << (2 * lg + 1); };
    cz_fill(xs[(z0 + 2) % 3], X4, plane(z0 - 1), tid, hx, x0, y0, lg);
    cz_fill(xs[z0 % 3], X4, plane(z0), tid, hx, x0, y0, lg);
    cz_fill(xs[(z0 + 1) % 3], X4, plane(z0 + 1), tid, hx, x0, y0, lg);
    const int w = tid >> 6, l = tid & 63;
    const int col = l & 15, grp = l >> 4;
    const int tsel = grp >> 1, cb = grp & 1;
    // the lane's weight operands of the 14 steps depend on the lane only: held in registers
    // (the 28th tap does not exist: its operands are zero)
    bf16x8 wa[14];
#pragma unroll
    for (int s = 0; s < 14; ++s) {
        const bool live = 2 * s + tsel < kTaps;
        const uint4 a4 = W4[((live ? 2 * s + tsel : kTaps - 1) * kC + col) * 2 + cb];
        wa[s] = __builtin_bit_cast(bf16x8, live ? a4 : make_uint4(0, 0, 0, 0));
    }
    for (int z = z0; z < z0 + zc; ++z) {
        __syncthreads();  // planes z - 1, z, z + 1 are in LDS
        for (int tt = 0; tt < txv / 16; ++tt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 14; ++s) {
                // the 28th tap does not exist: read tap 26's operand and zero it by value
                const bool live = 2 * s + tsel < kTaps;
                const int tap = live ? 2 * s + tsel : kTaps - 1;
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const int hv = (w + 1 + dy) * hx + (tt * 16 + col + 1 + dx);
                const uint4 b4 = xs[(z + dz + 3) % 3][hv * 2 + cb];
                const uint4 zz = make_uint4(0, 0, 0, 0);
                const bf16x8 av = wa[s];
                const bf16x8 bv = __builtin_bit_cast(bf16x8, live ? b4 : zz);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
            }
            // lane holds output channels 4*grp .. +3 of voxel `col`
            const int gx = x0 + tt * 16 + col, gy = y0 + w;
            const int64_t v = (((int64_t(z) << lg) + gy) << lg) + gx;
            float o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float t = acc[r] + (bias ? bias[4 * grp + r] : 0.f);
                if (RELU) t = t > 0.f ? t : 0.f;
                o[r] = t;
            }
            if (OUT32) {
                *reinterpret_cast<float4 *>(reinterpret_cast<float *>(Y) + v * kC + 4 * grp) =
                    make_float4(o[0], o[1], o[2], o[3]);
            } else {
                uint2 pk;
                pk.x = float2_to_bf16x2(o[0], o[1]);
                pk.y = float2_to_bf16x2(o[2], o[3]);
                *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(Y) + v * kC + 4 * grp) = pk;
            }
        }
        __syncthreads();  // every read of the oldest buffer is done before it takes plane z + 2
        if (z + 2 <= z0 + zc) cz_fill(xs[(z + 2) % 3], X4, plane(z + 2), tid, hx, x0, y0, lg);
    }
}

// Weight gradient partials: P[blk][tap*256 + o*16 + c] = sum over the
// workgroup's voxels of dZ[v][o] * X[v + tap][c]; P[blk][6912 + o] = sum dZ[v][o].
// Tiles of the forward shape, grid-strided over a capped number of workgroups.
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *__restrict__ X, const uint16_t *__restrict__ dZ,
                                               float *__restrict__ P, int lg) {
    __shared__ uint16_t xs[(64 + 2) * 6 * 3 * kC];
    __shared__ uint16_t zs[64 * 4 * kC];
    const int n = 1 << lg, txv = n < 64 ? n : 64, hx = txv + 2;
    const int tiles_x = n / txv, ntile = tiles_x * (n / 4) * n;
    const int tid = threadIdx.x, o = tid >> 4, c = tid & 15;
    float acc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc[t] = 0.f;
    float bacc = 0.f;
    for (int b = blockIdx.x; b < ntile; b += gridDim.x) {
        const int tx = b % tiles_x, y4 = (b / tiles_x) % (n / 4), z = b / (tiles_x * (n / 4));
        const int x0 = tx * txv, y0 = 4 * y4;
        __syncthreads();
        const int nh = hx * 6 * 3;
        for (int q = tid; q < nh * 2; q += 256) {
            const int v = q >> 1, half = q & 1;
            const int lx = v % hx, ly = (v / hx) % 6, lz = v / (hx * 6);
            const int gx = wrapi(x0 + lx - 1, n), gy = wrapi(y0 + ly - 1, n), gz = wrapi(z + lz - 1, n);
            reinterpret_cast<uint4 *>(xs)[q] =
                reinterpret_cast<const uint4 *>(X)[((((int64_t(gz) << lg) + gy) << lg) + gx) * 2 + half];
        }
        for (int q = tid; q < txv * 4 * 2; q += 256) {
            const int v = q >> 1, half = q & 1;
            const int lx = v % txv, ly = v / txv;
            reinterpret_cast<uint4 *>(zs)[q] =
                reinterpret_cast<const uint4 *>(dZ)[((((int64_t(z) << lg) + y0 + ly) << lg) + x0 + lx) * 2 + half];
        }
        __syncthreads();
        for (int ly = 0; ly < 4; ++ly)
            for (int lx = 0; lx < txv; ++lx) {
                const float g = b2f(zs[(ly * txv + lx) * kC + o]);
                bacc += g;
                if (g == 0.f) continue;
#pragma unroll
                for (int t = 0; t < kTaps; ++t) {
                    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                    const int hv = ((1 + dz) * 6 + (ly + 1 + dy)) * hx + (lx + 1 + dx);
                    acc[t] += g * b2f(xs[hv * kC + c]);
                }
            }
    }
    float *Pb = P + int64_t(blockIdx.x) * kPsz;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) Pb[t * 256 + o * 16 + c] = acc[t];
    if (c == 0) Pb[kWsz + o] = bacc;
}

// The same partials on the matrix cores: per tap t, dW_t[o][c] = sum over
// voxels v of dZ[v][o] X[v + t][c] is a 16 x 16 product with the voxels as the
// contraction (v_mfma_f32_16x16x32_bf16, 32 voxels per step).  Both tiles are
// staged channel-major in LDS, so a lane's operand (8 consecutive voxels of one
// channel) is one 16-byte read for dZ and, for X shifted by the tap's dx, two
// aligned 16-byte reads funnel-shifted by 0, 2 or 4 bytes (rows padded to a
// multiple of 8 voxels).  The three taps of a (dz, dy) group read one X row and
// differ by the shift; wave w owns groups w, w + 4 (and 8 for wave 0), so no
// partial crosses waves; the bias gradient is one more product with X = 1.
constexpr int kWmT = 256;

__device__ __forceinline__ uint32_t wm_shift(uint32_t lo, uint32_t hi, int bytes) {
    return bytes == 0 ? lo : __builtin_amdgcn_alignbyte(hi, lo, bytes);
}

__global__ __launch_bounds__(kWmT) void k_wgrad_mfma(const uint16_t *__restrict__ X, const uint16_t *__restrict__ dZ,
                                                     float *__restrict__ P, int lg) {
    constexpr int HXP = 72;  // padded halo row (txv + 2 <= 66 voxels), a multiple of 8
    __shared__ __align__(16) uint16_t xt[kC * 3 * 6 * HXP];   // [c][plane][row][x]
    __shared__ __align__(16) uint16_t zt[kC * 64 * 4];        // [o][voxel of the tile]
    const int n = 1 << lg, txv = n < 64 ? n : 64, hx = txv + 2;
    const int tiles_x = n / txv, ntile = tiles_x * (n / 4) * n;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ch = l & 15, g = l >> 4;  // operand channel (o for dZ, c for X); voxel run within 32
    f32x4 acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t one = 0x3f80;  // bf16 1.0
    const uint4 ones = make_uint4(one | (uint32_t(one) << 16), one | (uint32_t(one) << 16),
                                  one | (uint32_t(one) << 16), one | (uint32_t(one) << 16));
    const uint4 *X4 = reinterpret_cast<const uint4 *>(X), *Z4 = reinterpret_cast<const uint4 *>(dZ);
    for (int b = blockIdx.x; b < ntile; b += gridDim.x) {
        const int tx = b % tiles_x, y4 = (b / tiles_x) % (n / 4), z = b / (tiles_x * (n / 4));
        const int x0 = tx * txv, y0 = 4 * y4;
        __syncthreads();  // the previous tile's operands are read
        // X halo tile (3 planes x 6 rows x hx voxels), transposed to channel-major
        for (int q = tid; q < hx * 6 * 3 * 2; q += kWmT) {
            const int v = q >> 1, half = q & 1;
            const int lx = v % hx, ly = (v / hx) % 6, lz = v / (hx * 6);
            const uint4 d = X4[((((int64_t(wrapi(z + lz - 1, n)) << lg) + wrapi(y0 + ly - 1, n)) << lg) +
                                wrapi(x0 + lx - 1, n)) * 2 + half];
            const uint32_t dw[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                xt[(((8 * half + e) * 3 + lz) * 6 + ly) * HXP + lx] = uint16_t(dw[e >> 1] >> (16 * (e & 1)));
        }
        // dZ tile (4 rows x txv voxels), transposed
        for (int q = tid; q < txv * 4 * 2; q += kWmT) {
            const int v = q >> 1, half = q & 1;
            const int lx = v % txv, ly = v / txv;
            const uint4 d = Z4[((((int64_t(z) << lg) + y0 + ly) << lg) + x0 + lx) * 2 + half];
            const uint32_t dw[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) zt[(8 * half + e) * 256 + v] = uint16_t(dw[e >> 1] >> (16 * (e & 1)));
        }
        __syncthreads();
        for (int kb = 0; kb < txv * 4 / 32; ++kb) {
            const int v0 = kb * 32 + 8 * g, ly = v0 / txv, lx0 = v0 % txv;  // 8 voxels of one row
            const uint4 a4 = *reinterpret_cast<const uint4 *>(&zt[ch * 256 + v0]);
            const bf16x8 av = __builtin_bit_cast(bf16x8, a4);
#pragma unroll
            for (int jg = 0; jg < 3; ++jg) {
                const int G = w + 4 * jg;  // tap group (dz, dy): its three taps share one X row
                if (G < 9) {
                    const int dz = G / 3 - 1, dy = G % 3 - 1;
                    const uint16_t *row = &xt[((ch * 3 + 1 + dz) * 6 + (ly + 1 + dy)) * HXP + lx0];
                    const uint4 lo = *reinterpret_cast<const uint4 *>(row);
                    const uint4 hi = *reinterpret_cast<const uint4 *>(row + 8);
                    const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
                    for (int s0 = 0; s0 < 3; ++s0) {  // dx = s0 - 1: the run starts s0 voxels in
                        const int wsh = s0 >> 1, bsh = 2 * (s0 & 1);
                        uint4 b4;
                        b4.x = wm_shift(d[wsh + 0], d[wsh + 1], bsh);
                        b4.y = wm_shift(d[wsh + 1], d[wsh + 2], bsh);
                        b4.z = wm_shift(d[wsh + 2], d[wsh + 3], bsh);
                        b4.w = wm_shift(d[wsh + 3], d[wsh + 4], bsh);
                        acc[3 * jg + s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            av, __builtin_bit_cast(bf16x8, b4), acc[3 * jg + s0], 0, 0, 0);
                    }
                } else if (jg == 2 && w == 3) {
                    // wave 3's spare slot: the bias gradient, sum over voxels of dZ[v][o]
                    acc[6] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, ones), acc[6],
                                                                     0, 0, 0);
                }
            }
        }
    }
    // lane holds C[o = 4 g + r][c = ch] of each of its products
    float *Pb = P + int64_t(blockIdx.x) * kPsz;
#pragma unroll
    for (int jg = 0; jg < 3; ++jg) {
        const int G = w + 4 * jg;
#pragma unroll
        for (int s0 = 0; s0 < 3; ++s0)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (G < 9) Pb[(3 * G + s0) * 256 + (4 * g + r) * 16 + ch] = acc[3 * jg + s0][r];
                else if (jg == 2 && w == 3 && s0 == 0 && ch == 0) Pb[kWsz + 4 * g + r] = acc[6][r];
            }
    }
}

// G[i] += sum over workgroups of P[blk][i] (fixed order): a workgroup owns 32
// consecutive entries; its 8 slices of 32 threads sum every eighth partial,
// then the slices are added in order through LDS.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ P, int nblk, float *__restrict__ G) {
    __shared__ float part[8][32];
    const int li = threadIdx.x & 31, sl = threadIdx.x >> 5, i = blockIdx.x * 32 + li;
    float s = 0.f;
    if (i < kPsz)
        for (int b = sl; b < nblk; b += 8) s += P[int64_t(b) * kPsz + i];
    part[sl][li] = s;
    __syncthreads();
    if (sl == 0 && i < kPsz) {
        float t = part[0][li];
#pragma unroll
        for (int q = 1; q < 8; ++q) t += part[q][li];
        G[i] += t;
    }
}

// dZ = round_bf16(dY * (act > 0)) (act null: no mask).
__global__ __launch_bounds__(256) void k_mask(const float *__restrict__ dY, const uint16_t *__restrict__ act,
                                              uint16_t *__restrict__ dZ, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m) return;
    float g = dY[i];
    if (act && !(b2f(act[i]) > 0.f)) g = 0.f;
    dZ[i] = f2b(g);
}

// Flipped, transposed filter for the data gradient: Wt[26 - t][c][o] = W[t][o][c].
__global__ __launch_bounds__(256) void k_wflip(const uint16_t *__restrict__ W, uint16_t *__restrict__ Wt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kWsz) return;
    const int t = i / 256, o = (i / 16) % 16, c = i % 16;
    Wt[(26 - t) * 256 + c * 16 + o] = W[i];
}

// 2x2x2 average (n fine -> n/2), bf16.
__global__ __launch_bounds__(256) void k_pool(const uint16_t *__restrict__ X, uint16_t *__restrict__ Y, int lgc) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int nc = 1 << lgc;
    if (i >= (int64_t(kC) << (3 * lgc))) return;
    const int ch = int(i & 15);
    const int64_t v = i >> 4;
    const int x = int(v & (nc - 1)), y = int((v >> lgc) & (nc - 1)), z = int(v >> (2 * lgc));
    const int lg = lgc + 1;
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += b2f(X[(((((int64_t(2 * z + dz) << lg) + 2 * y + dy) << lg) + 2 * x + dx) << 4) + ch]);
    Y[i] = f2b(s * 0.125f);
}

// dX(fine) += dY(coarse) / 8, FP32.
__global__ __launch_bounds__(256) void k_pool_back(const float *__restrict__ dY, float *__restrict__ dX, int lg) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= (int64_t(kC) << (3 * lg))) return;
    const int ch = int(i & 15);
    const int64_t v = i >> 4;
    const int n = 1 << lg, lgc = lg - 1;
    const int x = int(v & (n - 1)), y = int((v >> lg) & (n - 1)), z = int(v >> (2 * lg));
    dX[i] += dY[(((((int64_t(z >> 1) << lgc) + (y >> 1)) << lgc) + (x >> 1)) << 4) + ch] * 0.125f;
}

// Y(fine) = up(Xc) + S, periodic cell-centred trilinear, bf16.
__global__ __launch_bounds__(256) void k_up_add(const uint16_t *__restrict__ Xc, const uint16_t *__restrict__ S,
                                                uint16_t *__restrict__ Y, int lg) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= (int64_t(kC) << (3 * lg))) return;
    const int ch = int(i & 15);
    const int64_t v = i >> 4;
    const int n = 1 << lg, lgc = lg - 1, nc = n >> 1;
    const int x = int(v & (n - 1)), y = int((v >> lg) & (n - 1)), z = int(v >> (2 * lg));
    const int ox = x >> 1, oy = y >> 1, oz = z >> 1;
    const int nx = wrapi((x & 1) ? ox + 1 : ox - 1, nc), ny = wrapi((y & 1) ? oy + 1 : oy - 1, nc),
              nz = wrapi((z & 1) ? oz + 1 : oz - 1, nc);
    float s = 0.f;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const float wgt = (cx ? 0.25f : 0.75f) * (cy ? 0.25f : 0.75f) * (cz ? 0.25f : 0.75f);
                const int64_t q = ((((int64_t(cz ? nz : oz) << lgc) + (cy ? ny : oy)) << lgc) + (cx ? nx : ox));
                s += wgt * b2f(Xc[(q << 4) + ch]);
            }
    Y[i] = f2b(s + b2f(S[i]));
}

// dXc(coarse) = up^T dY(fine): each coarse cell gathers the 4 fine cells per
// axis that reference it (weights 1/4, 3/4, 3/4, 1/4 at 2I-1 .. 2I+2).
__global__ __launch_bounds__(256) void k_up_back(const float *__restrict__ dY, float *__restrict__ dXc, int lgc) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= (int64_t(kC) << (3 * lgc))) return;
    const int ch = int(i & 15);
    const int64_t v = i >> 4;
    const int nc = 1 << lgc, lg = lgc + 1, n = nc << 1;
    const int X = int(v & (nc - 1)), Yc = int((v >> lgc) & (nc - 1)), Z = int(v >> (2 * lgc));
    const float w1[4] = {0.25f, 0.75f, 0.75f, 0.25f};
    float s = 0.f;
    for (int a = 0; a < 4; ++a) {
        const int fz = wrapi(2 * Z - 1 + a, n);
        for (int bb = 0; bb < 4; ++bb) {
            const int fy = wrapi(2 * Yc - 1 + bb, n);
            for (int c = 0; c < 4; ++c) {
                const int fx = wrapi(2 * X - 1 + c, n);
                s += w1[a] * w1[bb] * w1[c] * dY[(((((int64_t(fz) << lg) + fy) << lg) + fx) << 4) + ch];
            }
        }
    }
    dXc[i] = s;
}

// dst += src (FP32).
__global__ __launch_bounds__(256) void k_add(const float *__restrict__ src, float *__restrict__ dst, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < m) dst[i] += src[i];
}

// Input packing: channel 0 = f (FP32), others 0, bf16.
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ f, uint16_t *__restrict__ X, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m * kC) return;
    X[i] = (i & 15) ? uint16_t(0) : f2b(f[i >> 4]);
}

// Prediction = channel 0 of the FP32 output.
__global__ __launch_bounds__(256) void k_take0(const float *__restrict__ Y, float *__restrict__ y, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < m) y[i] = Y[i * kC];
}

// MSE: partials of (y - t)^2 / m per workgroup; dY[v][0] = 2 (y - t) / m, other channels 0.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Y, const float *__restrict__ t,
                                             float *__restrict__ dY, double *__restrict__ part, int64_t m) {
    const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double acc = 0.0;
    if (v < m) {
        const float d = Y[v * kC] - t[v];
        acc = double(d) * double(d) / double(m);
        dY[v * kC] = 2.f * d / float(m);
        for (int c = 1; c < kC; ++c) dY[v * kC + c] = 0.f;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_dsum(const double *__restrict__ part, int np, double *__restrict__ out) {
    double a = 0.0;
    for (int b = threadIdx.x; b < np; b += 256) a += part[b];
    a = block_sum(a);
    if (threadIdx.x == 0) out[0] += a;
}

// Adam on FP32 master weights (bias-corrected), refreshes the bf16 copies.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, uint16_t *__restrict__ wb, int64_t np,
                                              float lr, float b1, float b2, float eps, float c1, float c2, float gs) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i] * gs;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    const int64_t k = i / kPsz, r = i % kPsz;
    if (r < kWsz) wb[k * kWsz + r] = f2b(wi);
}

// bf16 copies of the master weights.
__global__ __launch_bounds__(256) void k_wcast(const float *__restrict__ w, uint16_t *__restrict__ wb, int64_t np) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= np) return;
    const int64_t k = i / kPsz, r = i % kPsz;
    if (r < kWsz) wb[k * kWsz + r] = f2b(w[i]);
}

// FP64 field -> FP32 * scale.
__global__ __launch_bounds__(256) void k_to32(const double *__restrict__ a, float *__restrict__ b, double s, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < m) b[i] = float(a[i] * s);
}

// FP32 * scale -> FP64.
__global__ __launch_bounds__(256) void k_to64(const float *__restrict__ a, double *__restrict__ b, double s, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < m) b[i] = double(a[i]) * s;
}

// 2^3-cell average, FP64 (no residual).
__global__ __launch_bounds__(256) void k_avg(const double *__restrict__ f, double *__restrict__ fc, int lgc) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= (int64_t(1) << (3 * lgc))) return;
    const int nc = 1 << lgc, lg = lgc + 1;
    const int X = int(i & (nc - 1)), Y = int((i >> lgc) & (nc - 1)), Z = int(i >> (2 * lgc));
    double s = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) s += f[(((int64_t(2 * Z + c) << lg) + 2 * Y + b) << lg) + 2 * X + a];
    fc[i] = 0.125 * s;
}

// ----------------------------------------------------------------- network
inline unsigned nb(int64_t m) { return unsigned((m + 255) / 256); }

struct Net {
    int levels = 0, lg0 = 0, nconv = 0;
    int64_t npar = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // FP32 master, Adam moments, gradient sums
    uint16_t *wb = nullptr, *wt = nullptr;                            // bf16 weights, flipped for the data gradient
    int64_t step = 0;
    // per level: h (input), a, e (encoder); u, c, d (decoder); Z (bf16 scratch); S0, S1, K (FP32 grads)
    std::vector<uint16_t *> h, a, e, u, c, d, Z;
    std::vector<float *> S0, S1, K;
    float *out = nullptr, *gout = nullptr;  // FP32 [n^3][16]
    float *wpart = nullptr;                 // weight-gradient partials
    double *lpart = nullptr, *lsum = nullptr, *hsum = nullptr;
    std::vector<void *> owned;
    std::mutex mu;
};

np_status nalloc(Net *N, void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes failed", bytes);
        return NP_ENOMEM;
    }
    N->owned.push_back(*p);
    return NP_OK;
}

int64_t vox(int lg) { return int64_t(1) << (3 * lg); }

np_status conv(Net *N, int k, const uint16_t *X, void *Y, int lg, bool relu, bool out32, bool flip, hipStream_t s) {
    const int n = 1 << lg, txv = n < 64 ? n : 64;
    const unsigned grid = unsigned((n / txv) * (n / 4) * n);
    const uint16_t *W = (flip ? N->wt : N->wb) + int64_t(k) * kWsz;
    const float *bias = flip ? nullptr : N->w + int64_t(k) * kPsz + kWsz;
    // z-marching tiles: n / 32 planes per workgroup at n = 64, n / 16 from n = 128 (measured best; below
    // n = 64 the one-plane form keeps more workgroups in flight and wins)
    int zc = g_conv3z == 1 ? (n >= 128 ? n / 16 : n / 32) : (g_conv3z < n ? g_conv3z : n);
    if (g_conv3z && zc >= 2) {
        const int tiles = (n / txv) * (n / kCzY);
        const unsigned g3 = unsigned(tiles * (n / zc));
        if (relu && !out32)
            hipLaunchKernelGGL((k_conv3z<true, false>), dim3(g3), dim3(kCzT), 0, s, X, W, bias, Y, lg, zc);
        else if (!relu && out32)
            hipLaunchKernelGGL((k_conv3z<false, true>), dim3(g3), dim3(kCzT), 0, s, X, W, bias, Y, lg, zc);
        else if (!relu && !out32)
            hipLaunchKernelGGL((k_conv3z<false, false>), dim3(g3), dim3(kCzT), 0, s, X, W, bias, Y, lg, zc);
        else
            hipLaunchKernelGGL((k_conv3z<true, true>), dim3(g3), dim3(kCzT), 0, s, X, W, bias, Y, lg, zc);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }
    if (relu && !out32) hipLaunchKernelGGL((k_conv<true, false>), dim3(grid), dim3(256), 0, s, X, W, bias, Y, lg);
    else if (!relu && out32) hipLaunchKernelGGL((k_conv<false, true>), dim3(grid), dim3(256), 0, s, X, W, bias, Y, lg);
    else if (!relu && !out32) hipLaunchKernelGGL((k_conv<false, false>), dim3(grid), dim3(256), 0, s, X, W, bias, Y, lg);
    else hipLaunchKernelGGL((k_conv<true, true>), dim3(grid), dim3(256), 0, s, X, W, bias, Y, lg);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// Backward through conv k with input `in`, post-activation `act` (null: no
// ReLU), upstream gradient `gy` (FP32); accumulates dW, db and writes the
// input gradient to gx (if not null).
np_status back(Net *N, int k, const uint16_t *in, const uint16_t *act, const float *gy, float *gx, int l,
               hipStream_t s) {
    const int lg = N->lg0 - l;
    const int64_t m = vox(lg) * kC;
    hipLaunchKernelGGL(k_mask, dim3(nb(m)), dim3(256), 0, s, gy, act, N->Z[l], m);
    NP_LAUNCH_CHECK();
    const int n = 1 << lg, txv = n < 64 ? n : 64, ntile = (n / txv) * (n / 4) * n;
    const int nblk = ntile < kWgBlocks ? ntile : kWgBlocks;
    if (g_wgrad_mfma) hipLaunchKernelGGL(k_wgrad_mfma, dim3(nblk), dim3(kWmT), 0, s, in, N->Z[l], N->wpart, lg);
    else hipLaunchKernelGGL(k_wgrad, dim3(nblk), dim3(256), 0, s, in, N->Z[l], N->wpart, lg);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(unsigned((kPsz + 31) / 32)), dim3(256), 0, s, N->wpart, nblk,
                       N->g + int64_t(k) * kPsz);
    NP_LAUNCH_CHECK();
    if (gx) NP_TRY(conv(N, k, N->Z[l], gx, lg, false, true, true, s));
    return NP_OK;
}

// Forward: f (FP32, n^3) -> out [n^3][16] FP32 (channel 0 = prediction).
np_status forward(Net *N, const float *f, hipStream_t s) {
    const int L = N->levels;
    const int64_t m0 = vox(N->lg0);
    hipLaunchKernelGGL(k_pack, dim3(nb(m0 * kC)), dim3(256), 0, s, f, N->h[0], m0);
    NP_LAUNCH_CHECK();
    int k = 0;
    for (int l = 0; l < L; ++l) {
        const int lg = N->lg0 - l;
        if (l > 0) {
            hipLaunchKernelGGL(k_pool, dim3(nb(vox(lg) * kC)), dim3(256), 0, s, N->e[l - 1], N->h[l], lg);
            NP_LAUNCH_CHECK();
        }
        NP_TRY(conv(N, k++, N->h[l], N->a[l], lg, true, false, false, s));
        NP_TRY(conv(N, k++, N->a[l], N->e[l], lg, true, false, false, s));
    }
    const uint16_t *dn = N->e[L - 1];
    for (int l = L - 2; l >= 0; --l) {
        const int lg = N->lg0 - l;
        hipLaunchKernelGGL(k_up_add, dim3(nb(vox(lg) * kC)), dim3(256), 0, s, dn, N->e[l], N->u[l], lg);
        NP_LAUNCH_CHECK();
        NP_TRY(conv(N, k++, N->u[l], N->c[l], lg, true, false, false, s));
        NP_TRY(conv(N, k++, N->c[l], N->d[l], lg, true, false, false, s));
        dn = N->d[l];
    }
    NP_TRY(conv(N, k, dn, N->out, N->lg0, false, true, false, s));
    return NP_OK;
}

// Backward from N->gout (gradient wrt out); gradient sums accumulate in N->g.
np_status backward(Net *N, hipStream_t s) {
    const int L = N->levels;
    const int kout = N->nconv - 1;
    const uint16_t *dtop = L >= 2 ? N->d[0] : N->e[0];
    NP_TRY(back(N, kout, dtop, nullptr, N->gout, N->S0[0], 0, s));
    // decoder levels 0 .. L-2 (conv indices 2L + 2 (L-2-l) .. +1)
    for (int l = 0; l <= L - 2; ++l) {
        const int k1 = 2 * L + 2 * (L - 2 - l), k2 = k1 + 1;
        NP_TRY(back(N, k2, N->c[l], N->d[l], N->S0[l], N->S1[l], l, s));
        NP_TRY(back(N, k1, N->u[l], N->c[l], N->S1[l], N->K[l], l, s));
        const int lgc = N->lg0 - l - 1;
        hipLaunchKernelGGL(k_up_back, dim3(nb(vox(lgc) * kC)), dim3(256), 0, s, N->K[l], N->S0[l + 1], lgc);
        NP_LAUNCH_CHECK();
    }
    for (int l = L - 1; l >= 0; --l) {
        const int lg = N->lg0 - l;
        const int64_t m = vox(lg) * kC;
        if (l < L - 1) {
            hipLaunchKernelGGL(k_add, dim3(nb(m)), dim3(256), 0, s, N->K[l], N->S0[l], m);
            NP_LAUNCH_CHECK();
        }
        NP_TRY(back(N, 2 * l + 1, N->a[l], N->e[l], N->S0[l], N->S1[l], l, s));
        NP_TRY(back(N, 2 * l, N->h[l], N->a[l], N->S1[l], l > 0 ? N->S0[l] : nullptr, l, s));
        if (l > 0) {
            NP_HIP_TRY(hipMemsetAsync(N->S0[l - 1], 0, sizeof(float) * vox(lg + 1) * kC, s));
            hipLaunchKernelGGL(k_pool_back, dim3(nb(vox(lg + 1) * kC)), dim3(256), 0, s, N->S0[l], N->S0[l - 1], lg + 1);
            NP_LAUNCH_CHECK();
        }
    }
    return NP_OK;
}

np_status refresh(Net *N, hipStream_t s) {
    hipLaunchKernelGGL(k_wcast, dim3(nb(N->npar)), dim3(256), 0, s, N->w, N->wb, N->npar);
    NP_LAUNCH_CHECK();
    for (int k = 0; k < N->nconv; ++k) {
        hipLaunchKernelGGL(k_wflip, dim3(nb(kWsz)), dim3(256), 0, s, N->wb + int64_t(k) * kWsz,
                           N->wt + int64_t(k) * kWsz);
        NP_LAUNCH_CHECK();
    }
    return NP_OK;
}

np_status loss_grad(Net *N, const float *target, hipStream_t s) {
    const int64_t m = vox(N->lg0);
    hipLaunchKernelGGL(k_mse, dim3(nb(m)), dim3(256), 0, s, N->out, target, N->gout, N->lpart, m);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_dsum, dim3(1), dim3(256), 0, s, N->lpart, int(nb(m)), N->lsum);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

void free_net(Net *N) {
    for (void *p : N->owned) (void)hipFree(p);
    if (N->hsum) (void)hipHostFree(N->hsum);
    delete N;
}

}  // namespace

// Attached network for warm starts (np_cnn_attach).
static std::mutex g_cnn_mu;
static Net *g_attached = nullptr;

// Warm start used by the solver: x0 (FP64, fine grid of 2^lg cells) from f
// through the attached network at its input resolution, with the fine f
// restricted by averaging and the prediction prolongated back.  tmp buffers:
// fl[l], xl[l] FP64 for levels 1..ell of the hierarchy.  Returns NP_EINVAL
// when no network fits this grid.
np_status cnn_warm_start(int d, int lg, int bc, const double *f, double *x0, const std::vector<void *> &fl,
                         const std::vector<void *> &xl, double *f32buf_bytes_unused, hipStream_t s, bool *used) {
    (void)f32buf_bytes_unused;
    *used = false;
    std::lock_guard<std::mutex> lk(g_cnn_mu);
    Net *N = g_attached;
    if (!N || d != 3 || lg < N->lg0) return NP_OK;
    const int ell = lg - N->lg0;
    if (ell >= int(fl.size())) return NP_OK;
    std::lock_guard<std::mutex> lk2(N->mu);
    // restrict f down to the network's grid
    const double *src = f;
    for (int l = 1; l <= ell; ++l) {
        hipLaunchKernelGGL(k_avg, dim3(nb(vox(lg - l))), dim3(256), 0, s, src, (double *)fl[l], lg - l);
        NP_LAUNCH_CHECK();
        src = (const double *)fl[l];
    }
    const int64_t mc = vox(N->lg0);
    // scale by the rms of the coarse rhs (the map f -> x is linear)
    const unsigned nb2 = std::min<unsigned>(kRedBlocks, unsigned((mc + 255) / 256));
    hipLaunchKernelGGL((k_sum<double>), dim3(nb2), dim3(256), 0, s, src, mc, 1, N->lpart);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, N->lpart, int(nb2), N->lsum, 0);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipMemcpyAsync(N->hsum, N->lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    const double rms = std::sqrt(N->hsum[0] / double(mc));
    if (!(rms > 0.0) || !std::isfinite(rms)) return NP_OK;
    float *in = N->S1[0], *pred = N->S1[0] + mc;  // FP32 scratch (the gradient buffers are idle)
    hipLaunchKernelGGL(k_to32, dim3(nb(mc)), dim3(256), 0, s, src, in, 1.0 / rms, mc);
    NP_LAUNCH_CHECK();
    NP_TRY(forward(N, in, s));
    hipLaunchKernelGGL(k_take0, dim3(nb(mc)), dim3(256), 0, s, N->out, pred, mc);
    NP_LAUNCH_CHECK();
    double *xc = ell > 0 ? (double *)xl[ell] : x0;
    hipLaunchKernelGGL(k_to64, dim3(nb(mc)), dim3(256), 0, s, pred, xc, rms, mc);
    NP_LAUNCH_CHECK();
    // prolongate back to the fine grid
    for (int l = ell - 1; l >= 0; --l) {
        double *xf = l > 0 ? (double *)xl[l] : x0;
        const int64_t mf = vox(lg - l);
        hipLaunchKernelGGL((k_zero<double>), dim3(nb(mf)), dim3(256), 0, s, xf, mf, nullptr);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_prolong_add<3, double>), dim3(nb(mf)), dim3(256), 0, s, (const double *)xc, xf,
                           lg - l - 1, bc, nullptr);
        NP_LAUNCH_CHECK();
        xc = xf;
    }
    *used = true;
    return NP_OK;
}

// log2 of the attached network's grid size per axis, -1 when none is attached.
int cnn_attached_lg() {
    std::lock_guard<std::mutex> lk(g_cnn_mu);
    return g_attached ? g_attached->lg0 : -1;
}

// Network prediction on a coarse level of the solver's cycle (the learned
// coarse-grid correction): xc = rms * N(fc / rms) on the attached network's own
// grid, fc the level's restricted residual (device FP64, n_in^3 cells, n_in =
// 2^lg), rms its root mean square.  *used = false (xc untouched) when no
// network is attached, its grid is not 2^lg per axis, or fc is zero.  Reads
// the rms on the host (the stream is synchronised).
np_status cnn_coarse_guess(int lg, const double *fc, double *xc, hipStream_t s, bool *used) {
    *used = false;
    std::lock_guard<std::mutex> lk(g_cnn_mu);
    Net *N = g_attached;
    if (!N || N->lg0 != lg) return NP_OK;
    std::lock_guard<std::mutex> lk2(N->mu);
    const int64_t mc = vox(lg);
    const unsigned nb2 = std::min<unsigned>(kRedBlocks, unsigned((mc + 255) / 256));
    hipLaunchKernelGGL((k_sum<double>), dim3(nb2), dim3(256), 0, s, fc, mc, 1, N->lpart);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, N->lpart, int(nb2), N->lsum, 0);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipMemcpyAsync(N->hsum, N->lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    const double rms = std::sqrt(N->hsum[0] / double(mc));
    if (!(rms > 0.0) || !std::isfinite(rms)) return NP_OK;
    float *in = N->S1[0], *pred = N->S1[0] + mc;  // FP32 scratch (the gradient buffers are idle)
    hipLaunchKernelGGL(k_to32, dim3(nb(mc)), dim3(256), 0, s, fc, in, 1.0 / rms, mc);
    NP_LAUNCH_CHECK();
    NP_TRY(forward(N, in, s));
    hipLaunchKernelGGL(k_take0, dim3(nb(mc)), dim3(256), 0, s, N->out, pred, mc);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_to64, dim3(nb(mc)), dim3(256), 0, s, pred, xc, rms, mc);
    NP_LAUNCH_CHECK();
    *used = true;
    return NP_OK;
}

}  // namespace np

using namespace np;

struct np_cnn {
    Net *net;
};

extern "C" np_status np_cnn_create(int n_in, int levels, np_cnn **out) {
    clear_error();
    if (!out || !is_pow2(n_in) || levels < 1 || levels > 6 || (n_in >> (levels - 1)) < 16 || n_in > 512) {
        set_error("network input must be a power of two >= 16 * 2^(levels-1), <= 512");
        return NP_EINVAL;
    }
    Net *N = new Net;
    N->levels = levels;
    N->lg0 = ilog2(n_in);
    N->nconv = 4 * levels - 1;
    N->npar = int64_t(N->nconv) * kPsz;
    np_status st = NP_OK;
    auto A = [&](void **p, size_t b) {
        if (st == NP_OK) st = nalloc(N, p, b);
        if (st == NP_OK) (void)hipMemset(*p, 0, b);
    };
    A((void **)&N->w, sizeof(float) * N->npar);
    A((void **)&N->m, sizeof(float) * N->npar);
    A((void **)&N->v, sizeof(float) * N->npar);
    A((void **)&N->g, sizeof(float) * N->npar);
    A((void **)&N->wb, sizeof(uint16_t) * N->nconv * kWsz);
    A((void **)&N->wt, sizeof(uint16_t) * N->nconv * kWsz);
    N->h.assign(levels, nullptr); N->a = N->h; N->e = N->h; N->u = N->h; N->c = N->h; N->d = N->h; N->Z = N->h;
    N->S0.assign(levels, nullptr); N->S1 = N->S0; N->K = N->S0;
    for (int l = 0; l < levels; ++l) {
        const size_t mb = size_t(vox(N->lg0 - l)) * kC;
        A((void **)&N->h[l], 2 * mb);
        A((void **)&N->a[l], 2 * mb);
        A((void **)&N->e[l], 2 * mb);
        A((void **)&N->Z[l], 2 * mb);
        A((void **)&N->S0[l], 4 * mb);
        A((void **)&N->S1[l], 4 * mb);
        if (l < levels - 1) {
            A((void **)&N->u[l], 2 * mb);
            A((void **)&N->c[l], 2 * mb);
            A((void **)&N->d[l], 2 * mb);
            A((void **)&N->K[l], 4 * mb);
        }
    }
    const size_t m0 = size_t(vox(N->lg0));
    A((void **)&N->out, 4 * m0 * kC);
    A((void **)&N->gout, 4 * m0 * kC);
    A((void **)&N->wpart, sizeof(float) * kWgBlocks * kPsz);
    A((void **)&N->lpart, sizeof(double) * std::max<size_t>(kRedBlocks, (m0 + 255) / 256));
    A((void **)&N->lsum, sizeof(double));
    if (st == NP_OK && hipHostMalloc((void **)&N->hsum, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc failed");
        st = NP_ENOMEM;
    }
    if (st != NP_OK) {
        free_net(N);
        return st;
    }
    *out = new np_cnn{N};
    return NP_OK;
}

extern "C" void np_cnn_destroy(np_cnn *net) {
    if (!net) return;
    {
        std::lock_guard<std::mutex> lk(g_cnn_mu);
        if (g_attached == net->net) g_attached = nullptr;
    }
    (void)hipDeviceSynchronize();
    free_net(net->net);
    delete net;
}

extern "C" int64_t np_cnn_num_params(const np_cnn *net) { return net ? net->net->npar : -1; }

extern "C" np_status np_cnn_set_params(np_cnn *net, const float *host, int64_t count) {
    clear_error();
    if (!net || !host || count != net->net->npar) { set_error("parameter count mismatch"); return NP_EINVAL; }
    Net *N = net->net;
    std::lock_guard<std::mutex> lk(N->mu);
    NP_HIP_TRY(hipMemcpy(N->w, host, sizeof(float) * count, hipMemcpyHostToDevice));
    NP_HIP_TRY(hipMemset(N->m, 0, sizeof(float) * count));
    NP_HIP_TRY(hipMemset(N->v, 0, sizeof(float) * count));
    N->step = 0;
    NP_TRY(refresh(N, nullptr));
    NP_HIP_TRY(hipDeviceSynchronize());
    return NP_OK;
}

extern "C" np_status np_cnn_get_params(const np_cnn *net, float *host, int64_t count) {
    clear_error();
    if (!net || !host || count != net->net->npar) { set_error("parameter count mismatch"); return NP_EINVAL; }
    NP_HIP_TRY(hipMemcpy(host, net->net->w, sizeof(float) * count, hipMemcpyDeviceToHost));
    return NP_OK;
}

extern "C" np_status np_cnn_get_grads(const np_cnn *net, float *host, int64_t count) {
    clear_error();
    if (!net || !host || count != net->net->npar) { set_error("parameter count mismatch"); return NP_EINVAL; }
    NP_HIP_TRY(hipMemcpy(host, net->net->g, sizeof(float) * count, hipMemcpyDeviceToHost));
    return NP_OK;
}

extern "C" np_status np_cnn_forward(np_cnn *net, const float *in, float *out, void *stream) {
    clear_error();
    if (!net || !in || !out) { set_error("null argument"); return NP_EINVAL; }
    Net *N = net->net;
    std::lock_guard<std::mutex> lk(N->mu);
    hipStream_t s = (hipStream_t)stream;
    NP_TRY(forward(N, in, s));
    hipLaunchKernelGGL(k_take0, dim3(nb(vox(N->lg0))), dim3(256), 0, s, N->out, out, vox(N->lg0));
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// Zeroes the gradient sums, then forward + MSE + backward for each pair; the
// gradient sums (not averaged) are left in the network.  *loss: sum of the
// pairs' MSE.
static np_status grads_for(Net *N, int batch, const float *const *in, const float *const *target, double *loss,
                           hipStream_t s) {
    NP_HIP_TRY(hipMemsetAsync(N->g, 0, sizeof(float) * N->npar, s));
    NP_HIP_TRY(hipMemsetAsync(N->lsum, 0, sizeof(double), s));
    for (int b = 0; b < batch; ++b) {
        NP_TRY(forward(N, in[b], s));
        NP_TRY(loss_grad(N, target[b], s));
        NP_TRY(backward(N, s));
    }
    NP_HIP_TRY(hipMemcpyAsync(N->hsum, N->lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    if (loss) *loss = N->hsum[0];
    return NP_OK;
}

extern "C" np_status np_cnn_gradients(np_cnn *net, int batch, const float *const *in, const float *const *target,
                                      double *loss, void *stream) {
    clear_error();
    if (!net || batch <= 0 || !in || !target) { set_error("bad argument"); return NP_EINVAL; }
    Net *N = net->net;
    std::lock_guard<std::mutex> lk(N->mu);
    return grads_for(N, batch, in, target, loss, (hipStream_t)stream);
}

// Gradients of the batch, then one Adam step on their mean.
static np_status train_step(Net *N, int batch, const float *const *in, const float *const *target, float lr,
                            double *loss, hipStream_t s) {
    NP_TRY(grads_for(N, batch, in, target, loss, s));
    N->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, float(N->step)), c2 = 1.f - std::pow(b2, float(N->step));
    hipLaunchKernelGGL(k_adam, dim3(nb(N->npar)), dim3(256), 0, s, N->w, N->m, N->v, N->g, N->wb, N->npar, lr, b1, b2,
                       eps, c1, c2, 1.f / float(batch));
    NP_LAUNCH_CHECK();
    for (int k = 0; k < N->nconv; ++k) {
        hipLaunchKernelGGL(k_wflip, dim3(nb(kWsz)), dim3(256), 0, s, N->wb + int64_t(k) * kWsz,
                           N->wt + int64_t(k) * kWsz);
        NP_LAUNCH_CHECK();
    }
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_cnn_train_step(np_cnn *net, int batch, const float *const *in, const float *const *target,
                                       float lr, double *loss, void *stream) {
    clear_error();
    if (!net || batch <= 0 || !in || !target || !(lr > 0.f)) { set_error("bad argument"); return NP_EINVAL; }
    Net *N = net->net;
    std::lock_guard<std::mutex> lk(N->mu);
    return train_step(N, batch, in, target, lr, loss, (hipStream_t)stream);
}

// Restricts f (and p) from the fine grid to the network's grid by repeated
// 2^3 averaging, scales both by 1 / rms(restricted f) and writes FP32 copies.
static np_status prepare(Net *N, int lg, const double *f, const double *p, float *in, float *target, double *scale,
                        hipStream_t s) {
    const int ell = lg - N->lg0;
    std::vector<double *> tmp;
    double *fb = nullptr, *pb = nullptr;
    auto chain = [&](const double *src, double **res) -> np_status {
        const double *cur = src;
        for (int l = 1; l <= ell; ++l) {
            double *dst = nullptr;
            if (hipMalloc((void **)&dst, sizeof(double) * vox(lg - l)) != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc failed");
                return NP_ENOMEM;
            }
            tmp.push_back(dst);
            hipLaunchKernelGGL(k_avg, dim3(nb(vox(lg - l))), dim3(256), 0, s, cur, dst, lg - l);
            NP_LAUNCH_CHECK();
            cur = dst;
        }
        *res = const_cast<double *>(cur);
        return NP_OK;
    };
    np_status st = chain(f, &fb);
    if (st == NP_OK && p) st = chain(p, &pb);
    const int64_t mc = vox(N->lg0);
    double rms = 0.0;
    if (st == NP_OK) {
        const unsigned nb2 = std::min<unsigned>(kRedBlocks, unsigned((mc + 255) / 256));
        hipLaunchKernelGGL((k_sum<double>), dim3(nb2), dim3(256), 0, s, fb, mc, 1, N->lpart);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, N->lpart, int(nb2), N->lsum, 0);
        if (hipMemcpyAsync(N->hsum, N->lsum, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("reduction failed");
            st = NP_EHIP;
        }
        rms = std::sqrt(N->hsum[0] / double(mc));
    }
    if (st == NP_OK) {
        const double sc = rms > 0.0 ? 1.0 / rms : 1.0;
        hipLaunchKernelGGL(k_to32, dim3(nb(mc)), dim3(256), 0, s, fb, in, sc, mc);
        if (p && target) hipLaunchKernelGGL(k_to32, dim3(nb(mc)), dim3(256), 0, s, pb, target, sc, mc);
        if (hipStreamSynchronize(s) != hipSuccess) { set_error("prepare failed"); st = NP_EHIP; }
        if (scale) *scale = rms;
    }
    for (double *q : tmp) (void)hipFree(q);
    return st;
}

extern "C" np_status np_cnn_prepare(np_cnn *net, np_dims dims, const double *f, const double *p, float *in,
                                    float *target, double *scale, void *stream) {
    clear_error();
    const int lg = check_grid(dims);
    if (lg < 0 || dims.ndim != 3 || !net || !f || !in) { set_error("bad argument"); return NP_EINVAL; }
    Net *N = net->net;
    if (lg < N->lg0) { set_error("grid coarser than the network input"); return NP_EINVAL; }
    std::lock_guard<std::mutex> lk(N->mu);
    return prepare(N, lg, f, p, in, target, scale, (hipStream_t)stream);
}

extern "C" np_status np_cnn_attach(np_cnn *net) {
    std::lock_guard<std::mutex> lk(g_cnn_mu);
    g_attached = net ? net->net : nullptr;
    return NP_OK;
}

// File: "NPCNN1\n", int32 levels, int32 n_in, int64 count, count float32 master weights.
extern "C" np_status np_cnn_save(const np_cnn *net, const char *path) {
    clear_error();
    if (!net || !path) { set_error("bad argument"); return NP_EINVAL; }
    const Net *N = net->net;
    std::vector<float> w(N->npar);
    NP_HIP_TRY(hipMemcpy(w.data(), N->w, sizeof(float) * N->npar, hipMemcpyDeviceToHost));
    FILE *fp = std::fopen(path, "wb");
    if (!fp) { set_error("cannot open %s", path); return NP_EINVAL; }
    const int32_t hdr[2] = {N->levels, 1 << N->lg0};
    const int64_t cnt = N->npar;
    const bool ok = std::fwrite("NPCNN1\n", 1, 7, fp) == 7 && std::fwrite(hdr, sizeof hdr, 1, fp) == 1 &&
                    std::fwrite(&cnt, sizeof cnt, 1, fp) == 1 && std::fwrite(w.data(), sizeof(float), cnt, fp) == size_t(cnt);
    std::fclose(fp);
    if (!ok) { set_error("write failed: %s", path); return NP_EINVAL; }
    return NP_OK;
}

extern "C" np_status np_cnn_open(const char *path, np_cnn **out) {
    clear_error();
    if (!path || !out) { set_error("bad argument"); return NP_EINVAL; }
    FILE *fp = std::fopen(path, "rb");
    if (!fp) { set_error("cannot open %s", path); return NP_EINVAL; }
    char magic[7];
    int32_t hdr[2];
    int64_t cnt = 0;
    bool ok = std::fread(magic, 1, 7, fp) == 7 && std::memcmp(magic, "NPCNN1\n", 7) == 0 &&
              std::fread(hdr, sizeof hdr, 1, fp) == 1 && std::fread(&cnt, sizeof cnt, 1, fp) == 1 && cnt > 0 &&
              cnt < (int64_t(1) << 30);
    std::vector<float> w;
    if (ok) {
        w.resize(cnt);
        ok = std::fread(w.data(), sizeof(float), cnt, fp) == size_t(cnt);
    }
    std::fclose(fp);
    if (!ok) { set_error("not a network file: %s", path); return NP_EINVAL; }
    NP_TRY(np_cnn_create(hdr[1], hdr[0], out));
    np_status st = np_cnn_set_params(*out, w.data(), cnt);
    if (st != NP_OK) {
        np_cnn_destroy(*out);
        *out = nullptr;
    }
    return st;
}

// Network owned by the library (np_cnn_load).
static np_cnn *g_owned = nullptr;

extern "C" np_status np_cnn_load(const char *path) {
    clear_error();
    np_cnn *net = nullptr;
    if (path) NP_TRY(np_cnn_open(path, &net));
    np_cnn *old = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cnn_mu);
        old = g_owned;
        g_owned = net;
        g_attached = net ? net->net : nullptr;
    }
    if (old) np_cnn_destroy(old);
    return NP_OK;
}

// He-normal weights from a seeded host generator: fan-in 27 for the first
// convolution (input channel 0 only), 27 x 16 otherwise; the output
// convolution writes channel 0 only and starts 10x smaller than its fan-in
// scale (the targets' variance is ~1e-2 of the inputs'; a full-scale first
// output makes the early Adam steps shrink every layer until the ReLUs die).
// Biases zero; Adam state reset.
extern "C" np_status np_cnn_init(np_cnn *net, uint64_t seed) {
    clear_error();
    if (!net) { set_error("bad argument"); return NP_EINVAL; }
    Net *N = net->net;
    std::vector<float> w(N->npar, 0.f);
    std::mt19937_64 eng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int k = 0; k < N->nconv; ++k) {
        float *W = w.data() + int64_t(k) * kPsz;
        for (int t = 0; t < kTaps; ++t)
            for (int o = 0; o < kC; ++o)
                for (int c = 0; c < kC; ++c) {
                    double sd;
                    if (k == 0) sd = c == 0 ? std::sqrt(2.0 / kTaps) : 0.0;
                    else if (k == N->nconv - 1) sd = o == 0 ? 0.1 * std::sqrt(1.0 / (kTaps * kC)) : 0.0;
                    else sd = std::sqrt(2.0 / (kTaps * kC));
                    W[(t * kC + o) * kC + c] = sd > 0.0 ? float(sd * nd(eng)) : 0.f;
                }
    }
    return np_cnn_set_params(net, w.data(), N->npar);
}

namespace {
// Reads `"key": number` members of a flat JSON object into the named slots;
// any other key or form is an error.
bool parse_cfg(const char *js, const char *const *keys, double *vals, int nkeys, std::string *err) {
    if (!js) return true;
    const char *q = js;
    auto ws = [&]() { while (*q == ' ' || *q == '\t' || *q == '\n' || *q == '\r') ++q; };
    ws();
    if (*q != '{') { *err = "configuration must be a JSON object"; return false; }
    ++q;
    ws();
    if (*q == '}') return true;
    for (;;) {
        ws();
        if (*q != '"') { *err = "expected a quoted key"; return false; }
        const char *k0 = ++q;
        while (*q && *q != '"') ++q;
        if (!*q) { *err = "unterminated key"; return false; }
        const std::string key(k0, q - k0);
        ++q;
        ws();
        if (*q != ':') { *err = "expected ':' after " + key; return false; }
        ++q;
        ws();
        char *end = nullptr;
        const double v = std::strtod(q, &end);
        if (end == q || !std::isfinite(v)) { *err = "value of " + key + " is not a number"; return false; }
        q = end;
        int idx = -1;
        for (int i = 0; i < nkeys; ++i)
            if (key == keys[i]) idx = i;
        if (idx < 0) { *err = "unknown key " + key; return false; }
        vals[idx] = v;
        ws();
        if (*q == ',') { ++q; continue; }
        if (*q == '}') {
            ++q;
            ws();
            if (*q) { *err = "text after the object"; return false; }
            return true;
        }
        *err = "expected ',' or '}'";
        return false;
    }
}
}  // namespace

// Trains a new network on (rhs, p) pairs and writes it to weights_out.
extern "C" np_status np_cnn_train(const np_dims *dims, np_bc bc, int npairs, const double *const *rhs,
                                  const double *const *p, const char *cfg_json, const char *weights_out,
                                  double *epoch_loss) {
    clear_error();
    if (!dims || !rhs || !p || !weights_out || npairs <= 0) { set_error("bad argument"); return NP_EINVAL; }
    if (bc != NP_BC_PERIODIC) { set_error("the network is periodic: bc must be NP_BC_PERIODIC"); return NP_EINVAL; }
    static const char *const keys[] = {"n_in", "levels", "epochs", "batch", "lr", "seed", "verbose"};
    double cfg[7] = {128, 4, 10, 4, 5e-4, 0, 0};
    std::string err;
    if (!parse_cfg(cfg_json, keys, cfg, 7, &err)) { set_error("configuration: %s", err.c_str()); return NP_EINVAL; }
    const bool verbose = cfg[6] != 0.0;
    const int n_in = int(cfg[0]), levels = int(cfg[1]), epochs = int(cfg[2]), batch = int(cfg[3]);
    const float lr = float(cfg[4]);
    const uint64_t seed = uint64_t(cfg[5]);
    if (epochs < 1 || batch < 1 || !(lr > 0.f) || cfg[5] < 0) { set_error("configuration: bad epochs, batch, lr or seed"); return NP_EINVAL; }
    std::vector<int> lgs(npairs);
    for (int i = 0; i < npairs; ++i) {
        lgs[i] = check_grid(dims[i]);
        if (lgs[i] < 0 || dims[i].ndim != 3 || !rhs[i] || !p[i]) { set_error("pair %d: bad grid or pointer", i); return NP_EINVAL; }
        if ((int64_t(1) << lgs[i]) < n_in) { set_error("pair %d: grid coarser than n_in", i); return NP_EINVAL; }
    }
    np_cnn *net = nullptr;
    NP_TRY(np_cnn_create(n_in, levels, &net));
    Net *N = net->net;
    const int64_t mc = vox(N->lg0);
    float *buf = nullptr;
    np_status st = np_cnn_init(net, seed);
    if (st == NP_OK && hipMalloc((void **)&buf, sizeof(float) * mc * 2 * npairs) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %lld bytes for the prepared pairs failed", (long long)(sizeof(float) * mc * 2 * npairs));
        st = NP_ENOMEM;
    }
    std::vector<const float *> xin(npairs), tgt(npairs);
    {
        std::lock_guard<std::mutex> lk(N->mu);
        for (int i = 0; i < npairs && st == NP_OK; ++i) {
            float *xi = buf + mc * 2 * i, *ti = xi + mc;
            xin[i] = xi;
            tgt[i] = ti;
            st = prepare(N, lgs[i], rhs[i], p[i], xi, ti, nullptr, nullptr);
        }
        const auto t0 = std::chrono::steady_clock::now();
        // seeded Fisher-Yates order per epoch, minibatches of `batch` pairs
        std::mt19937_64 eng(seed ^ 0x9e3779b97f4a7c15ull);
        std::vector<int> order(npairs);
        std::vector<const float *> bx, bt;
        for (int ep = 0; ep < epochs && st == NP_OK; ++ep) {
            for (int i = 0; i < npairs; ++i) order[i] = i;
            for (int i = npairs - 1; i > 0; --i) std::swap(order[i], order[eng() % uint64_t(i + 1)]);
            double tot = 0.0;
            for (int i0 = 0; i0 < npairs && st == NP_OK; i0 += batch) {
                const int nb2 = std::min(batch, npairs - i0);
                bx.assign(nb2, nullptr);
                bt.assign(nb2, nullptr);
                for (int j = 0; j < nb2; ++j) {
                    bx[j] = xin[order[i0 + j]];
                    bt[j] = tgt[order[i0 + j]];
                }
                double l = 0.0;
                st = train_step(N, nb2, bx.data(), bt.data(), lr, &l, nullptr);
                tot += l;
            }
            if (epoch_loss) epoch_loss[ep] = tot / npairs;
            if (verbose && st == NP_OK) {
                const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                std::fprintf(stderr, "np_cnn_train: epoch %d/%d mean mse %.4e (%.1f s)\n", ep + 1, epochs,
                             tot / npairs, sec);
                std::fflush(stderr);
            }
        }
    }
    if (buf) (void)hipFree(buf);
    if (st == NP_OK) st = np_cnn_save(net, weights_out);
    np_cnn_destroy(net);
    return st;
}
