// Level kernels of the default (unfused) multigrid path, tuned for gfx950:
//  - k_sweep:     one weighted-Jacobi sweep, two cells per thread, optionally
//                 reducing ||f - A x_in||^2 of its input (the residual the sweep
//                 computes anyway) into one partial sum per workgroup; ZERO:
//                 the sweep from a zero iterate (x = w f); ZERO2: the first two
//                 sweeps from a zero iterate in one pass (the iterate after the
//                 first, w f, is formed on the fly from f);
//  - k_sweep3, k_restrict3, k_prolong3, k_ir_resid3: the same operations on
//                 3D levels of n >= 128 with 2.5D (z-marching) blocking;
//  - k_restrict:  residual and 2^d-cell average with coalesced fine-grid reads:
//                 a workgroup owns a 64 x 2 x 2 (3D) / 128 x 2 (2D) block of fine
//                 cells, each thread one residual, children summed through LDS;
//  - k_tail:      the whole V-cycle below a level of 16^3 (3D) / 64^2 (2D) cells
//                 in one workgroup, every level resident in LDS.
// Arithmetic per cell is that of mg_kernels.h (same expressions and orders).
#pragma once

#include <type_traits>

#include "mg_kernels.h"
#include "np_internal.h"

namespace np {

constexpr int kSweepCells = 2 * kBlock;  // cells per workgroup of k_sweep

// Iterate w f read through a functor: the state after a first sweep from a
// zero iterate, formed on the fly (ZERO2 kernels fuse that sweep and the next).
template <class S> struct Pair;
template <class S> struct LdW {
    const S *f;
    typename St<S>::C w;
    __device__ __forceinline__ typename St<S>::C operator()(int64_t q) const { return w * St<S>::ld(f + q); }
    __device__ __forceinline__ void pair(int64_t q, typename St<S>::C &a, typename St<S>::C &b) const {
        Pair<S>::ld(f + q, a, b);
        a *= w;
        b *= w;
    }
};

template <int D, class S, bool ZERO, bool NORM, bool ZERO2 = false>
__global__ __launch_bounds__(kBlock) void k_sweep(const S *__restrict__ f, const S *__restrict__ xin,
                                                  S *__restrict__ xout, double *__restrict__ partial, int lg,
                                                  int bc, typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                  const int *stop) {
    typedef typename St<S>::C C;
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    // XCD-contiguous order for cache-resident (FP32/BF16) fields; measured slower
    // for FP64 fields, which stream from HBM
    const unsigned blk = sizeof(S) < 8 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    for (int64_t base = int64_t(blk) * kSweepCells; base < m; base += int64_t(gridDim.x) * kSweepCells)
#pragma unroll
    for (int u = 0; u < kSweepCells / kBlock; ++u) {
        const int64_t c = base + u * kBlock + threadIdx.x;
        if (c < m) {
            const C fc = St<S>::ld(f + c);
            if (ZERO) {
                St<S>::st(xout + c, wdiag * fc);
            } else {
                int i, j, k;
                decode<D>(c, lg, i, j, k);
                const C xc = ZERO2 ? wdiag * fc : St<S>::ld(xin + c);
                const C s = ZERO2 ? nb_sum<D, C>(LdW<S>{f, wdiag}, c, i, j, k, lg, bc, xc)
                                  : nb_sum<D, C>(Ld<S>{xin}, c, i, j, k, lg, bc, xc);
                const C r = fc - (C(2 * D) * xc - s) * inv_h2;
                if (NORM) acc += double(r) * double(r);
                St<S>::st(xout + c, xc + wdiag * r);
            }
        }
    }
    if (NORM) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// ------------------------------------------------------------- z-marching
// 2.5D blocking of 3D level kernels on n >= TX: a workgroup of kS3Threads
// threads owns a TX x TY column tile and `zc` consecutive planes; each thread
// owns CPT adjacent columns along x (CPT = 2 for 2-byte storage, so that each
// access moves 4 bytes; 1 otherwise).  A thread keeps its columns' values of
// the iterate at z-1, z, z+1 in registers; the in-plane neighbours come from
// a double-buffered LDS copy of the plane with a one-cell halo.  The loads of
// plane z+1 are issued before plane z is used, and every lane issues the same
// loads on every plane (the z+1 value through a clamped address and a sign,
// one halo slot per thread -- a single cell, loaded as the aligned pair that
// holds it when CPT = 2, or a run of CPT cells -- threads without a slot
// reloading their own cells, the plane after the last one clamped), so the
// compiler can wait for the older loads only and keep the next plane in
// flight.  Every value is read from HBM once (halo cells are L2 hits).
// Workgroups are mapped XCD-contiguously.
constexpr int kS3Threads = 512;

// Two adjacent values (at an even index) of a field in storage S, loaded and
// stored as one vector access.
template <class S> struct Pair;
template <> struct Pair<double> {
    static __device__ __forceinline__ void ld(const double *p, double &a, double &b) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        a = v.x;
        b = v.y;
    }
    static __device__ __forceinline__ void st(double *p, double a, double b) {
        *reinterpret_cast<double2 *>(p) = make_double2(a, b);
    }
};
template <> struct Pair<float> {
    static __device__ __forceinline__ void ld(const float *p, float &a, float &b) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        a = v.x;
        b = v.y;
    }
    static __device__ __forceinline__ void st(float *p, float a, float b) {
        *reinterpret_cast<float2 *>(p) = make_float2(a, b);
    }
};
template <> struct Pair<bf16> {  // element 0 in the low half (little endian)
    static __device__ __forceinline__ void ld(const bf16 *p, float &a, float &b) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
        a = __uint_as_float(v << 16);
        b = __uint_as_float(v & 0xffff0000u);
    }
    static __device__ __forceinline__ void st(bf16 *p, float a, float b) {
        *reinterpret_cast<uint32_t *>(p) = float2_to_bf16x2(a, b);
    }
};

// Tile shape of the z-marching kernels for storage S: two cells per thread
// along x in every precision (paired accesses of 4, 8 or 16 bytes).  The
// one-pass level kernels gained most: at 256^3 the up-leg FP64 109 -> 93 us,
// FP32 54 -> 47 us, the zero-start down-leg FP64 91 -> 74 us, FP32 56 -> 48 us
// against one cell per thread.
template <class S> struct ZCfg {
    static constexpr int TX = 128;  // cells per tile row
    static constexpr int CPT = 2;   // cells per thread along x
};

template <class C, int TX, int CPT>
struct ZMarch {
    static constexpr int TP = TX / CPT;          // threads per tile row
    static constexpr int TY = kS3Threads / TP;   // tile rows
    static constexpr int NH = 2 * TY + 2 * TP;   // halo slots: x-halo cells, then y-halo runs of CPT cells
    static_assert((CPT == 1 || CPT == 2) && TX % CPT == 0 && NH <= kS3Threads, "z-marching tile");
    typedef C Plane[TY + 2][TX + 2];
    int n, bc, tp, ty, i, j, k0, hy, hx, hsel;
    int64_t P, col, hsrc;
    bool hw, hrun;            // this thread has a halo slot; the slot is a run of CPT cells
    C hsg;                    // sign of the slot (-1: Dirichlet ghost)
    C xm[CPT], xc[CPT], xp[CPT], hv[CPT];  // plane k: below, own, above, halo slot
    C xpp[CPT], hn[CPT];                   // prefetched for plane k + 1

    __device__ ZMarch(int lg, int bc_, int zc) : n(1 << lg), bc(bc_) {
        const int ntx = n / TX, nty = n / TY;
        const int blk = int(xcd_block(blockIdx.x, gridDim.x));
        const int t = int(threadIdx.x);
        tp = t % TP;
        ty = t / TP;
        const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
        const int x0 = bx * TX, y0 = by * TY;
        i = x0 + CPT * tp;
        j = y0 + ty;
        k0 = bz * zc;
        P = int64_t(1) << (2 * lg);
        col = (int64_t(j) << lg) + i;
        hw = t < NH;
        hrun = false;
        hy = ty + 1;
        hx = CPT * tp + 1;
        hsrc = col;
        hsel = 0;
        hsg = C(1);
        if (hw) {
            int gi, gj;
            if (t < 2 * TY) {  // x-halo cell of a row
                hy = (t >> 1) + 1;
                hx = (t & 1) ? TX + 1 : 0;
                gj = y0 + hy - 1;
                gi = (t & 1) ? x0 + TX : x0 - 1;
            } else {           // y-halo run of CPT cells
                const int u = t - 2 * TY;
                hrun = true;
                hx = CPT * (u >> 1) + 1;
                hy = (u & 1) ? TY + 1 : 0;
                gi = x0 + hx - 1;
                gj = (u & 1) ? y0 + TY : y0 - 1;
            }
            // outside the grid: wrap (periodic) or the adjacent interior cell negated (Dirichlet)
            const bool out = gi < 0 || gi >= n || gj < 0 || gj >= n;
            if (gi < 0) gi = bc ? n - 1 : 0;
            if (gi >= n) gi = bc ? 0 : n - 1;
            if (gj < 0) gj = bc ? n - 1 : 0;
            if (gj >= n) gj = bc ? 0 : n - 1;
            if (out && !bc) hsg = C(-1);
            hsel = CPT == 2 ? (gi & 1) : 0;  // single cell: which half of its aligned pair
            hsrc = (int64_t(gj) << lg) + (CPT == 2 ? (gi & ~1) : gi);
        }
    }
    // offset of the value above plane k (z + 1) in the column, and its sign
    __device__ __forceinline__ int64_t up_at(int k) const { return k < n - 1 ? (k + 1) * P : (bc ? 0 : k * P); }
    __device__ __forceinline__ C up_sg(int k) const { return (k < n - 1 || bc) ? C(1) : C(-1); }
    // next plane index, clamped to the grid (a harmless reload on the top plane)
    __device__ __forceinline__ int next(int k) const { return k + 1 < n ? k + 1 : n - 1; }

    // this thread's CPT cells at offset q (q even when CPT = 2)
    template <class V>
    __device__ __forceinline__ void cells(const V &v, int64_t q, C (&o)[CPT]) const {
        if constexpr (CPT == 2) v.pair(q, o[0], o[1]);
        else o[0] = v(q);
    }
    // this thread's halo slot on the plane at offset pk
    template <class V>
    __device__ __forceinline__ void halo(const V &v, int64_t pk, C (&o)[CPT]) const {
        if constexpr (CPT == 2) {
            C a, b;
            v.pair(pk + hsrc, a, b);
            o[0] = hsg * (hrun || !hsel ? a : b);
            o[1] = hsg * b;
        } else {
            o[0] = hsg * v(pk + hsrc);
        }
    }
    template <class V>
    __device__ __forceinline__ void start(const V &v) {
        cells(v, k0 * P + col, xc);
        if (k0 > 0) cells(v, (k0 - 1) * P + col, xm);
        else if (bc) cells(v, (n - 1) * P + col, xm);
        else
            for (int c = 0; c < CPT; ++c) xm[c] = -xc[c];
        cells(v, up_at(k0) + col, xp);
        for (int c = 0; c < CPT; ++c) xp[c] *= up_sg(k0);
        halo(v, k0 * P, hv);
    }
    // issue the loads of plane k + 1
    template <class V>
    __device__ __forceinline__ void prefetch(const V &v, int k) {
        const int kn = next(k);
        cells(v, up_at(kn) + col, xpp);
        for (int c = 0; c < CPT; ++c) xpp[c] *= up_sg(kn);
        halo(v, kn * P, hn);
    }
    // publish plane k to LDS buffer b and return, per own cell, the sum of its
    // six face neighbours in the order x-, x+, y-, y+, z-, z+.  Two buffers and
    // one barrier per plane: a thread writing a buffer again (plane k + 2) has
    // passed plane k + 1's barrier, which follows every read of plane k.
    __device__ __forceinline__ void neighbours(Plane &b, C (&s)[CPT]) const {
        for (int c = 0; c < CPT; ++c) b[ty + 1][CPT * tp + c + 1] = xc[c];
        if (hw) {
            b[hy][hx] = hv[0];
            if constexpr (CPT == 2) {
                if (hrun) b[hy][hx + 1] = hv[1];
            }
        }
        __syncthreads();
        for (int c = 0; c < CPT; ++c) {
            const int lc = CPT * tp + c + 1;
            const C t = ((b[ty + 1][lc - 1] + b[ty + 1][lc + 1]) + b[ty][lc]) + b[ty + 2][lc];
            s[c] = (t + xm[c]) + xp[c];
        }
    }
    __device__ __forceinline__ void advance() {
        for (int c = 0; c < CPT; ++c) {
            xm[c] = xc[c];
            xc[c] = xp[c];
            xp[c] = xpp[c];
            hv[c] = hn[c];
        }
    }
};

template <class S> struct LdC {
    const S *p;
    __device__ __forceinline__ typename St<S>::C operator()(int64_t q) const { return St<S>::ld(p + q); }
    __device__ __forceinline__ void pair(int64_t q, typename St<S>::C &a, typename St<S>::C &b) const {
        Pair<S>::ld(p + q, a, b);
    }
};

template <class S, int CPT>
__device__ __forceinline__ void store_cells(S *p, const typename St<S>::C (&v)[CPT]) {
    if constexpr (CPT == 2) Pair<S>::st(p, v[0], v[1]);
    else St<S>::st(p, v[0]);
}

// 3D Jacobi sweep on the z-marching tiles (same arithmetic and summation order
// as k_sweep).  NORM: per-workgroup partial of r^2.  ZERO2: the first two
// sweeps from a zero iterate (xin is not read).
template <class S, bool NORM, bool ZERO2 = false>
__global__ __launch_bounds__(kS3Threads) void k_sweep3(const S *__restrict__ f, const S *__restrict__ xin,
                                                       S *__restrict__ xout, double *__restrict__ partial, int lg,
                                                       int bc, int zc, typename St<S>::C inv_h2,
                                                       typename St<S>::C wdiag, const int *stop) {
    typedef typename St<S>::C C;
    constexpr int CPT = ZCfg<S>::CPT;
    typedef ZMarch<C, ZCfg<S>::TX, CPT> Z;
    __shared__ typename Z::Plane pl[2];
    if (stop && *stop) return;
    Z z(lg, bc, zc);
    typedef typename std::conditional<ZERO2, LdW<S>, LdC<S>>::type V;
    V v;
    if constexpr (ZERO2) v = V{f, wdiag};
    else v = V{xin};
    const LdC<S> vf{f};
    z.start(v);
    C fc[CPT], fn[CPT], s[CPT], out[CPT];
    z.cells(vf, z.k0 * z.P + z.col, fc);
    double acc = 0.0;
    for (int k = z.k0, q = 0; k < z.k0 + zc; ++k, q ^= 1) {
        z.prefetch(v, k);
        z.cells(vf, z.next(k) * z.P + z.col, fn);
        z.neighbours(pl[q], s);
        for (int c = 0; c < CPT; ++c) {
            const C r = fc[c] - (C(6) * z.xc[c] - s[c]) * inv_h2;
            if (NORM) acc += double(r) * double(r);
            out[c] = z.xc[c] + wdiag * r;
            fc[c] = fn[c];
        }
        store_cells<S, CPT>(xout + k * z.P + z.col, out);
        z.advance();
    }
    if (NORM) {
        acc = block_sum_n<kS3Threads>(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// Residual + restriction on the z-marching tiles: each thread sums the
// residuals of its cells over a pair of planes (with CPT = 2, its own x-pair
// of cells too), then one thread per coarse cell adds the pair sums of the
// other children (through LDS) and writes the coarse cell, 2^-3 times the sum
// of its eight children.  zc even.
template <class S>
__global__ __launch_bounds__(kS3Threads) void k_restrict3(const S *__restrict__ f, const S *__restrict__ x,
                                                          S *__restrict__ fc, int lg, int bc, int zc,
                                                          typename St<S>::C inv_h2, const int *stop) {
    typedef typename St<S>::C C;
    constexpr int CPT = ZCfg<S>::CPT, TX = ZCfg<S>::TX;
    typedef ZMarch<C, TX, CPT> Z;
    __shared__ typename Z::Plane pl[2];
    __shared__ C rs[Z::TY][Z::TP];
    if (stop && *stop) return;
    Z z(lg, bc, zc);
    const LdC<S> v{x}, vf{f};
    z.start(v);
    const int lgc = lg - 1;
    C f0[CPT], fn[CPT], s[CPT];
    z.cells(vf, z.k0 * z.P + z.col, f0);
    C pair = C(0);
    for (int k = z.k0, q = 0; k < z.k0 + zc; ++k, q ^= 1) {
        z.prefetch(v, k);
        z.cells(vf, z.next(k) * z.P + z.col, fn);
        z.neighbours(pl[q], s);
        C r = f0[0] - (C(6) * z.xc[0] - s[0]) * inv_h2;
        if constexpr (CPT == 2) r += f0[1] - (C(6) * z.xc[1] - s[1]) * inv_h2;
        if (((k - z.k0) & 1) == 0) {
            pair = r;
        } else {
            pair += r;
            rs[z.ty][z.tp] = pair;
            __syncthreads();
            if constexpr (CPT == 2) {
                if ((z.ty & 1) == 0) {
                    const C t = rs[z.ty][z.tp] + rs[z.ty + 1][z.tp];
                    const int64_t cc = ((int64_t(k >> 1) << (2 * lgc)) | (int64_t(z.j >> 1) << lgc)) + (z.i >> 1);
                    St<S>::st(fc + cc, t * C(0.125));
                }
            } else {
                if (((z.tp | z.ty) & 1) == 0) {
                    const C t = ((rs[z.ty][z.tp] + rs[z.ty][z.tp + 1]) + rs[z.ty + 1][z.tp]) + rs[z.ty + 1][z.tp + 1];
                    const int64_t cc = ((int64_t(k >> 1) << (2 * lgc)) | (int64_t(z.j >> 1) << lgc)) + (z.i >> 1);
                    St<S>::st(fc + cc, t * C(0.125));
                }
            }
            // rs is written again two planes later, after plane k + 1's barrier
        }
        z.advance();
        for (int c = 0; c < CPT; ++c) f0[c] = fn[c];
    }
}

// Refinement step of the mixed path on the z-marching tiles (see
// k_ir_resid): x_out = x + e (HAS_E; else x_out is not written and e is not
// read), r = f - A x_out in FP64, r_lo = r rounded, per-workgroup partial of
// r^2.  CPT cells per thread along x: 1, or 2 (16-byte FP64 and paired
// low-precision accesses; the same arithmetic per cell).  XZ: x is zero and
// not read (x_out = 0 + e, the first update of a solve from a zero iterate).
template <class SL, bool HAS_E, int CPT = 1, bool XZ = false>
__global__ __launch_bounds__(kS3Threads) void k_ir_resid3(const double *__restrict__ x, const SL *__restrict__ e,
                                                          double *__restrict__ xout, const double *__restrict__ f,
                                                          SL *__restrict__ rlo, double *__restrict__ partial,
                                                          int lg, int bc, int zc, double inv_h2,
                                                          const int *stop) {
    typedef ZMarch<double, ZCfg<double>::TX, CPT> Z;
    typedef typename St<SL>::C CL;
    __shared__ typename Z::Plane pl[2];
    if (stop && *stop) return;
    Z z(lg, bc, zc);
    struct {
        const double *x;
        const SL *e;
        __device__ __forceinline__ double operator()(int64_t q) const {
            const double xq = XZ ? 0.0 : x[q];
            return HAS_E ? xq + double(St<SL>::ld(e + q)) : xq;
        }
        __device__ __forceinline__ void pair(int64_t q, double &a, double &b) const {
            if (XZ) a = b = 0.0;
            else Pair<double>::ld(x + q, a, b);
            if (HAS_E) {
                CL ea, eb;
                Pair<SL>::ld(e + q, ea, eb);
                a = a + double(ea);
                b = b + double(eb);
            }
        }
    } v{x, e};
    const LdC<double> vf{f};
    z.start(v);
    double fc[CPT], fn[CPT], s[CPT];
    z.cells(vf, z.k0 * z.P + z.col, fc);
    double acc = 0.0;
    for (int k = z.k0, q = 0; k < z.k0 + zc; ++k, q ^= 1) {
        z.prefetch(v, k);
        z.cells(vf, z.next(k) * z.P + z.col, fn);
        z.neighbours(pl[q], s);
        const int64_t c = k * z.P + z.col;
        CL rl[CPT];
        for (int i = 0; i < CPT; ++i) {
            const double r = fc[i] - (6.0 * z.xc[i] - s[i]) * inv_h2;
            rl[i] = CL(r);
            acc += r * r;
            fc[i] = fn[i];
        }
        if (HAS_E) store_cells<double, CPT>(xout + c, z.xc);
        store_cells<SL, CPT>(rlo + c, rl);
        z.advance();
    }
    acc = block_sum_n<kS3Threads>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// x += P ec on the z-marching tiles (fine level lg, n >= TX).  The workgroup
// keeps the coarse planes K-1, K, K+1 of its tile (with a one-cell halo,
// ghost values already carrying the boundary rule: wrapped, or the adjacent
// interior cell negated per axis for Dirichlet) in an LDS ring; each thread
// updates its CPT columns on fine planes 2K and 2K+1 from LDS values, while
// the coarse plane K+2 is in flight (one coarse cell per thread, clamped
// loads).  Weights 3/4 (own coarse cell) and 1/4 (neighbour) per axis.
// Cell-centred trilinear prolongation on the z-marching tiles (shared by the
// prolongation kernel and the fused prolongation + sweep, so that both do the
// same arithmetic).  A thread t < CX * CY holds one cell of the tile's coarse
// footprint (its coarse cells and a one-cell ring); load(K) is that cell's
// value on coarse plane K, for K in [-2, nc + 1]: outside the grid the wrapped
// value (periodic) or the adjacent interior value negated (Dirichlet), per axis.
template <class S, int CX, int CY>
struct CTile {
    typedef typename St<S>::C C;
    const S *ec;
    int nc, bc, cx, cy;
    bool cw;
    int64_t csrc, Pc;
    C csg;
    __device__ CTile(const S *ec_, int lgc, int bc_, int x0, int y0) : ec(ec_), nc(1 << lgc), bc(bc_) {
        const int t = int(threadIdx.x);
        cw = t < CX * CY;
        cx = t % CX;
        cy = t / CX;
        int gi = (x0 >> 1) - 1 + cx, gj = (y0 >> 1) - 1 + cy;
        csg = C(1);
        if (gi < 0) { gi = bc ? nc - 1 : 0; if (!bc) csg = -csg; }
        if (gi >= nc) { gi = bc ? 0 : nc - 1; if (!bc) csg = -csg; }
        if (gj < 0) { gj = bc ? nc - 1 : 0; if (!bc) csg = -csg; }
        if (gj >= nc) { gj = bc ? 0 : nc - 1; if (!bc) csg = -csg; }
        csrc = cw ? (int64_t(gj) << lgc) + gi : 0;
        Pc = int64_t(1) << (2 * lgc);
    }
    __device__ __forceinline__ C load(int K) const {
        C sg = csg;
        int kk = K;
        if (kk < 0) { kk = bc ? nc - 1 : 0; if (!bc) sg = -sg; }
        if (kk >= nc) { kk = bc ? 0 : nc - 1; if (!bc) sg = -sg; }
        return sg * St<S>::ld(ec + kk * Pc + csrc);
    }
};

// Weighted pair 3/4 a + 1/4 b with one rounding (b / 4 is exact): written as an
// explicit fused multiply-add so that every kernel that prolongates rounds the
// same way whatever the compiler's contraction choices.
__device__ __forceinline__ float wpair(float a, float b) { return __builtin_fmaf(0.75f, a, 0.25f * b); }
__device__ __forceinline__ double wpair(double a, double b) { return __builtin_fma(0.75, a, 0.25 * b); }

// In-plane bilinear value of a coarse plane tile at a fine column: own coarse
// row / column (ly, lx) weighted 3/4, the neighbour on the fine cell's side
// (ny, nx) 1/4, x first.
template <class C, int CY, int CX>
__device__ __forceinline__ C prolong_bil(const C (&pl)[CY][CX], int ly, int ny, int lx, int nx) {
    return wpair(wpair(pl[ly][lx], pl[ly][nx]), wpair(pl[ny][lx], pl[ny][nx]));
}
// The prolongated value from the own coarse plane's and the neighbour plane's bilinear values.
template <class C>
__device__ __forceinline__ C prolong_mix(C eo, C en) {
    return wpair(eo, en);
}

template <class S, int TX = ZCfg<S>::TX>
__global__ __launch_bounds__(kS3Threads) void k_prolong3(const S *__restrict__ ec, S *__restrict__ x, int lg, int bc,
                                                         int zc, const int *stop) {
    typedef typename St<S>::C C;
    constexpr int CPT = ZCfg<S>::CPT, TP = TX / CPT;
    constexpr int TY = kS3Threads / TP, CX = TX / 2 + 2, CY = TY / 2 + 2;
    static_assert(CX * CY <= kS3Threads, "one coarse cell per thread");
    __shared__ C cp[3][CY][CX];
    if (stop && *stop) return;
    const int n = 1 << lg, lgc = lg - 1, ntx = n / TX, nty = n / TY;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP;
    const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
    const int x0 = bx * TX, y0 = by * TY, k0 = bz * zc, K0 = k0 >> 1;
    const int64_t P = int64_t(1) << (2 * lg), col = (int64_t(y0 + ty) << lg) + x0 + CPT * tp;
    const CTile<S, CX, CY> ct(ec, lgc, bc, x0, y0);
    const bool cw = ct.cw;
    const int cx = ct.cx, cy = ct.cy;
    auto cload = [&](int K) -> C { return ct.load(K); };
    auto slot = [](int K) { return (K + 3) % 3; };
    {
        const C a = cload(K0 - 1), b = cload(K0), c = cload(K0 + 1);
        if (cw) {
            cp[slot(K0 - 1)][cy][cx] = a;
            cp[slot(K0)][cy][cx] = b;
            cp[slot(K0 + 1)][cy][cx] = c;
        }
    }
    __syncthreads();
    // per own cell: own coarse column and row in the tile and the neighbour side per axis
    int lx[CPT], nx[CPT];
    for (int c = 0; c < CPT; ++c) {
        const int ti = CPT * tp + c;  // cell index within the tile row
        lx[c] = (ti >> 1) + 1;
        nx[c] = lx[c] + ((ti & 1) ? 1 : -1);
    }
    const int ly = (ty >> 1) + 1, ny = ly + ((ty & 1) ? 1 : -1);
    const LdC<S> vx{x};
    for (int K = K0; K < K0 + (zc >> 1); ++K) {
        const int64_t c0 = int64_t(2 * K) * P + col, c1 = c0 + P;
        C xa[CPT], xb[CPT];
        if constexpr (CPT == 2) {
            vx.pair(c0, xa[0], xa[1]);
            vx.pair(c1, xb[0], xb[1]);
        } else {
            xa[0] = vx(c0);
            xb[0] = vx(c1);
        }
        const C nxt = cload(K + 2);  // ring slot of K - 1 after this plane pair
        const C(&own)[CY][CX] = cp[slot(K)];
        const C(&below)[CY][CX] = cp[slot(K - 1)];
        const C(&above)[CY][CX] = cp[slot(K + 1)];
        for (int c = 0; c < CPT; ++c) {
            const C eo = prolong_bil(own, ly, ny, lx[c], nx[c]), em = prolong_bil(below, ly, ny, lx[c], nx[c]),
                    ep = prolong_bil(above, ly, ny, lx[c], nx[c]);
            xa[c] = xa[c] + prolong_mix(eo, em);  // fine plane 2K: neighbour plane K - 1
            xb[c] = xb[c] + prolong_mix(eo, ep);  // fine plane 2K + 1: neighbour plane K + 1
        }
        store_cells<S, CPT>(x + c0, xa);
        store_cells<S, CPT>(x + c1, xb);
        __syncthreads();  // every read of slot(K - 1) is done
        if (cw) cp[slot(K + 2)][cy][cx] = nxt;
        __syncthreads();
    }
}

// Prolongation + correction of a level followed by its first Jacobi sweep, in
// one z-marching pass: xout = sweep(xin + P ec), the corrected iterate never
// stored.  Every value the sweep reads (own columns at z-1, z, z+1 and the
// in-plane halo) is corrected where it is loaded, from a ring of four coarse
// planes (with the tile's coarse ring) in LDS, and rounded to the storage
// precision as the stored iterate of the two-kernel path is: the result equals
// k_prolong3 then k_sweep3 bit for bit.  Ghost values are corrected at the
// ghost position from the coarse ghosts; by the symmetry of the cell-centred
// weights that is the ghost of the corrected value exactly (negated for
// Dirichlet, wrapped for periodic).  zc even.  TX: tile width (n >= TX; 128
// on the large levels, 64 and 32 on the 64^3 and 32^3 levels).
template <class S, int TX = ZCfg<S>::TX>
__global__ __launch_bounds__(kS3Threads) void k_psweep3(const S *__restrict__ ec, const S *__restrict__ f,
                                                        const S *__restrict__ xin, S *__restrict__ xout, int lg,
                                                        int bc, int zc, typename St<S>::C inv_h2,
                                                        typename St<S>::C wdiag, const int *stop) {
    typedef typename St<S>::C C;
    constexpr int CPT = ZCfg<S>::CPT;
    typedef ZMarch<C, TX, CPT> Z;
    constexpr int CX = TX / 2 + 2, CY = Z::TY / 2 + 2;
    static_assert(CX * CY <= kS3Threads, "one coarse cell per thread");
    __shared__ typename Z::Plane pl[2];
    __shared__ C cp[4][CY][CX];
    if (stop && *stop) return;
    Z z(lg, bc, zc);
    const CTile<S, CX, CY> ct(ec, lg - 1, bc, z.i - CPT * z.tp, z.j - z.ty);
    auto cs = [](int K) { return (K + 4) & 3; };  // ring slot of coarse plane K >= -2
    // corrected value at fine position (fx, fy) of the tile (ghost frame, the ring
    // at -1 and TX / TY) on fine plane p in [-1, n]
    auto corr = [&](C raw, int fx, int fy, int p) -> C {
        const int lx = (fx + 2) >> 1, nx = lx + ((fx & 1) ? 1 : -1);
        const int ly = (fy + 2) >> 1, ny = ly + ((fy & 1) ? 1 : -1);
        const int K = ((p + 2) >> 1) - 1, Kn = K + ((p & 1) ? 1 : -1);
        const C eo = prolong_bil(cp[cs(K)], ly, ny, lx, nx), en = prolong_bil(cp[cs(Kn)], ly, ny, lx, nx);
        return st_round<S>(raw + prolong_mix(eo, en));
    };
    auto corr_cells = [&](C (&v)[CPT], int p) {
        for (int c = 0; c < CPT; ++c) v[c] = corr(v[c], CPT * z.tp + c, z.ty, p);
    };
    // In the loop a correction is prolong_mix of two coarse planes' in-plane values
    // at the cell.  For the own columns each coarse plane's values are formed once
    // and kept (oa, ob) for the fine planes that use them; the halo slot's are
    // formed per plane (keeping them too costs occupancy, measured slower).
    const int oly = (z.ty + 2) >> 1, ony = oly + ((z.ty & 1) ? 1 : -1);
    const int hly = (z.hy + 1) >> 1, hny = hly + ((z.hy & 1) ? -1 : 1);  // fy = hy - 1
    int olx[CPT], onx[CPT], hlx[CPT], hnx[CPT];
    for (int c = 0; c < CPT; ++c) {
        const int fx = CPT * z.tp + c, gx = z.hx - 1 + c;
        olx[c] = (fx + 2) >> 1;
        onx[c] = olx[c] + ((fx & 1) ? 1 : -1);
        hlx[c] = (gx + 2) >> 1;
        hnx[c] = hlx[c] + ((gx & 1) ? 1 : -1);
    }
    auto bil_own = [&](int K, C (&e)[CPT]) {
        for (int c = 0; c < CPT; ++c) e[c] = prolong_bil(cp[cs(K)], oly, ony, olx[c], onx[c]);
    };
    auto bil_halo = [&](int K, C (&e)[CPT]) {
        if (!z.hw) return;  // no slot: the value is not used
        // a single-cell slot has only its first cell (the second's columns may lie off the tile)
        for (int c = 0; c < CPT; ++c)
            e[c] = c == 0 || z.hrun ? prolong_bil(cp[cs(K)], hly, hny, hlx[c], hnx[c]) : C(0);
    };
    auto mix_cells = [&](C (&v)[CPT], const C (&eo)[CPT], const C (&en)[CPT]) {
        for (int c = 0; c < CPT; ++c) v[c] = st_round<S>(v[c] + prolong_mix(eo[c], en[c]));
    };
    auto mix_halo = [&](C (&v)[CPT], const C (&eo)[CPT], const C (&en)[CPT]) {
        if (!z.hw) return;
        v[0] = st_round<S>(v[0] + prolong_mix(eo[0], en[0]));
        if constexpr (CPT == 2) {
            if (z.hrun) v[1] = st_round<S>(v[1] + prolong_mix(eo[1], en[1]));
        }
    };
    const LdC<S> vx{xin}, vf{f};
    const int K0 = z.k0 >> 1;
    {
        const C a = ct.load(K0 - 1), b = ct.load(K0), c = ct.load(K0 + 1);
        if (ct.cw) {
            cp[cs(K0 - 1)][ct.cy][ct.cx] = a;
            cp[cs(K0)][ct.cy][ct.cx] = b;
            cp[cs(K0 + 1)][ct.cy][ct.cx] = c;
        }
    }
    z.start(vx);
    __syncthreads();
    corr_cells(z.xm, z.k0 - 1);
    corr_cells(z.xc, z.k0);
    // own columns: planes J, J + 1 (J = k / 2); the halo slot's values are formed per plane
    C oa[CPT], ob[CPT];
    bil_own(K0, oa);
    bil_own(K0 + 1, ob);
    auto fix_halo = [&](int Ko, int Kn) {
        if (!z.hw) return;
        C ho[CPT], hn2[CPT];
        bil_halo(Ko, ho);
        bil_halo(Kn, hn2);
        mix_halo(z.hv, ho, hn2);
    };
    C fc[CPT], fn[CPT], s[CPT], out[CPT];
    z.cells(vf, z.k0 * z.P + z.col, fc);
    C cnext = C(0);
    // one fine plane: loads of the next, the corrections `fix` of the values loaded one
    // plane ago (after the new loads are issued, so that they stay in flight),
    // neighbours (one barrier), sweep and store
    auto plane = [&](int k, int q, auto &&fix) {
        z.prefetch(vx, k);
        z.cells(vf, z.next(k) * z.P + z.col, fn);
        fix();
        // coarse plane J + 2 is loaded on plane 2J and published on plane 2J + 1 (first read
        // at the start of plane 2J + 2); its slot held plane J - 2, last read on plane 2J - 2
        if ((k & 1) == 0) cnext = ct.load((k >> 1) + 2);
        else if (ct.cw) cp[cs((k >> 1) + 2)][ct.cy][ct.cx] = cnext;
        z.neighbours(pl[q], s);
        for (int c = 0; c < CPT; ++c) {
            const C r = fc[c] - (C(6) * z.xc[c] - s[c]) * inv_h2;
            out[c] = z.xc[c] + wdiag * r;
            fc[c] = fn[c];
        }
        store_cells<S, CPT>(xout + k * z.P + z.col, out);
        z.advance();
    };
    for (int k = z.k0; k < z.k0 + zc; k += 2) {
        const int J = k >> 1;
        // plane 2J: halo of 2J (own J, neighbour J - 1); column value of 2J + 1 (J, J + 1)
        plane(k, 0, [&] {
            fix_halo(J, J - 1);
            mix_cells(z.xp, oa, ob);
        });
        // plane 2J + 1: halo of 2J + 1 (J, J + 1); column value of 2J + 2 (J + 1, J)
        plane(k + 1, 1, [&] {
            fix_halo(J, J + 1);
            mix_cells(z.xp, ob, oa);
        });
        // slide to J + 1: coarse plane J + 2 was published on plane 2J + 1
        for (int c = 0; c < CPT; ++c) oa[c] = ob[c];
        bil_own(J + 2, ob);
    }
}

// Planes per workgroup of the z-marching kernels on an n^3 level with `cpt`
// cells per thread: enough workgroups to fill the chip, and at most
// `max_blocks` of them (one norm partial each).
inline int sweep3_planes(int lg, int cpt, int64_t max_blocks) {
    const int n = 1 << lg;
    const int64_t cols = int64_t(n) * n / (int64_t(kS3Threads) * cpt);  // column tiles
    // measured: 16 planes beat 8 at 256^3 in every precision; levels below 128^3 are
    // launch-bound and take the shortest chains (two planes)
    int zc = n >= 256 ? 16 : (n >= 128 ? 4 : 2);
    if (g_zc3 >= 2 && g_zc3 <= n) zc = g_zc3;  // tuning knob "zc3" (a power of two)
    while (cols * (n / zc) > max_blocks && zc < n) zc *= 2;
    return zc;
}

// Workgroups of a z-marching launch on an n^3 level (cpt cells per thread, zc planes).
inline unsigned zblocks(int lg, int cpt, int zc) {
    return unsigned((int64_t(1) << (3 * lg)) / (int64_t(kS3Threads) * cpt * zc));
}

// Fine cells per workgroup along x in k_restrict.
template <int D> struct RBlk {
    static constexpr int FX = D == 3 ? 64 : 128;
};

template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_restrict(const S *__restrict__ f, const S *__restrict__ x,
                                                     S *__restrict__ fc, int lg, int bc,
                                                     typename St<S>::C inv_h2, const int *stop) {
    typedef typename St<S>::C C;
    constexpr int FX = RBlk<D>::FX;
    __shared__ C r[kBlock];
    if (stop && *stop) return;
    const int n = 1 << lg, nc = n >> 1, tid = threadIdx.x;
    const int bxn = n / FX;
    // workgroup -> (x block, coarse row J, coarse plane K)
    const int b = int(sizeof(S) < 8 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x);
    const int bx = b % bxn, J = (b / bxn) % nc, K = D == 3 ? b / (bxn * nc) : 0;
    const int a = tid % FX, yb = (tid / FX) & 1, zb = D == 3 ? tid / (2 * FX) : 0;
    const int i = bx * FX + a, j = 2 * J + yb, k = D == 3 ? 2 * K + zb : 0;
    const int64_t c = (int64_t(k) << (2 * lg)) | (int64_t(j) << lg) | i;
    r[tid] = resid_at<D, S>(f, x, c, i, j, k, lg, bc, inv_h2);
    __syncthreads();
    if (tid < FX / 2) {
        C acc = C(0);
        for (int cz = 0; cz < (D == 3 ? 2 : 1); ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) acc += r[(cz * 2 + cy) * FX + 2 * tid + cx];
        const int I = bx * (FX / 2) + tid;
        St<S>::st(fc + ((int64_t(K) * nc + J) * nc + I), acc * C(D == 3 ? 0.125 : 0.25));
    }
}

// ------------------------------------------------------------- coarse tail
template <int D> struct Tail {
    static constexpr int LG = D == 3 ? 4 : 6;  // finest level handled: 16^3 / 64^2
    static constexpr int64_t cells(int lg) { return int64_t(1) << (D * lg); }
    static constexpr int64_t levels_sum() {
        int64_t s = 0;
        for (int l = LG; l >= 2; --l) s += cells(l);
        return s;
    }
    // threads (2D 512: the 128^2 solve measured 0.571 -> 0.552 ms against 1024; 3D 512 no
    // faster, 256 slower); NT_B: the batched solver's 2D tail, one workgroup per problem
    static constexpr int NT = D == 3 ? 1024 : 512;
    static constexpr int NT_B = 1024;
    // threads of the advection-diffusion tail (3D measured slower with 1024: 19.3 against 17.3 us)
    static constexpr int NT_AD = D == 3 ? 512 : 1024;
};

// nb_sum for a level held in LDS, without branches: every neighbour is read
// unconditionally (a Dirichlet ghost reads the cell itself and flips its sign,
// a periodic one reads the wrapped cell), so the six reads are in flight
// together.  Same values and summation order as nb_sum.
template <int D, class C>
__device__ __forceinline__ C nb_sum_lds(const C *X, int c, int i, int j, int k, int lg, int bc) {
    const int last = (1 << lg) - 1, sy = 1 << lg, sz = 1 << (2 * lg);
    const bool per = bc != 0;
    const C xm = X[i > 0 ? c - 1 : (per ? c + last : c)];
    const C xp = X[i < last ? c + 1 : (per ? c - last : c)];
    const C ym = X[j > 0 ? c - sy : (per ? c + last * sy : c)];
    const C yp = X[j < last ? c + sy : (per ? c - last * sy : c)];
    C s = (((i > 0 || per) ? xm : -xm) + ((i < last || per) ? xp : -xp) + ((j > 0 || per) ? ym : -ym)) +
          ((j < last || per) ? yp : -yp);
    if (D == 3) {
        const C zm = X[k > 0 ? c - sz : (per ? c + last * sz : c)];
        const C zp = X[k < last ? c + sz : (per ? c - last * sz : c)];
        s = (s + ((k > 0 || per) ? zm : -zm)) + ((k < last || per) ? zp : -zp);
    }
    return s;
}

// One weighted-Jacobi sweep T = X + wdiag (F - A X) (RESID: the residual
// T = F - A X) of a level of the one-workgroup tail (all three in LDS).  Each thread marches along the last
// axis over a run of one column's cells: the neighbours along that axis come
// from registers, the in-plane ones from offsets fixed per column.  Same
// values and summation order as nb_sum.  Needs n^(D-1) <= NT.
template <int D, class C, int NT, bool RESID = false, bool ZERO2 = false>
__device__ __forceinline__ void tail_sweep(const C *__restrict__ X, const C *__restrict__ F, C *__restrict__ T,
                                           int lg, int bc, C inv_h2, C wdiag) {
    // ZERO2: the sweep after a first one from zero; its input iterate w f is formed from F (X unused)
    auto xv = [&](int q) -> C { return ZERO2 ? wdiag * F[q] : X[q]; };
    const int n = 1 << lg, last = n - 1, sm = D == 3 ? n * n : n;  // sm: cells per plane = marching stride
    const int chunks = NT / sm < n ? NT / sm : n, len = n / chunks;
    const int t = threadIdx.x;
    if (t < sm * chunks) {
        const bool per = bc != 0;
        const int i = t & last, j = D == 3 ? (t >> lg) & last : 0, z0 = (t / sm) * len;
        const int oxm = i > 0 ? -1 : (per ? last : 0), oxp = i < last ? 1 : (per ? -last : 0);
        const bool fxm = i > 0 || per, fxp = i < last || per;
        const int oym = j > 0 ? -n : (per ? last * n : 0), oyp = j < last ? n : (per ? -last * n : 0);
        const bool fym = j > 0 || per, fyp = j < last || per;
        int c = z0 * sm + (t & (sm - 1));
        C xc = xv(c);
        C zm = xv(z0 > 0 ? c - sm : (per ? c + last * sm : c));
        bool fzm = z0 > 0 || per;
        for (int z = z0; z < z0 + len; ++z, c += sm) {
            const C zp = xv(z < last ? c + sm : (per ? c - last * sm : c));
            const bool fzp = z < last || per;
            const C xm = xv(c + oxm), xp = xv(c + oxp);
            C s = (fxm ? xm : -xc) + (fxp ? xp : -xc);
            if (D == 3) {
                const C ym = xv(c + oym), yp = xv(c + oyp);
                s = (s + (fym ? ym : -xc)) + (fyp ? yp : -xc);
            }
            s = (s + (fzm ? zm : -xc)) + (fzp ? zp : -xc);
            if (RESID) T[c] = F[c] - (C(2 * D) * xc - s) * inv_h2;  // the residual only
            else T[c] = xc + wdiag * (F[c] - (C(2 * D) * xc - s) * inv_h2);
            zm = xc;
            fzm = true;
            xc = zp;
        }
    }
}

// X += P E on a level of the one-workgroup tail (E: the next coarser level),
// marching like tail_sweep: the in-plane interpolation indices and signs are
// fixed per column.  Same terms and summation order as k_prolong_add.
template <int D, class C, int NT>
__device__ __forceinline__ void tail_prolong(const C *__restrict__ E, C *__restrict__ X, int lg, int bc) {
    const int n = 1 << lg, last = n - 1, lgc = lg - 1, nc = n >> 1, sm = D == 3 ? n * n : n;
    const int chunks = NT / sm < n ? NT / sm : n, len = n / chunks;
    const int t = threadIdx.x;
    if (t < sm * chunks) {
        const int z0 = (t / sm) * len;
        int oi, ni, oj = 0, nj = 0;
        float si, sj = 1.0f;
        pro_axis(t & last, nc, bc, oi, ni, si);
        if (D == 3) pro_axis((t >> lg) & last, nc, bc, oj, nj, sj);
        int c = z0 * sm + (t & (sm - 1));
        for (int z = z0; z < z0 + len; ++z, c += sm) {
            int oz, nz;
            float sz;
            pro_axis(z, nc, bc, oz, nz, sz);
            C s = C(0);
            if (D == 3) {
                for (int cz = 0; cz < 2; ++cz)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const C w = C(a ? 0.25 : 0.75) * C(b ? 0.25 : 0.75) * C(cz ? 0.25 : 0.75);
                            const C sg = C((a ? si : 1.0f) * (b ? sj : 1.0f) * (cz ? sz : 1.0f));
                            const int q = ((cz ? nz : oz) << (2 * lgc)) | ((b ? nj : oj) << lgc) | (a ? ni : oi);
                            s = np_fma(w, sg * E[q], s);
                        }
            } else {
                // the marching axis is y
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        const C w = C(a ? 0.25 : 0.75) * C(b ? 0.25 : 0.75) * C(1.0);
                        const C sg = C((a ? si : 1.0f) * (b ? sz : 1.0f) * 1.0f);
                        const int q = ((b ? nz : oz) << lgc) | (a ? ni : oi);
                        s = np_fma(w, sg * E[q], s);
                    }
            }
            X[c] = X[c] + s;
        }
    }
}

// V(nu1, nu2) cycle on levels lg_t .. 2 in one workgroup, every level in LDS
// (xs, fs: all levels, finest first; ts: scratch of the finest level).
// f_t: right-hand side of level lg_t (global); x_t: result (global); x_in:
// starting iterate of level lg_t (global), or null for a zero iterate (then
// the first sweep is w f).  Coarser levels always start from zero.
// h_t: spacing of level lg_t.  nu1 >= 1 when x_in is null.  Entry (i, q) of
// the coarsest inverse sits at Minv[i * m_rs + q * m_cs].
template <int D, class S, int NT>
__device__ __forceinline__ void tail_cycle(typename St<S>::C *xs, typename St<S>::C *fs, typename St<S>::C *ts,
                                           const S *__restrict__ f_t, S *__restrict__ x_t,
                                           const S *__restrict__ x_in, const double *__restrict__ Minv, int lg_t,
                                           int bc, double h_t, double omega, int nu1, int nu2,
                                           int m_rs = D == 3 ? 64 : 16, int m_cs = 1) {
    typedef typename St<S>::C C;
    const int tid = threadIdx.x;
    // level l starts after the finer levels lg_t .. l+1 (geometric sum)
    auto off = [&](int l) -> int64_t {
        return ((int64_t(1) << (D * (lg_t + 1))) - (int64_t(1) << (D * (l + 1)))) / ((int64_t(1) << D) - 1);
    };
    // cnt sweeps on level lg, alternating between X and ts; the result ends in X
    auto sweeps = [&](C *X, const C *F, int lg, C inv_h2, C wdiag, int cnt) {
        C *cur = X, *nxt = ts;
        for (int it = 0; it < cnt; ++it) {
            tail_sweep<D, C, NT>(cur, F, nxt, lg, bc, inv_h2, wdiag);
            __syncthreads();
            C *t = cur;
            cur = nxt;
            nxt = t;
        }
        if (cur != X) {
            const int m = 1 << (D * lg);
            for (int c = tid; c < m; c += NT) X[c] = cur[c];
            __syncthreads();
        }
    };
    static_assert(Tail<D>::cells(Tail<D>::LG) >> Tail<D>::LG <= NT, "tail_sweep needs n^(D-1) <= NT");
    const int64_t mt = int64_t(1) << (D * lg_t);
    {
        // all of this thread's loads first, then the LDS stores: one round trip to memory
        constexpr int per = int((Tail<D>::cells(Tail<D>::LG) + NT - 1) / NT);
        C fv[per], xv[per];
#pragma unroll
        for (int u = 0; u < per; ++u) {
            const int c = tid + u * NT;
            if (c < mt) {
                fv[u] = St<S>::ld(f_t + c);
                if (x_in) xv[u] = St<S>::ld(x_in + c);
            }
        }
#pragma unroll
        for (int u = 0; u < per; ++u) {
            const int c = tid + u * NT;
            if (c < mt) {
                fs[off(lg_t) + c] = fv[u];
                if (x_in) xs[off(lg_t) + c] = xv[u];
            }
        }
    }
    __syncthreads();
    double h = h_t;
    // ------------------------------------------------------------- down
    for (int lg = lg_t; lg > 2; --lg, h *= 2.0) {
        const int64_t m = int64_t(1) << (D * lg);
        C *X = xs + off(lg), *F = fs + off(lg);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        int it0 = 0;
        if (!(x_in && lg == lg_t)) {
            if (nu1 >= 2) {
                // the first two sweeps from zero in one pass, straight into X
                tail_sweep<D, C, NT, false, true>(F, F, X, lg, bc, inv_h2, wdiag);
                __syncthreads();
                it0 = 2;
            } else {
                // first sweep from zero
                for (int64_t c = tid; c < m; c += NT) X[c] = wdiag * F[c];
                __syncthreads();
                it0 = 1;
            }
        }
        sweeps(X, F, lg, inv_h2, wdiag, nu1 - it0);
        // residual into ts, then its 2^d-cell average into the next level's rhs
        tail_sweep<D, C, NT, true>(X, F, ts, lg, bc, inv_h2, wdiag);
        __syncthreads();
        const int lgc = lg - 1;
        const int mc = 1 << (D * lgc);
        C *Fc = fs + off(lgc);
        for (int cc = tid; cc < mc; cc += NT) {
            int I, J, K;
            decode<D>(cc, lgc, I, J, K);
            C acc = C(0);
            for (int kk = 0; kk < (D == 3 ? 2 : 1); ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii) {
                        const int i = 2 * I + ii, j = 2 * J + jj, k = D == 3 ? 2 * K + kk : 0;
                        acc += ts[(k << (2 * lg)) | (j << lg) | i];
                    }
            Fc[cc] = acc * C(D == 3 ? 0.125 : 0.25);
        }
        __syncthreads();
    }
    // ------------------------------------------------- coarsest (zero guess)
    {
        constexpr int m = D == 3 ? 64 : 16;
        C *X = xs + off(2), *F = fs + off(2);
        if (lg_t == 2) {
            // the whole grid is the coarsest: x <- x + Minv (f - A x)
            __shared__ double rr[m];
            if (tid < m) {
                int i, j, k;
                decode<D>(tid, 2, i, j, k);
                const double xc = x_in ? double(X[tid]) : 0.0;
                double s = 0.0;
                if (x_in) s = double(nb_sum_lds<D, C>(X, tid, i, j, k, 2, bc));
                rr[tid] = double(F[tid]) - (double(2 * D) * xc - s) / (h * h);
            }
            __syncthreads();
            if (tid < m) {
                double acc = 0.0;
                for (int q = 0; q < m; ++q) acc += Minv[tid * m_rs + q * m_cs] * rr[q];
                X[tid] = C((x_in ? double(X[tid]) : 0.0) + acc);
            }
        } else if (tid < m) {
            double acc = 0.0;
            for (int q = 0; q < m; ++q) acc += Minv[tid * m_rs + q * m_cs] * double(F[q]);
            X[tid] = C(0.0 + acc);
        }
        __syncthreads();
    }
    // --------------------------------------------------------------- up
    for (int lg = 3; lg <= lg_t; ++lg) {
        h *= 0.5;
        const int lgc = lg - 1;
        C *X = xs + off(lg), *F = fs + off(lg), *E = xs + off(lgc);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        tail_prolong<D, C, NT>(E, X, lg, bc);
        __syncthreads();
        sweeps(X, F, lg, inv_h2, wdiag, nu2);
    }
    for (int64_t c = tid; c < mt; c += NT) St<S>::st(x_t + c, xs[off(lg_t) + c]);
}

// One-workgroup V-cycle from a zero iterate on levels lg_t .. 2.  ctl: first the
// cycle's convergence check on the np partials of the finest level's residual
// norm (the check of k_check), and nothing more if it stops the solve.
template <int D, class S>
__global__ __launch_bounds__(Tail<D>::NT) void k_tail(const S *__restrict__ f_t, S *__restrict__ x_t,
                                                      const double *__restrict__ Minv, int lg_t, int bc,
                                                      double h_t, double omega, int nu1, int nu2,
                                                      const int *stop, const double *__restrict__ partial,
                                                      int np, Ctl *ctl) {
    typedef typename St<S>::C C;
    __shared__ C xs[Tail<D>::levels_sum()];
    __shared__ C fs[Tail<D>::levels_sum()];
    __shared__ C ts[Tail<D>::cells(Tail<D>::LG)];
    // The coarsest inverse, staged in LDS transposed with padded rows: the loads
    // are issued with the right-hand side's (one round trip to memory, not one per
    // term of the product), and thread i reading entry (i, q) hits consecutive banks.
    constexpr int m = D == 3 ? 64 : 16, mp = m + 1;
    __shared__ double Ms[m * mp];
    if (stop && *stop) return;
    if (ctl) {
        __shared__ int halt;
        const int st = check_block<Tail<D>::NT>(partial, np, ctl);
        if (threadIdx.x == 0) halt = st;
        __syncthreads();
        if (halt) return;
    }
    for (int g = threadIdx.x; g < m * m; g += Tail<D>::NT) Ms[(g % m) * mp + g / m] = Minv[g];
    tail_cycle<D, S, Tail<D>::NT>(xs, fs, ts, f_t, x_t, nullptr, Ms, lg_t, bc, h_t, omega, nu1, nu2, 1, mp);
}

}  // namespace np
