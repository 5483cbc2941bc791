// Device kernels of the multigrid cycle (gfx950).  Included by mg.hip only.
//
// Grid of n = 2^lg cells per axis, index c = (k*n + j)*n + i, x fastest.
// Ghost rule: bc == 0 (Dirichlet-0) ghost = -(own value); bc == 1 wraps.
// The operator is A x = (2d x_c - sum of face neighbours) * inv_h2.
#pragma once

#include "np_internal.h"

namespace np {

// Sum of the 2d face neighbours of cell c = (i, j, k), read through `ld`
// (a functor index -> value); ghosts by the boundary rule.  Summation order
// x-, x+, y-, y+, z-, z+.
template <int D, class C, class L>
__device__ __forceinline__ C nb_sum(const L &ld, int64_t c, int i, int j, int k, int lg, int bc,
                                    C xc) {
    const int n = 1 << lg;
    const int64_t sy = int64_t(1) << lg;
    const C xm = i > 0 ? ld(c - 1) : (bc ? ld(c + (n - 1)) : -xc);
    const C xp = i < n - 1 ? ld(c + 1) : (bc ? ld(c - (n - 1)) : -xc);
    const C ym = j > 0 ? ld(c - sy) : (bc ? ld(c + (n - 1) * sy) : -xc);
    const C yp = j < n - 1 ? ld(c + sy) : (bc ? ld(c - (n - 1) * sy) : -xc);
    C s = ((xm + xp) + ym) + yp;
    if (D == 3) {
        const int64_t sz = int64_t(1) << (2 * lg);
        const C zm = k > 0 ? ld(c - sz) : (bc ? ld(c + (n - 1) * sz) : -xc);
        const C zp = k < n - 1 ? ld(c + sz) : (bc ? ld(c - (n - 1) * sz) : -xc);
        s = (s + zm) + zp;
    }
    return s;
}

template <class S> struct Ld {
    const S *p;
    __device__ __forceinline__ typename St<S>::C operator()(int64_t q) const { return St<S>::ld(p + q); }
};

template <int D>
__device__ __forceinline__ void decode(int64_t c, int lg, int &i, int &j, int &k) {
    const int n = 1 << lg;
    i = int(c & (n - 1));
    j = int((c >> lg) & (n - 1));
    k = D == 3 ? int(c >> (2 * lg)) : 0;
}

// r = f - A x at cell c.
template <int D, class S>
__device__ __forceinline__ typename St<S>::C resid_at(const S *__restrict__ f, const S *__restrict__ x,
                                                      int64_t c, int i, int j, int k, int lg, int bc,
                                                      typename St<S>::C inv_h2) {
    typedef typename St<S>::C C;
    const C xc = St<S>::ld(x + c);
    const C s = nb_sum<D, C>(Ld<S>{x}, c, i, j, k, lg, bc, xc);
    return St<S>::ld(f + c) - (C(2 * D) * xc - s) * inv_h2;
}

// One weighted-Jacobi sweep x_out = x_in + wdiag (f - A x_in), wdiag = omega/A_00.
// ZERO: x_in is identically zero (first sweep on a coarse level), x_out = wdiag f.
template <int D, class S, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_jacobi(const S *__restrict__ f, const S *__restrict__ xin,
                                                   S *__restrict__ xout, int lg, int bc,
                                                   typename St<S>::C inv_h2,
                                                   typename St<S>::C wdiag, const int *stop) {
    typedef typename St<S>::C C;
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const C fc = St<S>::ld(f + c);
    if (ZERO) {
        St<S>::st(xout + c, wdiag * fc);
        return;
    }
    int i, j, k;
    decode<D>(c, lg, i, j, k);
    const C xc = St<S>::ld(xin + c);
    const C s = nb_sum<D, C>(Ld<S>{xin}, c, i, j, k, lg, bc, xc);
    St<S>::st(xout + c, xc + wdiag * (fc - (C(2 * D) * xc - s) * inv_h2));
}

// fc = R (f - A x): one thread per coarse cell averages the residual of its
// 2^d children (z outer, then y, then x).  lg is the fine level's log2 size.
template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(const S *__restrict__ f,
                                                           const S *__restrict__ x,
                                                           S *__restrict__ fc, int lg, int bc,
                                                           typename St<S>::C inv_h2, const int *stop) {
    typedef typename St<S>::C C;
    if (stop && *stop) return;
    const int lgc = lg - 1;
    const int64_t mc = int64_t(1) << (D * lgc);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= mc) return;
    int I, J, K;
    decode<D>(c, lgc, I, J, K);
    C acc = C(0);
    for (int kk = 0; kk < (D == 3 ? 2 : 1); ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii) {
                const int i = 2 * I + ii, j = 2 * J + jj, k = D == 3 ? 2 * K + kk : 0;
                const int64_t cf = (int64_t(k) << (2 * lg)) | (int64_t(j) << lg) | i;
                acc += resid_at<D, S>(f, x, cf, i, j, k, lg, bc, inv_h2);
            }
    St<S>::st(fc + c, acc * C(D == 3 ? 0.125 : 0.25));
}

// Coarse index along one axis for the linear prolongation: the neighbour of
// the own coarse cell on the side of fine cell `i`, with its ghost sign.
__device__ __forceinline__ void pro_axis(int i, int nc, int bc, int &own, int &nb, float &sgn) {
    own = i >> 1;
    nb = (i & 1) ? own + 1 : own - 1;
    sgn = 1.0f;
    if (nb < 0) {
        if (bc) nb = nc - 1;
        else { nb = 0; sgn = -1.0f; }
    } else if (nb >= nc) {
        if (bc) nb = 0;
        else { nb = nc - 1; sgn = -1.0f; }
    }
}

// (P ec) at fine cell (i, j, k), lgc the coarse level's log2 size.  Per axis
// the own coarse cell has weight 3/4 and the neighbour 1/4; ghost neighbours
// carry the sign of the boundary rule.  The 2^D terms in a fixed order, each
// accumulated with one explicit fused multiply-add.
template <int D, class S>
__device__ __forceinline__ typename St<S>::C pro_cell(const S *__restrict__ ec, int i, int j, int k, int lgc,
                                                      int bc) {
    typedef typename St<S>::C C;
    const int nc = 1 << lgc;
    int oi, ni, oj, nj, ok = 0, nk = 0;
    float si, sj, sk = 1.0f;
    pro_axis(i, nc, bc, oi, ni, si);
    pro_axis(j, nc, bc, oj, nj, sj);
    if (D == 3) pro_axis(k, nc, bc, ok, nk, sk);
    C s = C(0);
    for (int cz = 0; cz < (D == 3 ? 2 : 1); ++cz)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const C w = C(a ? 0.25 : 0.75) * C(b ? 0.25 : 0.75) * C(D == 3 ? (cz ? 0.25 : 0.75) : 1.0);
                const C sg = C((a ? si : 1.0f) * (b ? sj : 1.0f) * (cz ? sk : 1.0f));
                const int64_t q = (int64_t(cz ? nk : ok) << (2 * lgc)) | (int64_t(b ? nj : oj) << lgc) |
                                  (a ? ni : oi);
                s = np_fma(w, sg * St<S>::ld(ec + q), s);
            }
    return s;
}

// x += P ec, one thread per fine cell.  lgc is the coarse level's log2 size.
template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_prolong_add(const S *__restrict__ ec, S *__restrict__ x,
                                                        int lgc, int bc, const int *stop) {
    if (stop && *stop) return;
    const int lg = lgc + 1;
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(sizeof(S) < 8 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int i, j, k;
    decode<D>(c, lg, i, j, k);
    St<S>::st(x + c, St<S>::ld(x + c) + pro_cell<D, S>(ec, i, j, k, lgc, bc));
}

// The corrected iterate x + P ec at flat index q, rounded to the storage
// precision as the stored iterate of prolongation then sweep is.
template <int D, class S> struct LdPro {
    const S *x, *ec;
    int lg, bc;
    __device__ __forceinline__ typename St<S>::C operator()(int64_t q) const {
        int i, j, k;
        decode<D>(q, lg, i, j, k);
        return st_round<S>(St<S>::ld(x + q) + pro_cell<D, S>(ec, i, j, k, lg - 1, bc));
    }
};

// Prolongation + correction followed by one Jacobi sweep, one thread per fine
// cell: xout = sweep(xin + P ec), the corrected iterate formed for the cell and
// its neighbours where they are read (same arithmetic as k_prolong_add then
// k_sweep, so the same result bit for bit).  Used on the 2D levels above the
// one-workgroup tail, where every launch costs about as much as the work.
template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_psweep(const S *__restrict__ ec, const S *__restrict__ f,
                                                   const S *__restrict__ xin, S *__restrict__ xout, int lg, int bc,
                                                   typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                   const int *stop) {
    typedef typename St<S>::C C;
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(sizeof(S) < 8 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int i, j, k;
    decode<D>(c, lg, i, j, k);
    const LdPro<D, S> ld{xin, ec, lg, bc};
    const C fc = St<S>::ld(f + c), xc = ld(c);
    const C s = nb_sum<D, C>(ld, c, i, j, k, lg, bc, xc);
    const C r = fc - (C(2 * D) * xc - s) * inv_h2;
    St<S>::st(xout + c, xc + wdiag * r);
}

// Exact solve on the 4^d coarsest grid: x <- x + Minv (f - A x), Minv the
// dense FP64 inverse (periodic: of A + 1 1^T / m).  One workgroup of 64.
template <int D, class S>
__global__ __launch_bounds__(64) void k_coarse(const S *__restrict__ f, S *__restrict__ x,
                                               const double *__restrict__ Minv, int bc, double inv_h2,
                                               int zero, const int *stop) {
    constexpr int m = D == 3 ? 64 : 16;
    if (stop && *stop) return;
    __shared__ double xs[64], rs[64];
    const int t = threadIdx.x;
    if (t < m) xs[t] = zero ? 0.0 : double(St<S>::ld(x + t));
    __syncthreads();
    if (t < m) {
        int i, j, k;
        decode<D>(t, 2, i, j, k);
        struct {
            const double *p;
            __device__ double operator()(int64_t q) const { return p[q]; }
        } ldx{xs};
        const double s = nb_sum<D, double>(ldx, t, i, j, k, 2, bc, xs[t]);
        rs[t] = double(St<S>::ld(f + t)) - (double(2 * D) * xs[t] - s) * inv_h2;
    }
    __syncthreads();
    if (t < m) {
        double acc = 0.0;
        for (int q = 0; q < m; ++q) acc += Minv[t * m + q] * rs[q];
        St<S>::st(x + t, typename St<S>::C(xs[t] + acc));
    }
}

// Partial sums of (f - A x)^2 in FP64 over a fixed grid of blocks.
template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_resid_sq(const S *__restrict__ f, const S *__restrict__ x,
                                                     double *__restrict__ partial, int lg, int bc,
                                                     typename St<S>::C inv_h2) {
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m;
         c += int64_t(gridDim.x) * blockDim.x) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const double r = double(resid_at<D, S>(f, x, c, i, j, k, lg, bc, inv_h2));
        acc += r * r;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Partial sums of x (f + r), r = f - A x, in FP64.  The energy-norm error of
// x relative to that of the zero iterate is ||x - x*||_A^2 - ||x*||_A^2 =
// x'Ax - 2 f'x = -sum x (f + r): a positive sum means x is closer to the
// solution than zero in the norm the V-cycle contracts.
template <int D, class S>
__global__ __launch_bounds__(kBlock) void k_energy(const S *__restrict__ f, const S *__restrict__ x,
                                                   double *__restrict__ partial, int lg, int bc,
                                                   typename St<S>::C inv_h2) {
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m;
         c += int64_t(gridDim.x) * blockDim.x) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const double r = double(resid_at<D, S>(f, x, c, i, j, k, lg, bc, inv_h2));
        acc += double(St<S>::ld(x + c)) * (double(St<S>::ld(f + c)) + r);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Partial sums of v (square = 0) or v^2 (square = 1) in FP64.
template <class S>
__global__ __launch_bounds__(kBlock) void k_sum(const S *__restrict__ v, int64_t m, int square,
                                                double *__restrict__ partial) {
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m;
         c += int64_t(gridDim.x) * blockDim.x) {
        const double a = double(St<S>::ld(v + c));
        acc += square ? a * a : a;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// k_sum's squared-norm partials of an FP64 field (the same order) and the field
// rounded to the storage S: the mixed solve's first residual r = f, and its
// check, when the iterate starts at zero.
template <class S>
__global__ __launch_bounds__(kBlock) void k_sum_round(const double *__restrict__ v, int64_t m,
                                                      S *__restrict__ lo, double *__restrict__ partial) {
    typedef typename St<S>::C C;
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m;
         c += int64_t(gridDim.x) * blockDim.x) {
        const double a = v[c];
        acc += a * a;
        St<S>::st(lo + c, C(a));
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// out[slot] = sum of partial[0..np) in a fixed order (sqrt when root).
static __global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partial, int np,
                                                     double *__restrict__ out, int root) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < np; b += blockDim.x) acc += partial[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[0] = root ? sqrt(acc) : acc;
}

// v[c] -= sum[0] * scale (mean removal with the sum left on the device).
static __global__ __launch_bounds__(kBlock) void k_sub_scaled(double *__restrict__ v, int64_t m,
                                                       const double *__restrict__ sum, double scale) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < m) v[c] -= sum[0] * scale;
}

// FP64 refinement step of the mixed-precision solve: x_out = x + e (e in the
// inner precision; has_e = 0 means e = 0 and x_out is not written),
// r = f - A x_out in FP64, r_lo = r rounded to the inner precision, and FP64
// partial sums of r^2, one per workgroup of kIrCells cells.  Neighbour values
// of x_out are formed on the fly, so x and x_out must be different buffers.
constexpr int kIrCells = 4 * kBlock;
template <int D, class SL>
__global__ __launch_bounds__(kBlock) void k_ir_resid(const double *__restrict__ x,
                                                     const SL *__restrict__ e,
                                                     double *__restrict__ xout,
                                                     const double *__restrict__ f,
                                                     SL *__restrict__ rlo,
                                                     double *__restrict__ partial, int lg, int bc,
                                                     double inv_h2, int has_e, const int *stop) {
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    struct {
        const double *x;
        const SL *e;
        int he;
        __device__ double operator()(int64_t q) const {
            return he ? x[q] + double(St<SL>::ld(e + q)) : x[q];
        }
    } ldx{x, e, has_e};
    const unsigned blk = blockIdx.x;
    for (int64_t base = int64_t(blk) * kIrCells; base < m; base += int64_t(gridDim.x) * kIrCells)
#pragma unroll
    for (int u = 0; u < kIrCells / kBlock; ++u) {
        const int64_t c = base + u * kBlock + threadIdx.x;
        if (c < m) {
            int i, j, k;
            decode<D>(c, lg, i, j, k);
            const double xc = ldx(c);
            const double s = nb_sum<D, double>(ldx, c, i, j, k, lg, bc, xc);
            const double r = f[c] - (double(2 * D) * xc - s) * inv_h2;
            if (has_e) xout[c] = xc;
            St<SL>::st(rlo + c, typename St<SL>::C(r));
            acc += r * r;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// ---------------------------------------------------- the sawtooth cycle
// Kernels of the paper's sawtooth cycle (Section 2.2; Appendix B), FP64.

// r = f - A x, with partial sums of r^2 over a fixed grid of blocks.
template <int D>
__global__ __launch_bounds__(kBlock) void k_saw_resid(const double *__restrict__ f, const double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ partial, int lg,
                                                      int bc, double inv_h2, const int *stop) {
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m; c += int64_t(gridDim.x) * blockDim.x) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const double v = resid_at<D, double>(f, x, c, i, j, k, lg, bc, inv_h2);
        r[c] = v;
        acc += v * v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// rc = R r: the 2^d-cell average of a field (no residual).  lgc: coarse size.
template <int D>
__global__ __launch_bounds__(kBlock) void k_restrict_field(const double *__restrict__ r, double *__restrict__ rc,
                                                           int lgc, const int *stop) {
    if (stop && *stop) return;
    const int64_t mc = int64_t(1) << (D * lgc);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= mc) return;
    int I, J, K;
    decode<D>(c, lgc, I, J, K);
    const int lg = lgc + 1;
    double s = 0.0;
    for (int kk = 0; kk < (D == 3 ? 2 : 1); ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii)
                s += r[(int64_t(D == 3 ? 2 * K + kk : 0) << (2 * lg)) | (int64_t(2 * J + jj) << lg) | (2 * I + ii)];
    rc[c] = s * (D == 3 ? 0.125 : 0.25);
}

// Start of a level's correction on the way up: e = r / A_00 + P ec, P the
// paper's copy (pconst) or the linear prolongation; ec null on the coarsest
// level.  lg: this level's size.
template <int D>
__global__ __launch_bounds__(kBlock) void k_saw_up(const double *__restrict__ r, const double *__restrict__ ec,
                                                   double *__restrict__ e, int lg, int bc, double inv_a00, int pconst,
                                                   const int *stop) {
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double v = r[c] * inv_a00;
    if (ec) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const int lgc = lg - 1, nc = 1 << lgc;
        if (pconst) {
            v += ec[(int64_t(k >> 1) << (2 * lgc)) | (int64_t(j >> 1) << lgc) | (i >> 1)];
        } else {
            int oi, ni, oj, nj, ok = 0, nk = 0;
            float si, sj, sk = 1.0f;
            pro_axis(i, nc, bc, oi, ni, si);
            pro_axis(j, nc, bc, oj, nj, sj);
            if (D == 3) pro_axis(k, nc, bc, ok, nk, sk);
            double s = 0.0;
            for (int cz = 0; cz < (D == 3 ? 2 : 1); ++cz)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (D == 3 ? (cz ? 0.25 : 0.75) : 1.0);
                        const double sg = double((a ? si : 1.0f) * (b ? sj : 1.0f) * (cz ? sk : 1.0f));
                        s += w * (sg * ec[(int64_t(cz ? nk : ok) << (2 * lgc)) | (int64_t(b ? nj : oj) << lgc) |
                                          (a ? ni : oi)]);
                    }
            v += s;
        }
    }
    e[c] = v;
}

// x += e.
static __global__ __launch_bounds__(kBlock) void k_add_to(double *__restrict__ x, const double *__restrict__ e,
                                                          int64_t m, const int *stop) {
    if (stop && *stop) return;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < m) x[c] += e[c];
}

// Solve controller kept in device memory so that cycles can be enqueued (and
// replayed from graphs) without a host round trip per cycle.
struct Ctl {
    int stop;       // 0 running; otherwise the reason (StopReason)
    int k;          // cycles (or refinement steps) completed
    int fixed;      // > 0: stop after exactly this many
    int maxc;       // cap
    double nf;      // ||f||_2
    double tol;
    int nhist;
    int pad;
    double hist[256];
};
enum StopReason { kRunning = 0, kConverged = 1, kFixedDone = 2, kMaxCycles = 3, kNonFinite = 4, kDiverged = 5 };

// Convergence check before cycle k: rr = sqrt(sum of partials)/||f|| (fixed
// summation order), recorded in hist[k]; then the stop rule: non-finite,
// fixed count reached, rr <= tol, k >= max, or three consecutive increases.
// Run by a whole workgroup of NT >= kBlock threads: the first kBlock sum the
// partials (four interleaved accumulators, a fixed assignment) and the others
// add zeros, so that every NT gives the same sum.  Returns the stop state to
// thread 0 (0 to the others).
template <int NT>
__device__ __forceinline__ int check_block(const double *__restrict__ partial, int np, Ctl *__restrict__ c) {
    if (c->stop) return threadIdx.x == 0 ? c->stop : 0;  // uniform: one value for the workgroup
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (int(threadIdx.x) < kBlock) {
        int b = threadIdx.x;
        for (; b + 3 * kBlock < np; b += 4 * kBlock) {
            a0 += partial[b];
            a1 += partial[b + kBlock];
            a2 += partial[b + 2 * kBlock];
            a3 += partial[b + 3 * kBlock];
        }
        for (; b < np; b += kBlock) a0 += partial[b];
    }
    const double acc = block_sum_n<NT>((a0 + a1) + (a2 + a3));
    if (threadIdx.x != 0) return 0;
    const int k = c->k;
    const double rr = sqrt(acc) / c->nf;
    if (k < 256) c->hist[k] = rr;
    c->nhist = k + 1 < 256 ? k + 1 : 256;
    int st = kRunning;
    if (!(rr <= 1.0e300)) st = kNonFinite;  // NaN or Inf
    else if (c->fixed > 0) { if (k >= c->fixed) st = kFixedDone; }
    else if (rr <= c->tol) st = kConverged;
    else if (k >= c->maxc) st = kMaxCycles;
    else if (k >= 3 && k < 256 && c->hist[k - 3] < c->hist[k - 2] && c->hist[k - 2] < c->hist[k - 1] &&
             c->hist[k - 1] < rr)
        st = kDiverged;
    if (st != kRunning) c->stop = st;
    else c->k = k + 1;
    return st;
}

// The controller at the start of a solve: running, k0 cycles done (history
// entry 0 = h0 when k0 > 0), the rest of the history zero.
static __global__ __launch_bounds__(kBlock) void k_init_ctl(Ctl *__restrict__ c, int k0, int fixed, int maxc,
                                                     double nf, double tol, double h0) {
    for (int i = threadIdx.x; i < 256; i += kBlock) c->hist[i] = (i == 0 && k0 > 0) ? h0 : 0.0;
    if (threadIdx.x == 0) {
        c->stop = kRunning;
        c->k = k0;
        c->fixed = fixed;
        c->maxc = maxc;
        c->nf = nf;
        c->tol = tol;
        c->nhist = k0;
        c->pad = 0;
    }
}

static __global__ __launch_bounds__(kBlock) void k_check(const double *__restrict__ partial, int np,
                                                  Ctl *__restrict__ c) {
    (void)check_block<kBlock>(partial, np, c);
}

// y = A x (FP64).
template <int D>
__global__ __launch_bounds__(kBlock) void k_apply(const double *__restrict__ x, double *__restrict__ y, int lg,
                                                  int bc, double inv_h2) {
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int i, j, k;
    decode<D>(c, lg, i, j, k);
    const double xc = x[c];
    const double s = nb_sum<D, double>(Ld<double>{x}, c, i, j, k, lg, bc, xc);
    y[c] = (double(2 * D) * xc - s) * inv_h2;
}

// dst = src (gated copy used inside captured cycles).
template <class S>
__global__ __launch_bounds__(kBlock) void k_copy(const S *__restrict__ src, S *__restrict__ dst, int64_t m,
                                                 const int *stop) {
    if (stop && *stop) return;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < m) dst[c] = src[c];
}

// Fill with zeros (used instead of a memset so the work stays in kernels).
template <class S>
__global__ __launch_bounds__(kBlock) void k_zero(S *__restrict__ v, int64_t m, const int *stop) {
    if (stop && *stop) return;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < m) St<S>::st(v + c, typename St<S>::C(0));
}

}  // namespace np
