// Device kernels of the implicit advection-diffusion multigrid (gfx950), FP64.
// Included by mg.hip after mg_kernels.h.
//
// The backward-Euler operator of Section 2.2 with constant coefficients,
// re-discretised on every level with that level's spacing:
//   (A x)_c = c0 x_c + sum_e (cm[e] x_{c - e} + cp[e] x_{c + e}),
// with the weights of AdW (see ad_weights in mg.hip); ghosts by the boundary
// rule (Dirichlet-0: -(own value); periodic: wrap).  The centre weight c0 is
// the filter centre A_00 that Jacobi divides by.
#pragma once

#include "mg_kernels.h"
#include "mg_level.h"

namespace np {

struct AdW {
    double c0;
    double cm[3], cp[3];
};

// (A x)_c at cell c = (i, j, k).
template <int D>
__device__ __forceinline__ double ad_ax(const double *__restrict__ x, int64_t c, int i, int j, int k, int lg, int bc,
                                        const AdW &W) {
    const int n = 1 << lg;
    const int64_t sy = int64_t(1) << lg;
    const double xc = x[c];
    const double xm = i > 0 ? x[c - 1] : (bc ? x[c + (n - 1)] : -xc);
    const double xp = i < n - 1 ? x[c + 1] : (bc ? x[c - (n - 1)] : -xc);
    const double ym = j > 0 ? x[c - sy] : (bc ? x[c + (n - 1) * sy] : -xc);
    const double yp = j < n - 1 ? x[c + sy] : (bc ? x[c - (n - 1) * sy] : -xc);
    double s = W.c0 * xc + (W.cm[0] * xm + W.cp[0] * xp) + (W.cm[1] * ym + W.cp[1] * yp);
    if (D == 3) {
        const int64_t sz = int64_t(1) << (2 * lg);
        const double zm = k > 0 ? x[c - sz] : (bc ? x[c + (n - 1) * sz] : -xc);
        const double zp = k < n - 1 ? x[c + sz] : (bc ? x[c - (n - 1) * sz] : -xc);
        s += W.cm[2] * zm + W.cp[2] * zp;
    }
    return s;
}

// y = A x.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ad_apply(const double *__restrict__ x, double *__restrict__ y, int lg,
                                                     int bc, AdW W) {
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t c = int64_t(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int i, j, k;
    decode<D>(c, lg, i, j, k);
    y[c] = ad_ax<D>(x, c, i, j, k, lg, bc, W);
}

// One relaxed-Jacobi sweep x_out = x_in + omega (f - A x_in) / c0 (wdiag =
// omega / c0).  ZERO: x_in is identically zero, x_out = wdiag f.  NORM: the
// grid is strided (gridDim.x <= the partial count) and each workgroup writes
// its share of ||f - A x_in||^2 to partial[blockIdx.x] (fixed order).
template <int D, bool ZERO, bool NORM>
__global__ __launch_bounds__(kBlock) void k_ad_sweep(const double *__restrict__ f, const double *__restrict__ xin,
                                                     double *__restrict__ xout, double *__restrict__ partial, int lg,
                                                     int bc, AdW W, double wdiag, const int *stop) {
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    if (!NORM) {
        const int64_t c = int64_t(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
        if (c >= m) return;
        if (ZERO) {
            xout[c] = wdiag * f[c];
            return;
        }
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        xout[c] = xin[c] + wdiag * (f[c] - ad_ax<D>(xin, c, i, j, k, lg, bc, W));
        return;
    }
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m; c += int64_t(gridDim.x) * blockDim.x) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const double r = f[c] - ad_ax<D>(xin, c, i, j, k, lg, bc, W);
        xout[c] = xin[c] + wdiag * r;
        acc += r * r;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// r = f - A x; with partial != null each workgroup of the strided grid also
// writes its share of ||r||^2 (r may be null: the norm alone).
template <int D>
__global__ __launch_bounds__(kBlock) void k_ad_resid(const double *__restrict__ f, const double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ partial, int lg,
                                                     int bc, AdW W, const int *stop) {
    if (stop && *stop) return;
    const int64_t m = int64_t(1) << (D * lg);
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m; c += int64_t(gridDim.x) * blockDim.x) {
        int i, j, k;
        decode<D>(c, lg, i, j, k);
        const double v = f[c] - ad_ax<D>(x, c, i, j, k, lg, bc, W);
        if (r) r[c] = v;
        acc += v * v;
    }
    if (!partial) return;
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// fc = R (f - A x): one thread per coarse cell averages the residual of its
// 2^d children.  lg is the fine level's log2 size.
template <int D>
__global__ __launch_bounds__(kBlock) void k_ad_resid_restrict(const double *__restrict__ f,
                                                              const double *__restrict__ x, double *__restrict__ fc,
                                                              int lg, int bc, AdW W, const int *stop) {
    if (stop && *stop) return;
    const int lgc = lg - 1;
    const int64_t mc = int64_t(1) << (D * lgc);
    const int64_t c = int64_t(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (c >= mc) return;
    int I, J, K;
    decode<D>(c, lgc, I, J, K);
    double acc = 0.0;
    for (int kk = 0; kk < (D == 3 ? 2 : 1); ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii) {
                const int i = 2 * I + ii, j = 2 * J + jj, k = D == 3 ? 2 * K + kk : 0;
                const int64_t cf = (int64_t(k) << (2 * lg)) | (int64_t(j) << lg) | i;
                acc += f[cf] - ad_ax<D>(x, cf, i, j, k, lg, bc, W);
            }
    fc[c] = acc * (D == 3 ? 0.125 : 0.25);
}

// Exact solve on the 4^d coarsest grid: x <- x + Minv (f - A x), Minv the
// dense inverse of the level's operator.  One workgroup of 64.
template <int D>
__global__ __launch_bounds__(64) void k_ad_coarse(const double *__restrict__ f, double *__restrict__ x,
                                                  const double *__restrict__ Minv, int bc, AdW W, int zero,
                                                  const int *stop) {
    constexpr int m = D == 3 ? 64 : 16;
    if (stop && *stop) return;
    __shared__ double xs[64], rs[64];
    const int t = threadIdx.x;
    if (t < m) xs[t] = zero ? 0.0 : x[t];
    __syncthreads();
    if (t < m) {
        int i, j, k;
        decode<D>(t, 2, i, j, k);
        rs[t] = f[t] - ad_ax<D>(xs, t, i, j, k, 2, bc, W);
    }
    __syncthreads();
    if (t < m) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += Minv[t * m + q] * rs[q];
        x[t] = xs[t] + s;
    }
}

// ------------------------------------------ 3D levels on z-marching tiles
// The tiles of ZMarch (one FP64 cell per thread): planes k - 1, k, k + 1 of the
// own column in registers, plane k with its halo in LDS, plane k + 1 loaded
// while plane k is computed.  Requires n >= 128.

// Publishes plane k of the tile to buffer b and returns (A x) at the thread's
// cell (one barrier per plane; the buffer is written again two planes later).
template <class Z>
__device__ __forceinline__ double ad_zm_ax(const Z &z, typename Z::Plane &b, const AdW &W) {
    b[z.ty + 1][z.tp + 1] = z.xc[0];
    if (z.hw) b[z.hy][z.hx] = z.hv[0];
    __syncthreads();
    const int lc = z.tp + 1;
    return W.c0 * z.xc[0] + (W.cm[0] * b[z.ty + 1][lc - 1] + W.cp[0] * b[z.ty + 1][lc + 1]) +
           (W.cm[1] * b[z.ty][lc] + W.cp[1] * b[z.ty + 2][lc]) + (W.cm[2] * z.xm[0] + W.cp[2] * z.xp[0]);
}

typedef ZMarch<double, ZCfg<double>::TX, 1> AdZ;

// Relaxed-Jacobi sweep (as k_ad_sweep) over zc planes per workgroup.  NORM:
// per-workgroup partial of ||f - A x_in||^2.
template <bool NORM>
__global__ __launch_bounds__(kS3Threads) void k_ad_sweep3(const double *__restrict__ f, const double *__restrict__ xin,
                                                          double *__restrict__ xout, double *__restrict__ partial,
                                                          int lg, int bc, int zc, AdW W, double wdiag,
                                                          const int *stop) {
    __shared__ AdZ::Plane pl[2];
    if (stop && *stop) return;
    AdZ z(lg, bc, zc);
    const LdC<double> v{xin};
    z.start(v);
    double fc = f[z.k0 * z.P + z.col];
    double acc = 0.0;
    for (int k = z.k0, q = 0; k < z.k0 + zc; ++k, q ^= 1) {
        z.prefetch(v, k);
        const double fn = f[z.next(k) * z.P + z.col];
        const double r = fc - ad_zm_ax(z, pl[q], W);
        if (NORM) acc += r * r;
        xout[k * z.P + z.col] = z.xc[0] + wdiag * r;
        fc = fn;
        z.advance();
    }
    if (NORM) {
        acc = block_sum_n<kS3Threads>(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// Residual + restriction (as k_ad_resid_restrict): each thread sums its
// residuals over a pair of planes, then one thread per coarse cell adds the
// pair sums of its 2 x 2 row neighbours through LDS.  zc even.
__global__ __launch_bounds__(kS3Threads) void k_ad_restrict3(const double *__restrict__ f,
                                                             const double *__restrict__ x, double *__restrict__ fc,
                                                             int lg, int bc, int zc, AdW W, const int *stop) {
    __shared__ AdZ::Plane pl[2];
    __shared__ double rs[AdZ::TY][AdZ::TP];
    if (stop && *stop) return;
    AdZ z(lg, bc, zc);
    const LdC<double> v{x};
    z.start(v);
    const int lgc = lg - 1;
    double f0 = f[z.k0 * z.P + z.col];
    double pair = 0.0;
    for (int k = z.k0, q = 0; k < z.k0 + zc; ++k, q ^= 1) {
        z.prefetch(v, k);
        const double fn = f[z.next(k) * z.P + z.col];
        const double r = f0 - ad_zm_ax(z, pl[q], W);
        if (((k - z.k0) & 1) == 0) {
            pair = r;
        } else {
            pair += r;
            rs[z.ty][z.tp] = pair;
            __syncthreads();
            if (((z.tp | z.ty) & 1) == 0) {
                const double t =
                    ((rs[z.ty][z.tp] + rs[z.ty][z.tp + 1]) + rs[z.ty + 1][z.tp]) + rs[z.ty + 1][z.tp + 1];
                const int64_t cc = ((int64_t(k >> 1) << (2 * lgc)) | (int64_t(z.j >> 1) << lgc)) + (z.i >> 1);
                fc[cc] = t * 0.125;
            }
            // rs is written again two planes later, after plane k + 1's barrier
        }
        z.advance();
        f0 = fn;
    }
}

// ------------------------------------------ 2D levels on row-marching strips
// A workgroup of kR2 threads owns kR2 consecutive columns and ry consecutive
// rows: rows j - 1, j, j + 1 of the own column in registers, row j with its
// two halo cells in LDS (two buffers, one barrier per row), row j + 2 and the
// halo of row j + 1 loaded while row j is computed.  Every thread issues the
// halo load (threads without a halo cell reload their own cell), so no load
// is conditional.  Requires n >= kR2.
constexpr int kR2 = kBlock;

struct RMarch {
    int n, lg, bc, i, j0, hx;
    bool hw;
    int64_t hsrc;
    double hsg;
    double xm, xc, xp, hv, xpp, hn;
    __device__ RMarch(int lg_, int bc_, int ry) : n(1 << lg_), lg(lg_), bc(bc_) {
        const int strips = n / kR2;
        const int blk = int(xcd_block(blockIdx.x, gridDim.x));
        const int t = int(threadIdx.x);
        const int x0 = (blk % strips) * kR2;
        j0 = (blk / strips) * ry;
        i = x0 + t;
        hw = t < 2;
        hx = t == 0 ? 0 : kR2 + 1;
        int gi = t == 0 ? x0 - 1 : (t == 1 ? x0 + kR2 : i);
        hsg = 1.0;
        if (gi < 0) {  // outside: wrap (periodic) or the adjacent cell negated (Dirichlet)
            gi = bc ? n - 1 : 0;
            if (!bc) hsg = -1.0;
        } else if (gi >= n) {
            gi = bc ? 0 : n - 1;
            if (!bc) hsg = -1.0;
        }
        hsrc = gi;
    }
    __device__ __forceinline__ int64_t row(int j) const { return int64_t(j) << lg; }
    // offset of the row above j and its sign (the top Dirichlet ghost is -(own value))
    __device__ __forceinline__ int64_t up_at(int j) const { return j < n - 1 ? row(j + 1) : (bc ? 0 : row(j)); }
    __device__ __forceinline__ double up_sg(int j) const { return (j < n - 1 || bc) ? 1.0 : -1.0; }
    __device__ __forceinline__ int next(int j) const { return j + 1 < n ? j + 1 : n - 1; }
    __device__ __forceinline__ void start(const double *__restrict__ x) {
        xc = x[row(j0) + i];
        if (j0 > 0) xm = x[row(j0 - 1) + i];
        else if (bc) xm = x[row(n - 1) + i];
        else xm = -xc;
        xp = x[up_at(j0) + i] * up_sg(j0);
        hv = hsg * x[row(j0) + hsrc];
    }
    __device__ __forceinline__ void prefetch(const double *__restrict__ x, int j) {
        const int jn = next(j);
        xpp = x[up_at(jn) + i] * up_sg(jn);
        hn = hsg * x[row(jn) + hsrc];
    }
    // publish row j to b and return (A x) at the own cell
    __device__ __forceinline__ double ax(double (&b)[kR2 + 2], const AdW &W) const {
        b[threadIdx.x + 1] = xc;
        if (hw) b[hx] = hv;
        __syncthreads();
        const int l = int(threadIdx.x) + 1;
        return W.c0 * xc + (W.cm[0] * b[l - 1] + W.cp[0] * b[l + 1]) + (W.cm[1] * xm + W.cp[1] * xp);
    }
    __device__ __forceinline__ void advance() {
        xm = xc;
        xc = xp;
        xp = xpp;
        hv = hn;
    }
};

// Rows per workgroup of a row-marching launch on an n^2 level: enough
// workgroups to fill the chip, at least 4 rows.
inline int r2_rows(int lg) {
    const int n = 1 << lg, strips = n / kR2;
    int ry = 32;
    while (int64_t(strips) * (n / ry) < 2048 && ry > 4) ry /= 2;
    return ry;
}

// Relaxed-Jacobi sweep (as k_ad_sweep) over ry rows per workgroup.  NORM:
// per-workgroup partial of ||f - A x_in||^2.
template <bool NORM>
__global__ __launch_bounds__(kR2) void k_ad_sweep2(const double *__restrict__ f, const double *__restrict__ xin,
                                                   double *__restrict__ xout, double *__restrict__ partial, int lg,
                                                   int bc, int ry, AdW W, double wdiag, const int *stop) {
    __shared__ double b[2][kR2 + 2];
    if (stop && *stop) return;
    RMarch z(lg, bc, ry);
    z.start(xin);
    double fc = f[z.row(z.j0) + z.i];
    double acc = 0.0;
    for (int j = z.j0, q = 0; j < z.j0 + ry; ++j, q ^= 1) {
        z.prefetch(xin, j);
        const double fn = f[z.row(z.next(j)) + z.i];
        const double r = fc - z.ax(b[q], W);
        if (NORM) acc += r * r;
        xout[z.row(j) + z.i] = z.xc + wdiag * r;
        fc = fn;
        z.advance();
    }
    if (NORM) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// Residual + restriction on row-marching strips: each thread sums its
// residuals over a pair of rows, then one thread per coarse cell adds its
// right neighbour's pair sum through LDS.  ry even.
__global__ __launch_bounds__(kR2) void k_ad_restrict2(const double *__restrict__ f, const double *__restrict__ x,
                                                      double *__restrict__ fc, int lg, int bc, int ry, AdW W,
                                                      const int *stop) {
    __shared__ double b[2][kR2 + 2];
    __shared__ double rs[kR2];
    if (stop && *stop) return;
    RMarch z(lg, bc, ry);
    z.start(x);
    const int lgc = lg - 1;
    double f0 = f[z.row(z.j0) + z.i];
    double pair = 0.0;
    for (int j = z.j0, q = 0; j < z.j0 + ry; ++j, q ^= 1) {
        z.prefetch(x, j);
        const double fn = f[z.row(z.next(j)) + z.i];
        const double r = f0 - z.ax(b[q], W);
        if (((j - z.j0) & 1) == 0) {
            pair = r;
        } else {
            pair += r;
            rs[threadIdx.x] = pair;
            __syncthreads();
            if ((threadIdx.x & 1) == 0)
                fc[(int64_t(j >> 1) << lgc) + (z.i >> 1)] = (rs[threadIdx.x] + rs[threadIdx.x + 1]) * 0.25;
            // rs is written again two rows later, after row j + 1's barrier
        }
        f0 = fn;
        z.advance();
    }
}

// ------------------------------------- small levels in one workgroup (LDS)
// Weights of the levels handled by k_ad_tail, finest first.
struct AdLevels {
    AdW w[12];
};

// One relaxed-Jacobi sweep T = X + wd (F - A X) (RESID: the residual T = F - A X)
// of a level of k_ad_tail, all three in LDS.  Each thread marches along the
// last axis over a run of one column's cells (neighbours along that axis from
// registers, in-plane offsets fixed per column); same terms and grouping as
// ad_ax.  Needs n^(D-1) <= NT.
template <int D, int NT, bool RESID, bool ZERO2 = false>
__device__ __forceinline__ void ad_tail_sweep(const double *__restrict__ X, const double *__restrict__ F,
                                              double *__restrict__ T, int lg, int bc, const AdW &W, double wd) {
    // ZERO2: the sweep after a first one from zero; its input iterate wd f is formed from F (X unused)
    auto xv = [&](int q) -> double { return ZERO2 ? wd * F[q] : X[q]; };
    const int n = 1 << lg, last = n - 1, sm = D == 3 ? n * n : n;
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
        double xc = xv(c);
        double zm = xv(z0 > 0 ? c - sm : (per ? c + last * sm : c));
        bool fzm = z0 > 0 || per;
        for (int z = z0; z < z0 + len; ++z, c += sm) {
            const double zp = xv(z < last ? c + sm : (per ? c - last * sm : c));
            const bool fzp = z < last || per;
            const double rxm = xv(c + oxm), rxp = xv(c + oxp);  // unconditional: no branch around a load
            const double xm = fxm ? rxm : -xc, xp = fxp ? rxp : -xc;
            const double am = fzm ? zm : -xc, ap = fzp ? zp : -xc;  // along the marching axis
            double s;
            if (D == 3) {
                const double rym = xv(c + oym), ryp = xv(c + oyp);
                const double ym = fym ? rym : -xc, yp = fyp ? ryp : -xc;
                s = W.c0 * xc + (W.cm[0] * xm + W.cp[0] * xp) + (W.cm[1] * ym + W.cp[1] * yp);
                s += W.cm[2] * am + W.cp[2] * ap;
            } else {
                s = W.c0 * xc + (W.cm[0] * xm + W.cp[0] * xp) + (W.cm[1] * am + W.cp[1] * ap);
            }
            if (RESID) T[c] = F[c] - s;
            else T[c] = xc + wd * (F[c] - s);
            zm = xc;
            fzm = true;
            xc = zp;
        }
    }
}

// V(nu1, nu2) cycle on levels lg_t .. 2 (coarsest 4^d) in one workgroup,
// every level in LDS, from a zero iterate on every level (the levels below
// the finest ones of a cycle): first sweep x = wdiag f, nu1 - 1 further
// sweeps, residual restriction, the exact solve Minv f on 4^d, then per
// level up prolongation + nu2 sweeps.  f_t: right-hand side of level lg_t
// (global); x_t: its correction (global).  nu1 >= 1; lg_t <= Tail<D>::LG.
template <int D>
__global__ __launch_bounds__(Tail<D>::NT_AD) void k_ad_tail(const double *__restrict__ f_t, double *__restrict__ x_t,
                                                         const double *__restrict__ Minv, int lg_t, int bc,
                                                         AdLevels Wl, double omega, int nu1, int nu2,
                                                         const int *stop) {
    constexpr int NT = Tail<D>::NT_AD;
    static_assert(Tail<D>::cells(Tail<D>::LG) >> Tail<D>::LG <= NT, "ad_tail_sweep needs n^(D-1) <= NT");
    __shared__ double xs[Tail<D>::levels_sum()];
    __shared__ double fs[Tail<D>::levels_sum()];
    __shared__ double ts[Tail<D>::cells(Tail<D>::LG)];
    // the coarsest inverse, transposed with padded rows (thread i reading entry
    // (i, q) hits consecutive banks); its loads go out with the right-hand side's
    constexpr int mq = D == 3 ? 64 : 16, mp = mq + 1;
    __shared__ double Ms[mq * mp];
    if (stop && *stop) return;
    const int tid = threadIdx.x;
    auto off = [&](int l) -> int64_t {  // level l follows the finer levels lg_t .. l + 1
        return ((int64_t(1) << (D * (lg_t + 1))) - (int64_t(1) << (D * (l + 1)))) / ((int64_t(1) << D) - 1);
    };
    const int mt = 1 << (D * lg_t);
    {
        constexpr int per = int(Tail<D>::cells(Tail<D>::LG) / NT);
        double fv[per];
#pragma unroll
        for (int u = 0; u < per; ++u)
            if (tid + u * NT < mt) fv[u] = f_t[tid + u * NT];
        for (int g = tid; g < mq * mq; g += NT) Ms[(g % mq) * mp + g / mq] = Minv[g];
#pragma unroll
        for (int u = 0; u < per; ++u)
            if (tid + u * NT < mt) fs[tid + u * NT] = fv[u];
    }
    __syncthreads();
    // cnt sweeps alternating between X and ts; the result ends in X
    auto sweeps = [&](double *X, const double *F, int lg, const AdW &W, double wd, int cnt) {
        double *cur = X, *nxt = ts;
        for (int it = 0; it < cnt; ++it) {
            ad_tail_sweep<D, NT, false>(cur, F, nxt, lg, bc, W, wd);
            __syncthreads();
            double *t = cur;
            cur = nxt;
            nxt = t;
        }
        if (cur != X) {
            for (int c = tid; c < (1 << (D * lg)); c += NT) X[c] = cur[c];
            __syncthreads();
        }
    };
    for (int lg = lg_t; lg > 2; --lg) {
        const int m = 1 << (D * lg);
        double *X = xs + off(lg), *F = fs + off(lg);
        const AdW W = Wl.w[lg_t - lg];
        const double wd = omega / W.c0;
        if (nu1 >= 2) {
            // the first two sweeps from zero in one pass, straight into X
            ad_tail_sweep<D, NT, false, true>(F, F, X, lg, bc, W, wd);
            __syncthreads();
            sweeps(X, F, lg, W, wd, nu1 - 2);
        } else {
            for (int c = tid; c < m; c += NT) X[c] = wd * F[c];
            __syncthreads();
            sweeps(X, F, lg, W, wd, nu1 - 1);
        }
        // residual into ts, then its 2^d-cell average into the next level's rhs
        ad_tail_sweep<D, NT, true>(X, F, ts, lg, bc, W, wd);
        __syncthreads();
        const int lgc = lg - 1, mc = 1 << (D * lgc);
        double *Fc = fs + off(lgc);
        for (int cc = tid; cc < mc; cc += NT) {
            int I, J, K;
            decode<D>(cc, lgc, I, J, K);
            double acc = 0.0;
            for (int kk = 0; kk < (D == 3 ? 2 : 1); ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii) {
                        const int i = 2 * I + ii, j = 2 * J + jj, k = D == 3 ? 2 * K + kk : 0;
                        acc += ts[(k << (2 * lg)) | (j << lg) | i];
                    }
            Fc[cc] = acc * (D == 3 ? 0.125 : 0.25);
        }
        __syncthreads();
    }
    {
        double *X = xs + off(2), *F = fs + off(2);
        if (tid < mq) {
            double acc = 0.0;
            for (int q = 0; q < mq; ++q) acc += Ms[tid + q * mp] * F[q];
            X[tid] = acc;
        }
        __syncthreads();
    }
    for (int lg = 3; lg <= lg_t; ++lg) {
        const int lgc = lg - 1;
        double *X = xs + off(lg), *F = fs + off(lg), *E = xs + off(lgc);
        const AdW W = Wl.w[lg_t - lg];
        tail_prolong<D, double, NT>(E, X, lg, bc);
        __syncthreads();
        sweeps(X, F, lg, W, omega / W.c0, nu2);
    }
    for (int c = tid; c < mt; c += NT) x_t[c] = xs[c];
}

// Partials of ||a - b||_1 (||a||_1 when b is null) over a strided grid (fixed
// order), gated by the controller: the change of the iterate over the cycle
// just run.
static __global__ __launch_bounds__(kBlock) void k_l1_diff(const double *__restrict__ a, const double *__restrict__ b,
                                                         int64_t m, double *__restrict__ partial, const int *stop) {
    if (stop && *stop) return;
    double acc = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m; c += int64_t(gridDim.x) * blockDim.x)
        acc += fabs(b ? a[c] - b[c] : a[c]);
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Sums the partials of k_l1_diff into out[k - 1], k the controller's count of
// cycles started (the cycle just run), while the controller runs.
static __global__ __launch_bounds__(kBlock) void k_l1_store(const double *__restrict__ partial, int np,
                                                          const Ctl *__restrict__ c, double *__restrict__ out) {
    if (c->stop) return;
    double a = 0.0;
    for (int b = threadIdx.x; b < np; b += kBlock) a += partial[b];
    a = block_sum(a);
    if (threadIdx.x == 0 && c->k >= 1 && c->k <= 256) out[c->k - 1] = a;
}

}  // namespace np
