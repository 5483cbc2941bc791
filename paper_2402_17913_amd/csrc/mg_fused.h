// Fused multigrid level kernels (gfx950): several stencil stages of one level
// in a single pass over HBM.
//
// A workgroup owns an output tile of BX (x) [x BY (y)] columns and a chunk of
// `bz` planes along the marching axis (z in 3D, y in 2D).  It loads its tile
// with a halo of H = (number of stencil stages) columns on every side and
// marches through the chunk plane by plane.  Stage j of the pipeline lags the
// loads by j planes: at step t, stage j produces plane t - j.  Each stage keeps
// the last three planes of its output in registers (the marching-axis
// neighbours of its own columns) and publishes the newest plane in LDS (the
// in-plane neighbours of other columns).  LDS is double buffered per stage, so
// a stage reads the plane its producer wrote one step earlier while the
// producer writes the next: one barrier per step.
//
// Stages (all in the arithmetic type of the storage):
//   stage 0  input  x (PRE_NONE), w f (PRE_ZERO: the first Jacobi sweep from a
//            zero iterate) or x + P e_coarse (PRE_PROLONG: linear prolongation
//            and correction);
//   stage j  weighted Jacobi  s_j = s_{j-1} + w (f - A s_{j-1}),  j = 1..NJ;
//            with NORM, stage 1 also accumulates ||f - A s_0||^2 (the residual
//            of the input iterate) over the owned cells;
//   RES      r = f - A s_NJ, averaged over 2^d children into the coarse right-
//            hand side (restriction).
// Output: s_NJ on the owned cells (when NJ > 0 or PRE != PRE_NONE) and the
// restricted residual.  Arithmetic per cell is identical to the single-
// operation kernels (same expressions, same summation order).
#pragma once

#include "mg_kernels.h"
#include "np_internal.h"

namespace np {

enum { PRE_NONE = 0, PRE_ZERO = 1, PRE_PROLONG = 2 };

template <class S> struct FusedArgs {
    const S *xin;      // stage-0 iterate (PRE_NONE, PRE_PROLONG)
    const S *f;        // right-hand side of this level
    S *xout;           // iterate after the Jacobi stages
    const S *ec;       // coarse error (PRE_PROLONG)
    S *fc;             // restricted residual (RES)
    double *partial;   // per-workgroup ||f - A x_in||^2 (NORM)
    const int *stop;   // nonzero: the solve has stopped, exit at once (may be null)
    int lg, bc, bz;    // log2 n, boundary rule, planes per workgroup
    int tiles_x, tiles_y, nblocks;
    typename St<S>::C inv_h2, wdiag;
};

// Linear prolongation value P e at fine cell (gx, gy, gz) of a grid of 2^lg cells.
template <int D, class S>
__device__ __forceinline__ typename St<S>::C prolong_at(const S *__restrict__ ec, int gx, int gy, int gz,
                                                        int lg, int bc) {
    typedef typename St<S>::C C;
    const int lgc = lg - 1, nc = 1 << lgc;
    int oi, ni, oj, nj, ok = 0, nk = 0;
    float si, sj, sk = 1.0f;
    pro_axis(gx, nc, bc, oi, ni, si);
    pro_axis(gy, nc, bc, oj, nj, sj);
    if (D == 3) pro_axis(gz, nc, bc, ok, nk, sk);
    C s = C(0);
#pragma unroll
    for (int cz = 0; cz < (D == 3 ? 2 : 1); ++cz)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const C w = C(a ? 0.25 : 0.75) * C(b ? 0.25 : 0.75) * C(D == 3 ? (cz ? 0.25 : 0.75) : 1.0);
                const C sg = C((a ? si : 1.0f) * (b ? sj : 1.0f) * (cz ? sk : 1.0f));
                const int64_t q = (int64_t(cz ? nk : ok) << (2 * lgc)) | (int64_t(b ? nj : oj) << lgc) |
                                  (a ? ni : oi);
                s += w * (sg * St<S>::ld(ec + q));
            }
    return s;
}

// TX x TY: tile with halo (TY = 1 in 2D).  NJ Jacobi stages, optional
// restriction stage, optional input-residual norm.
template <int D, class S, int TX, int TY, int NJ, int PRE, bool RES, bool NORM>
__global__ __launch_bounds__(256) void k_fused(FusedArgs<S> a) {
    typedef typename St<S>::C C;
    constexpr int H = NJ + (RES ? 1 : 0);
    constexpr int BX = TX - 2 * H;
    constexpr int BY = D == 3 ? TY - 2 * H : 1;
    constexpr int NC = TX * TY;
    constexpr int R = (NC + 255) / 256;
    constexpr int NST = H;                     // stage outputs read through LDS by a stencil
    constexpr int NCC = (BX / 2) * (D == 3 ? BY / 2 : 1);  // coarse columns owned
    constexpr int RC = (NCC + 255) / 256;
    static_assert(BX > 0 && BX % 2 == 0 && (D == 2 || (BY > 0 && BY % 2 == 0)), "tile too small");

    __shared__ C lds[NST + (RES ? 1 : 0)][2][NC];

    if (a.stop && *a.stop) return;

    // XCD-aware block order: consecutive tiles land on the same XCD (one L2).
    int bid = blockIdx.x;
    if ((a.nblocks & 7) == 0) bid = (blockIdx.x & 7) * (a.nblocks >> 3) + (blockIdx.x >> 3);
    const int btx = bid % a.tiles_x;
    const int bty = (bid / a.tiles_x) % a.tiles_y;
    const int btz = bid / (a.tiles_x * a.tiles_y);

    const int lg = a.lg, n = 1 << lg, bc = a.bc;
    const int x0 = btx * BX, y0 = D == 3 ? bty * BY : 0, z0 = btz * a.bz;
    const int zend = min(z0 + a.bz, n);
    const int64_t plane = D == 3 ? (int64_t(1) << (2 * lg)) : (int64_t(1) << lg);
    const int tid = threadIdx.x;

    // per-column state
    int64_t coff[R];       // in-plane offset of the column's global cell (wrapped when periodic)
    int cidx[R];           // column index in the tile, -1 when the slot is unused
    bool live[R];          // column maps to a cell of the domain
    bool own[R];           // column is in the owned output region
    unsigned char bnd[R];  // Dirichlet boundary flags: 1 x-lo, 2 x-hi, 4 y-lo, 8 y-hi
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int c = tid + 256 * r;
        cidx[r] = c < NC ? c : -1;
        const int cx = c % TX, cy = c / TX;
        int gx = x0 - H + cx, gy = D == 3 ? y0 - H + cy : 0;
        bool in = c < NC;
        if (bc) {
            gx = (gx % n + n) % n;
            if (D == 3) gy = (gy % n + n) % n;
        } else {
            in = in && gx >= 0 && gx < n && gy >= 0 && gy < n;
        }
        live[r] = in;
        own[r] = in && cx >= H && cx < H + BX && x0 - H + cx < n &&
                 (D == 2 || (cy >= H && cy < H + BY && y0 - H + cy < n));
        coff[r] = in ? (D == 3 ? int64_t(gy) * n + gx : int64_t(gx)) : 0;
        unsigned char fl = 0;
        if (!bc && in) {
            if (gx == 0) fl |= 1;
            if (gx == n - 1) fl |= 2;
            if (D == 3 && gy == 0) fl |= 4;
            if (D == 3 && gy == n - 1) fl |= 8;
        }
        bnd[r] = fl;
    }

    // register queues: q[j][r][0..2] = stage j at planes (p-1, p, p+1) of its consumer
    C q[NST + 1][R][3];
    C fq[R][H + 1];  // f at planes t, t-1, ..., t-H
#pragma unroll
    for (int j = 0; j <= NST; ++j)
#pragma unroll
        for (int r = 0; r < R; ++r) q[j][r][0] = q[j][r][1] = q[j][r][2] = C(0);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k <= H; ++k) fq[r][k] = C(0);

    C racc[RC];
#pragma unroll
    for (int k = 0; k < RC; ++k) racc[k] = C(0);
    double nacc = 0.0;

    const int t0 = z0 - H;
    const int t1 = z0 + a.bz - 1 + H + (RES ? 1 : 0);
    const int tload = z0 + a.bz - 1 + H;  // last plane any stage needs

    // Software prefetch: the raw loads of plane t + PF are issued at step t, so
    // each load has PF steps (compute + barrier) to arrive before it is used.
    constexpr int PF = 2;
    C px[PF][R], pf[PF][R];
    auto issue = [&](int tt, C *dx, C *df) {
        const bool pv = bc ? true : (tt >= 0 && tt < n);
        const bool load = pv && tt <= tload;
        int gz = tt;
        if (bc) { gz = tt % n; if (gz < 0) gz += n; }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C vx = C(0), vf = C(0);
            if (load && live[r]) {
                const int64_t g = int64_t(gz) * plane + coff[r];
                vf = St<S>::ld(a.f + g);
                if (PRE != PRE_ZERO) vx = St<S>::ld(a.xin + g);
            }
            dx[r] = vx;
            df[r] = vf;
        }
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) issue(t0 + k, px[k], pf[k]);

    for (int t = t0; t <= t1; ++t) {
        const int sl = t & 1, ps = sl ^ 1;
        // ---------------------------------------------------------- stage 0
        {
            const bool pv = bc ? true : (t >= 0 && t < n);
            const bool load = pv && t <= tload;
            int gz = t;
            if (bc) { gz = t % n; if (gz < 0) gz += n; }
            C cx_[R], cf_[R];
#pragma unroll
            for (int r = 0; r < R; ++r) { cx_[r] = px[0][r]; cf_[r] = pf[0][r]; }
#pragma unroll
            for (int k = 0; k + 1 < PF; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) { px[k][r] = px[k + 1][r]; pf[k][r] = pf[k + 1][r]; }
            issue(t + PF, px[PF - 1], pf[PF - 1]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                C s0 = C(0), fv = C(0);
                if (load && live[r]) {
                    fv = cf_[r];
                    if (PRE == PRE_ZERO) {
                        s0 = a.wdiag * fv;
                    } else {
                        s0 = cx_[r];
                        if (PRE == PRE_PROLONG) {
                            const int gxx = int(coff[r] & (n - 1));
                            const int gyy = D == 3 ? int(coff[r] >> lg) : gz;
                            s0 = s0 + prolong_at<D, S>(a.ec, gxx, gyy, D == 3 ? gz : 0, lg, bc);
                        }
                    }
                }
#pragma unroll
                for (int k = H; k > 0; --k) fq[r][k] = fq[r][k - 1];
                fq[r][0] = fv;
                q[0][r][0] = q[0][r][1];
                q[0][r][1] = q[0][r][2];
                q[0][r][2] = s0;
                if (cidx[r] >= 0 && NST > 0) lds[0][sl][cidx[r]] = s0;
            }
        }
        // ------------------------------------------- stencil stages 1..H
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int p = t - j;
            const bool pv = bc ? true : (p >= 0 && p < n);
            const bool isres = RES && j == H;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                C out = C(0);
                if (pv && live[r]) {
                    const int c = cidx[r];
                    const C xc = q[j - 1][r][1];
                    const C* L = lds[j - 1][ps];
                    const int cx = c % TX;
                    const C xm = (bnd[r] & 1) ? -xc : L[cx > 0 ? c - 1 : c];
                    const C xp = (bnd[r] & 2) ? -xc : L[cx < TX - 1 ? c + 1 : c];
                    C s;
                    if (D == 3) {
                        const int cy = c / TX;
                        const C ym = (bnd[r] & 4) ? -xc : L[cy > 0 ? c - TX : c];
                        const C yp = (bnd[r] & 8) ? -xc : L[cy < TY - 1 ? c + TX : c];
                        const C zm = (!bc && p == 0) ? -xc : q[j - 1][r][0];
                        const C zp = (!bc && p == n - 1) ? -xc : q[j - 1][r][2];
                        s = ((((xm + xp) + ym) + yp) + zm) + zp;
                    } else {
                        const C ym = (!bc && p == 0) ? -xc : q[j - 1][r][0];
                        const C yp = (!bc && p == n - 1) ? -xc : q[j - 1][r][2];
                        s = ((xm + xp) + ym) + yp;
                    }
                    const C res = fq[r][j] - (C(2 * D) * xc - s) * a.inv_h2;
                    if (NORM && j == 1 && own[r] && p >= z0 && p < zend) nacc += double(res) * double(res);
                    out = isres ? res : xc + a.wdiag * res;
                }
                if (!isres) {
                    q[j][r][0] = q[j][r][1];
                    q[j][r][1] = q[j][r][2];
                    q[j][r][2] = out;
                }
                if (cidx[r] >= 0) {
                    if (j < NST) lds[j][sl][cidx[r]] = out;
                    else if (isres) lds[NST][sl][cidx[r]] = out;
                }
                // write the smoothed iterate
                if (j == NJ && !isres && own[r] && pv && p >= z0 && p < zend)
                    St<S>::st(a.xout + int64_t(p) * plane + coff[r], out);
            }
        }
        if (NJ == 0 && PRE != PRE_NONE) {
            // no Jacobi stage: the stage-0 value itself is the output (plane t)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (own[r] && t >= z0 && t < zend) St<S>::st(a.xout + int64_t(t) * plane + coff[r], q[0][r][2]);
        }
        // ---------------------------------------------------- restriction
        if (RES) {
            const int pr = t - 1 - H;  // residual plane published in the previous step
            if (pr >= z0 && pr < zend) {
                const C *Lr = lds[NST][ps];
#pragma unroll
                for (int k = 0; k < RC; ++k) {
                    const int cc = tid + 256 * k;
                    if (cc < NCC) {
                        const int ci = cc % (BX / 2), cj = D == 3 ? cc / (BX / 2) : 0;
                        const int fx = H + 2 * ci, fy = D == 3 ? H + 2 * cj : 0;
                        const int b = fy * TX + fx;
                        C sum = Lr[b] + Lr[b + 1];
                        if (D == 3) sum = sum + Lr[b + TX] + Lr[b + TX + 1];
                        if (((pr - z0) & 1) == 0) {
                            racc[k] = sum;
                        } else {
                            const int Ic = (x0 >> 1) + ci, Jc = D == 3 ? (y0 >> 1) + cj : 0;
                            const int nc = n >> 1;
                            if (Ic < nc && Jc < nc) {
                                const int64_t gc = D == 3
                                    ? (int64_t(pr >> 1) * nc + Jc) * nc + Ic
                                    : int64_t(pr >> 1) * nc + Ic;
                                St<S>::st(a.fc + gc, (racc[k] + sum) * C(D == 3 ? 0.125 : 0.25));
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (NORM) {
        nacc = block_sum(nacc);
        if (tid == 0) a.partial[blockIdx.x] = nacc;
    }
}

}  // namespace np
