// Temporally blocked 3D level kernels for the small levels (32^3 and 64^3 by
// default), where each of a level's kernels costs about a launch:
//  - k_down0_b: the two weighted-Jacobi sweeps from a zero iterate, the
//               residual and its restriction (the down-leg of a level whose
//               correction starts from zero);
//  - k_up2_b:   prolongation + correction and the two post-sweeps (the up-leg).
// A workgroup of B^3 threads owns a B^3 block of cells and reads its operands
// once, with a two-cell ring, into LDS; each stage is then one LDS pass over
// the block and the ring it needs.  Ring values outside the grid follow the
// boundary rule: periodic grids compute them as ordinary cells at the wrapped
// position; a Dirichlet stage takes minus the value of the mirror cell (the
// adjacent interior cell).  Every stage does the arithmetic of the per-kernel
// path on these levels in the same term order (k_sweep, k_restrict /
// k_resid_restrict, k_psweep3) and rounds to the storage precision where that
// path stores: the results equal it bit for bit.
#pragma once

#include "mg_level.h"

namespace np {

// Boundary rule along one axis for a position g at most two cells outside
// [0, n): the cell whose value it holds (periodic: wrapped; Dirichlet: the
// mirror about the face, with the sign flipped).
__device__ __forceinline__ int bmap(int g, int n, int bc, int &sgn) {
    if (g < 0) {
        if (bc) return g + n;
        sgn = -sgn;
        return -1 - g;
    }
    if (g >= n) {
        if (bc) return g - n;
        sgn = -sgn;
        return 2 * n - 1 - g;
    }
    return g;
}

// Block of B^3 cells and its one- and two-cell rings; NT_ threads (B^3 or more: the ring
// stages then take fewer passes per thread).
template <int B, int NT_ = B * B * B> struct BTile {
    static_assert(NT_ >= B * B * B, "a thread per block cell");
    static constexpr int NT = NT_;
    static constexpr int W1 = B + 2, R1 = W1 * W1 * W1, W2 = B + 4, R2 = W2 * W2 * W2;
    static constexpr int U1 = (R1 + NT - 1) / NT, U2 = (R2 + NT - 1) / NT;
};

// Block of workgroup blk on a level of n = 2^lg cells per axis: its first cell.
template <int B>
__device__ __forceinline__ void block_origin(int n, int &x0, int &y0, int &z0) {
    const int nb = n / B, blk = int(xcd_block(blockIdx.x, gridDim.x));
    x0 = (blk % nb) * B;
    y0 = ((blk / nb) % nb) * B;
    z0 = (blk / (nb * nb)) * B;
}

// Cell e of a cubic region of width W around the block (ring cells on each
// side): its position relative to the block origin.
__device__ __forceinline__ void region_pos(int e, int W, int ring, int &a, int &b, int &c) {
    a = e % W - ring;
    b = (e / W) % W - ring;
    c = e / (W * W) - ring;
}

// Where a stage is evaluated for region position (a, b, c) of a block at
// (x0, y0, z0): periodic: the position itself; Dirichlet: the mirror of a
// position outside the grid, with sign -1 (0 when it is outside along two or
// more axes: such ghosts are never read by a 7-point stage).
__device__ __forceinline__ int eval_pos(int &a, int &b, int &c, int x0, int y0, int z0, int n, int bc) {
    if (bc) return 1;
    int sa = 1, sb = 1, sc = 1;
    a = bmap(x0 + a, n, 0, sa) - x0;
    b = bmap(y0 + b, n, 0, sb) - y0;
    c = bmap(z0 + c, n, 0, sc) - z0;
    const int outs = (sa < 0) + (sb < 0) + (sc < 0);
    return outs == 0 ? 1 : (outs == 1 ? -1 : 0);
}

// Down-leg from zero on a block: x2 (two sweeps from zero) on the block and a
// one-cell ring from f on a two-cell ring, x2 stored; the residuals of the
// block's cells; their restriction, summed per coarse cell in the order of
// k_restrict (z, then y, then x children, from zero).
template <class S, int B, int NTH = B * B * B>
__global__ __launch_bounds__(NTH) void k_down0_b(const S *__restrict__ f, S *__restrict__ xout,
                                                          S *__restrict__ fc, int lg, int bc,
                                                          typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                          const int *stop) {
    typedef typename St<S>::C C;
    typedef BTile<B, NTH> T;
    constexpr int NT = T::NT, W1 = T::W1, W2 = T::W2, Q2 = W2 * W2, Q1 = W1 * W1;
    __shared__ C F[T::R2];     // f, boundary rule applied
    __shared__ C X[T::R1];     // x2
    __shared__ C Rr[B * B * B];  // residuals of the block's cells
    if (stop && *stop) return;
    const int n = 1 << lg, t = int(threadIdx.x);
    int x0, y0, z0;
    block_origin<B>(n, x0, y0, z0);
    for (int u = 0; u < T::U2; ++u) {
        const int e = t + u * NT;
        if (e >= T::R2) break;
        int a, b, c, s = 1;
        region_pos(e, W2, 2, a, b, c);
        const int gi = bmap(x0 + a, n, bc, s), gj = bmap(y0 + b, n, bc, s), gk = bmap(z0 + c, n, bc, s);
        F[e] = C(s) * St<S>::ld(f + ((int64_t(gk) << lg) + gj) * n + gi);
    }
    __syncthreads();
    for (int u = 0; u < T::U1; ++u) {
        const int e = t + u * NT;
        if (e >= T::R1) break;
        int a, b, c;
        region_pos(e, W1, 1, a, b, c);
        const bool own = a >= 0 && a < B && b >= 0 && b < B && c >= 0 && c < B;
        const int sgn = eval_pos(a, b, c, x0, y0, z0, n, bc);
        C v = C(0);
        if (sgn != 0) {
            const int q = ((c + 2) * W2 + b + 2) * W2 + a + 2;
            // x1 = w f formed per value, each product a statement of its own (k_sweep's zero-start pair)
            const C fcv = F[q];
            const C xc = wdiag * fcv;
            const C xm = wdiag * F[q - 1];
            const C xp = wdiag * F[q + 1];
            const C ym = wdiag * F[q - W2];
            const C yp = wdiag * F[q + W2];
            const C zm = wdiag * F[q - Q2];
            const C zp = wdiag * F[q + Q2];
            C s = ((xm + xp) + ym) + yp;
            s = (s + zm) + zp;
            const C r = fcv - (C(6) * xc - s) * inv_h2;
            v = C(sgn) * st_round<S>(xc + wdiag * r);
        }
        X[e] = v;
        if (own) St<S>::st(xout + ((int64_t(z0 + c) << lg) + y0 + b) * n + x0 + a, v);
    }
    __syncthreads();
    if (t < B * B * B) {
        const int a = t % B, b = (t / B) % B, c = t / (B * B);
        const int q = ((c + 1) * W1 + b + 1) * W1 + a + 1;
        const C xc = X[q];
        C s = ((X[q - 1] + X[q + 1]) + X[q - W1]) + X[q + W1];
        s = (s + X[q - Q1]) + X[q + Q1];
        Rr[t] = F[((c + 2) * W2 + b + 2) * W2 + a + 2] - (C(6) * xc - s) * inv_h2;
    }
    __syncthreads();
    constexpr int BC = B / 2;
    if (t < BC * BC * BC) {
        const int I = t % BC, J = (t / BC) % BC, K = t / (BC * BC);
        C acc = C(0);
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) acc += Rr[((2 * K + cz) * B + 2 * J + cy) * B + 2 * I + cx];
        const int nc = n >> 1;
        St<S>::st(fc + ((int64_t((z0 >> 1) + K) * nc + (y0 >> 1) + J) * nc + (x0 >> 1) + I), acc * C(0.125));
    }
}

// Up-leg on a block: x' = x + P ec on the block and a two-cell ring (formed at
// each position, ghosts from the coarse ghosts, as k_psweep3 does), the first
// sweep on the block and a one-cell ring (Dirichlet ghosts minus the mirror),
// the second sweep on the block, stored.
template <class S, int B, int NTH = B * B * B>
__global__ __launch_bounds__(NTH) void k_up2_b(const S *__restrict__ ec, const S *__restrict__ f,
                                                        const S *__restrict__ xin, S *__restrict__ xout, int lg,
                                                        int bc, typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                        const int *stop) {
    typedef typename St<S>::C C;
    typedef BTile<B, NTH> T;
    constexpr int NT = T::NT, W1 = T::W1, W2 = T::W2, Q2 = W2 * W2, Q1 = W1 * W1;
    constexpr int CW = B / 2 + 4, CR = CW * CW * CW;  // coarse cells of the region and their neighbours
    __shared__ C E[CR];
    __shared__ C Xp[T::R2];  // x'
    __shared__ C Y[T::R1];   // first sweep
    if (stop && *stop) return;
    const int n = 1 << lg, nc = n >> 1, lgc = lg - 1, t = int(threadIdx.x);
    int x0, y0, z0;
    block_origin<B>(n, x0, y0, z0);
    const int X0 = x0 >> 1, Y0 = y0 >> 1, Z0 = z0 >> 1;
    for (int e = t; e < CR; e += NT) {
        int a, b, c, s = 1;
        region_pos(e, CW, 2, a, b, c);
        const int gi = bmap(X0 + a, nc, bc, s), gj = bmap(Y0 + b, nc, bc, s), gk = bmap(Z0 + c, nc, bc, s);
        E[e] = C(s) * St<S>::ld(ec + ((int64_t(gk) << lgc) + gj) * nc + gi);
    }
    C raw[T::U2];
    for (int u = 0; u < T::U2; ++u) {
        const int e = t + u * NT;
        int a, b, c, s = 1;
        region_pos(e < T::R2 ? e : 0, W2, 2, a, b, c);
        const int gi = bmap(x0 + a, n, bc, s), gj = bmap(y0 + b, n, bc, s), gk = bmap(z0 + c, n, bc, s);
        raw[u] = C(s) * St<S>::ld(xin + ((int64_t(gk) << lg) + gj) * n + gi);
    }
    __syncthreads();
    for (int u = 0; u < T::U2; ++u) {
        const int e = t + u * NT;
        if (e >= T::R2) break;
        int a, b, c;
        region_pos(e, W2, 2, a, b, c);
        // own coarse cell and the neighbour on the fine cell's side, per axis (region coordinates)
        const int fx = x0 + a, fy = y0 + b, fz = z0 + c;
        const int lx = (fx >> 1) - X0 + 2, nx = lx + ((fx & 1) ? 1 : -1);
        const int ly = (fy >> 1) - Y0 + 2, ny = ly + ((fy & 1) ? 1 : -1);
        const int lz = (fz >> 1) - Z0 + 2, nz = lz + ((fz & 1) ? 1 : -1);
        auto bil = [&](int zz) -> C {
            const C *P0 = E + zz * CW * CW;
            return wpair(wpair(P0[ly * CW + lx], P0[ly * CW + nx]), wpair(P0[ny * CW + lx], P0[ny * CW + nx]));
        };
        Xp[e] = st_round<S>(raw[u] + prolong_mix(bil(lz), bil(nz)));
    }
    __syncthreads();
    for (int u = 0; u < T::U1; ++u) {
        const int e = t + u * NT;
        if (e >= T::R1) break;
        int a, b, c;
        region_pos(e, W1, 1, a, b, c);
        const int sgn = eval_pos(a, b, c, x0, y0, z0, n, bc);
        C v = C(0);
        if (sgn != 0) {
            int s = 1;
            const int gi = bmap(x0 + a, n, bc, s), gj = bmap(y0 + b, n, bc, s), gk = bmap(z0 + c, n, bc, s);
            const C fcv = St<S>::ld(f + ((int64_t(gk) << lg) + gj) * n + gi);
            const int q = ((c + 2) * W2 + b + 2) * W2 + a + 2;
            const C xc = Xp[q];
            C sm = ((Xp[q - 1] + Xp[q + 1]) + Xp[q - W2]) + Xp[q + W2];
            sm = (sm + Xp[q - Q2]) + Xp[q + Q2];
            const C r = fcv - (C(6) * xc - sm) * inv_h2;
            v = C(sgn) * st_round<S>(xc + wdiag * r);
        }
        Y[e] = v;
    }
    __syncthreads();
    if (t < B * B * B) {
        const int a = t % B, b = (t / B) % B, c = t / (B * B);
        const int64_t g = ((int64_t(z0 + c) << lg) + y0 + b) * n + x0 + a;
        const int q = ((c + 1) * W1 + b + 1) * W1 + a + 1;
        const C xc = Y[q];
        C s = ((Y[q - 1] + Y[q + 1]) + Y[q - W1]) + Y[q + W1];
        s = (s + Y[q - Q1]) + Y[q + Q1];
        const C r = St<S>::ld(f + g) - (C(6) * xc - s) * inv_h2;
        St<S>::st(xout + g, xc + wdiag * r);
    }
}

}  // namespace np
