// 2D level kernels on 64 x 16 blocks for the levels above the one-workgroup
// tail (128^2 .. 1024^2), where each per-cell kernel costs about a launch:
//  - MODE 0 (down-leg from a zero iterate): the two sweeps from zero (the
//    first, w f, formed per value as k_sweep's zero-start pair forms it), the
//    residual and its restriction;
//  - MODE 1 (down-leg of an iterate): two sweeps, the residual and its
//    restriction; NORM also gives the per-workgroup partial of |f - A x|^2 of
//    the input iterate (the convergence check);
//  - MODE 2 (up-leg): prolongation + correction (formed at every position it
//    is read, rounded to storage, as k_psweep forms it) and the two post-sweeps.
// A workgroup of 1024 threads reads its operands once, with the rings its
// stages need, into LDS; each stage is one LDS pass over the block and its
// ring.  Ring values outside the grid follow the boundary rule: periodic grids
// compute them as ordinary cells at the wrapped position, a Dirichlet stage
// takes minus its value at the mirror cell (the 5-point stencil reads such a
// value only next to the wall, where it is minus the cell's own).  Every stage
// does the arithmetic of the per-cell path (k_sweep, k_restrict, k_psweep) in
// the same term order and rounds to storage where that path stores: the
// results equal it bit for bit.
#pragma once

#include "mg_fused3.h"

namespace np {

template <class S> struct B2 {
    static constexpr int BX = 64, BY = 16, NT = 1024;
    static constexpr int W(int k) { return BX + 2 * k; }
    static constexpr int H(int k) { return BY + 2 * k; }
    static constexpr int R(int k) { return W(k) * H(k); }
    static constexpr int CW = BX / 2 + 4, CH = BY / 2 + 4;  // coarse cells an up-leg block reads
};

// Position (a, b) relative to the block origin of element e of the region of
// width W with `ring` cells around the block.
__device__ __forceinline__ void region_pos2(int e, int W, int ring, int &a, int &b) {
    a = e % W - ring;
    b = e / W - ring;
}

// Where a stage is evaluated for position (a, b) of a block at (x0, y0):
// periodic: the position itself (sign 1); Dirichlet: the mirror of a position
// outside the grid (sign -1), 0 for a corner outside along both axes (never
// read by a 5-point stage).
__device__ __forceinline__ int eval_pos2(int &a, int &b, int x0, int y0, int n, int bc) {
    if (bc) return 1;
    int sa = 1, sb = 1;
    a = bmap(x0 + a, n, 0, sa) - x0;
    b = bmap(y0 + b, n, 0, sb) - y0;
    const int outs = (sa < 0) + (sb < 0);
    return outs == 0 ? 1 : (outs == 1 ? -1 : 0);
}

template <class S, int MODE, bool NORM>
__global__ __launch_bounds__(B2<S>::NT) void k_lvl2_b(const S *__restrict__ ec, const S *__restrict__ f,
                                                      const S *__restrict__ xin, S *__restrict__ xout,
                                                      S *__restrict__ fc, double *__restrict__ partial, int lg,
                                                      int bc, typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                      const int *stop) {
    typedef typename St<S>::C C;
    typedef B2<S> G;
    constexpr int BX = G::BX, BY = G::BY, NT = G::NT;
    // region widths: input x on ring 3 (MODE 1) / 2 (MODE 2), f on ring 2 (down) / 1 (up)
    constexpr int WA = MODE == 1 ? G::W(3) : G::W(2), RA = MODE == 1 ? G::R(3) : G::R(2);
    constexpr int RING_A = MODE == 1 ? 3 : 2;
    constexpr int WF = MODE == 2 ? G::W(1) : G::W(2), RF = MODE == 2 ? G::R(1) : G::R(2);
    constexpr int RING_F = MODE == 2 ? 1 : 2;
    constexpr int W2 = G::W(2), W1 = G::W(1);
    // A: the input (x, or x' in the up-leg); S1: first sweep (ring 2 down, ring 1 up); S2: second
    // sweep (ring 1, down only); the block's residuals reuse A
    __shared__ C A[MODE == 0 ? 1 : (RA > BX * BY ? RA : BX * BY)];
    __shared__ C Raw[MODE == 2 ? G::R(2) : 1];
    __shared__ C Fs[RF];
    __shared__ C S1[MODE == 2 ? G::R(1) : (MODE == 1 ? G::R(2) : 1)];
    __shared__ C S2[MODE == 2 ? 1 : G::R(1)];
    __shared__ C Rr0[MODE == 0 ? BX * BY : 1];
    __shared__ C E[MODE == 2 ? G::CW * G::CH : 1];
    if (stop && *stop) return;
    const int n = 1 << lg, t = int(threadIdx.x);
    const int nbx = n / BX, blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int x0 = (blk % nbx) * BX, y0 = (blk / nbx) * BY;
    // flat index of block position (a, b) by the boundary rule, its sign into s
    auto gidx = [&](int a, int b, int &s) -> int64_t {
        const int gi = bmap(x0 + a, n, bc, s), gj = bmap(y0 + b, n, bc, s);
        return (int64_t(gj) << lg) + gi;
    };
    // ------------------------------------------------------------------ loads
    for (int e = t; e < RF; e += NT) {
        int a, b, s = 1;
        region_pos2(e, WF, RING_F, a, b);
        const int64_t g = gidx(a, b, s);
        Fs[e] = C(s) * St<S>::ld(f + g);
    }
    if constexpr (MODE == 1) {
        for (int e = t; e < RA; e += NT) {
            int a, b, s = 1;
            region_pos2(e, WA, RING_A, a, b);
            const int64_t g = gidx(a, b, s);
            A[e] = C(s) * St<S>::ld(xin + g);
        }
    }
    if constexpr (MODE == 2) {
        const int nc = n >> 1, lgc = lg - 1, X0 = x0 >> 1, Y0 = y0 >> 1;
        for (int e = t; e < G::CW * G::CH; e += NT) {
            int a, b, s = 1;
            region_pos2(e, G::CW, 2, a, b);
            const int gi = bmap(X0 + a, nc, bc, s), gj = bmap(Y0 + b, nc, bc, s);
            E[e] = C(s) * St<S>::ld(ec + (int64_t(gj) << lgc) + gi);
        }
        for (int e = t; e < G::R(2); e += NT) {
            int a, b, s = 1;
            region_pos2(e, W2, 2, a, b);
            const int64_t g = gidx(a, b, s);
            Raw[e] = C(s) * St<S>::ld(xin + g);
        }
    }
    __syncthreads();
    // -------------------------------------------------- up-leg: x' = x + P ec
    if constexpr (MODE == 2) {
        const int X0 = x0 >> 1, Y0 = y0 >> 1;
        for (int e = t; e < G::R(2); e += NT) {
            int a, b;
            region_pos2(e, W2, 2, a, b);
            const int sgn = eval_pos2(a, b, x0, y0, n, bc);
            C v = C(0);
            if (sgn != 0) {
                // own coarse cell and the neighbour on the fine cell's side, per axis, in the coarse
                // tile (ghosts already carry the boundary rule); terms and order of pro_cell
                const int fx = x0 + a, fy = y0 + b;
                const int oi = (fx >> 1) - X0 + 2, ni = oi + ((fx & 1) ? 1 : -1);
                const int oj = (fy >> 1) - Y0 + 2, nj = oj + ((fy & 1) ? 1 : -1);
                C p = C(0);
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int aa = 0; aa < 2; ++aa) {
                        const C w = C(aa ? 0.25 : 0.75) * C(bb ? 0.25 : 0.75) * C(1.0);
                        p = np_fma(w, E[(bb ? nj : oj) * G::CW + (aa ? ni : oi)], p);
                    }
                v = C(sgn) * st_round<S>(Raw[(b + 2) * W2 + a + 2] + p);
            }
            A[e] = v;
        }
        __syncthreads();
    }
    // ------------------------------------------------------- first sweep (S1)
    // down (MODE 1): on ring 2 from the input; up: on ring 1 from x'.  From zero (MODE 0) the
    // first sweep, w f, is formed where the second reads it.
    double acc = 0.0;
    if constexpr (MODE != 0) {
        constexpr int RS = MODE == 2 ? 1 : 2, WS = G::W(RS), NS = G::R(RS);
        for (int e = t; e < NS; e += NT) {
            int a, b;
            region_pos2(e, WS, RS, a, b);
            const bool own = a >= 0 && a < BX && b >= 0 && b < BY;
            const int sgn = eval_pos2(a, b, x0, y0, n, bc);
            C v = C(0);
            if (sgn != 0) {
                const C fv = Fs[(b + RING_F) * WF + a + RING_F];
                const int q = (b + RING_A) * WA + a + RING_A;
                const C xc = A[q];
                const C s = ((A[q - 1] + A[q + 1]) + A[q - WA]) + A[q + WA];
                const C r = fv - (C(4) * xc - s) * inv_h2;
                if (NORM && own) acc += double(r) * double(r);
                v = C(sgn) * st_round<S>(xc + wdiag * r);
            }
            S1[e] = v;
        }
        __syncthreads();
    }
    // ------------------------------------------------------ second sweep
    if constexpr (MODE == 2) {
        // on the block from S1 (ring 1), stored
        for (int e = t; e < BX * BY; e += NT) {
            const int a = e % BX, b = e / BX;
            const int q = (b + 1) * W1 + a + 1;
            const C xc = S1[q];
            const C s = ((S1[q - 1] + S1[q + 1]) + S1[q - W1]) + S1[q + W1];
            const C r = Fs[q] - (C(4) * xc - s) * inv_h2;
            St<S>::st(xout + (int64_t(y0 + b) << lg) + x0 + a, xc + wdiag * r);
        }
    } else {
        // on ring 1 from S1 (ring 2); MODE 0 forms each neighbour's w f as its own product, as
        // k_sweep's zero-start pair does
        for (int e = t; e < G::R(1); e += NT) {
            int a, b;
            region_pos2(e, W1, 1, a, b);
            const bool own = a >= 0 && a < BX && b >= 0 && b < BY;
            const int sgn = eval_pos2(a, b, x0, y0, n, bc);
            C v = C(0);
            if (sgn != 0) {
                const int q = (b + 2) * W2 + a + 2;
                const C fv = Fs[q];
                C xc, s;
                if constexpr (MODE == 0) {
                    xc = wdiag * fv;
                    const C xm = wdiag * Fs[q - 1];
                    const C xp = wdiag * Fs[q + 1];
                    const C ym = wdiag * Fs[q - W2];
                    const C yp = wdiag * Fs[q + W2];
                    s = ((xm + xp) + ym) + yp;
                } else {
                    xc = S1[q];
                    s = ((S1[q - 1] + S1[q + 1]) + S1[q - W2]) + S1[q + W2];
                }
                const C r = fv - (C(4) * xc - s) * inv_h2;
                v = C(sgn) * st_round<S>(xc + wdiag * r);
            }
            S2[e] = v;
            if (own && sgn != 0) St<S>::st(xout + (int64_t(y0 + b) << lg) + x0 + a, v);
        }
        __syncthreads();
        // residual of the second sweep on the block, then its restriction (k_restrict's order:
        // the y-pair outer, the x-pair inner, from zero)
        C *Rr = MODE == 0 ? Rr0 : A;
        for (int e = t; e < BX * BY; e += NT) {
            const int a = e % BX, b = e / BX;
            const int q = (b + 1) * W1 + a + 1;
            const C xc = S2[q];
            const C s = ((S2[q - 1] + S2[q + 1]) + S2[q - W1]) + S2[q + W1];
            Rr[e] = Fs[(b + 2) * W2 + a + 2] - (C(4) * xc - s) * inv_h2;
        }
        __syncthreads();
        if (t < (BX / 2) * (BY / 2)) {
            const int I = t % (BX / 2), J = t / (BX / 2), nc = n >> 1;
            C r = C(0);
#pragma unroll
            for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                for (int cx = 0; cx < 2; ++cx) r += Rr[(2 * J + cy) * BX + 2 * I + cx];
            St<S>::st(fc + (int64_t((y0 >> 1) + J) * nc + (x0 >> 1) + I), r * C(0.25));
        }
        if constexpr (NORM) {
            acc = block_sum_n<NT>(acc);
            if (threadIdx.x == 0) partial[blockIdx.x] = acc;
        }
    }
}

}  // namespace np
