// Temporally blocked 3D level kernels on z-marching tiles: several steps of
// the V-cycle on one level in a single pass over its fields.
//  - k_down0_3: the two weighted-Jacobi sweeps from a zero iterate, the
//               residual and its restriction (the whole down-leg of a level
//               whose correction starts from zero);
//  - k_up2_3:   prolongation + correction and the two post-sweeps (the whole
//               up-leg of a level).
// A workgroup owns a TX x TY column tile and zc consecutive planes and marches
// along z.  Each stage is computed one plane behind the previous one; a
// stage whose results the next reads as in-plane neighbours covers the tile
// and a ring around it.  Operands come from rings of planes in LDS; the
// global loads of a plane are issued a step before it is used.  Ring values
// outside the grid follow the boundary rule: periodic grids compute them as
// ordinary cells at the wrapped position; Dirichlet grids take minus the
// value of the mirror cell (the adjacent interior cell, per axis).  Every
// stage does the arithmetic of the per-kernel path in the same term order and
// rounds to the storage precision where that path stores, so the results
// equal the z-marching per-kernel path (k_sweep3, k_restrict3, k_psweep3)
// bit for bit.
#pragma once

#include "mg_level.h"

namespace np {

// Tile of a fused kernel: TX x TY interior columns, NT = (TX / 2) (TY / 2)
// threads (one coarse column each where a stage works per coarse cell); R1 /
// R2: the tile with a one- / two-cell ring.
template <int TX, int TY> struct FTile {
    static constexpr int NT = (TX / 2) * (TY / 2);
    static constexpr int W1 = TX + 2, H1 = TY + 2, R1 = W1 * H1;
    static constexpr int W2 = TX + 4, H2 = TY + 4, R2 = W2 * H2;
    static constexpr int U1 = (R1 + NT - 1) / NT, U2 = (R2 + NT - 1) / NT;
    static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
};

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

// Tile rows of the fused kernels: 16 for 4- and 2-byte storage, 8 for FP64
// (LDS); the tile is 128 columns wide on levels of 128^3 and more, the
// level's width below.
template <class S> struct FCfg {
    static constexpr int TY = sizeof(S) == 8 ? 8 : 16;
};

// Where a stage is evaluated for cell e of a ring region of width W around the
// tile: the tile position (for a Dirichlet ring cell outside the grid, that of
// its mirror) and the sign applied (-1 for a mirrored cell, 0 for a corner
// ghost, which no stage reads).
struct RCell {
    int a, b, sgn;
};
__device__ __forceinline__ RCell ring_cell(int e, int W, int ring, int x0, int y0, int n, int bc) {
    RCell r;
    const int a = e % W - ring, b = e / W - ring;
    int sa = 1, sb = 1;
    r.a = bc ? a : bmap(x0 + a, n, 0, sa) - x0;
    r.b = bc ? b : bmap(y0 + b, n, 0, sb) - y0;
    r.sgn = (sa < 0 && sb < 0) ? 0 : sa * sb;
    return r;
}

// ---------------------------------------------------------------- down-leg
// x2 = two weighted-Jacobi sweeps of A x = f from x = 0 (x1 = w f formed from
// f, x2 = x1 + w (f - A x1) stored), then fc = R (f - A x2), the restricted
// residual (coarse cell = 1/8 of the sum of its children, summed in the order
// of k_restrict3).  Stage 1 (x2 on the tile and its ring) runs one plane ahead
// of stage 2 (residuals of a pair of fine planes and their restriction, one
// coarse cell per thread).  Rings: f on three planes with a two-cell ring, x2
// on four planes with a one-cell ring.  zc even.  Equals k_sweep3<S, false,
// true> then k_restrict3<S> bit for bit.
template <class S, int TX, int TY>
__global__ __launch_bounds__((FTile<TX, TY>::NT)) void k_down0_3(const S *__restrict__ f, S *__restrict__ xout,
                                                                 S *__restrict__ fc, int lg, int bc, int zc,
                                                                 typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                                 const int *stop) {
    typedef typename St<S>::C C;
    typedef FTile<TX, TY> T;
    constexpr int NT = T::NT, W1 = T::W1, W2 = T::W2, CXN = TX / 2, U1 = T::U1, U2 = T::U2;
    __shared__ S Fr[3][T::R2];  // f (signed by the boundary rule), slot = plane mod 3
    __shared__ S Xr[4][T::R1];  // x2, slot = plane mod 4
    if (stop && *stop) return;
    const int n = 1 << lg, ntx = n / TX, nty = n / TY;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
    const int x0 = bx * TX, y0 = by * TY, k0 = bz * zc;
    const int64_t P = int64_t(1) << (2 * lg);
    const int t = int(threadIdx.x);
    auto fs = [](int q) { return (q + 6) % 3; };
    auto xs = [](int q) { return (q + 8) & 3; };
    // this thread's cells of the two-ring region: in-plane source and sign
    int src[U2];
    C sg[U2];
    for (int u = 0; u < U2; ++u) {
        const int e = t + u * NT;
        int s = 1;
        const int gi = bmap(x0 + (e % W2) - 2, n, bc, s), gj = bmap(y0 + (e / W2) - 2, n, bc, s);
        src[u] = e < T::R2 ? (gj << lg) + gi : 0;
        sg[u] = C(s);
    }
    // stage-1 cells: R2-frame index of the evaluated position, sign, store offset (-1: not own)
    int c1[U1], st1[U1];
    C s1[U1];
    for (int u = 0; u < U1; ++u) {
        const int e = t + u * NT;
        const RCell r = ring_cell(e < T::R1 ? e : 0, W1, 1, x0, y0, n, bc);
        const int a = e % W1 - 1, b = e / W1 - 1;
        c1[u] = (r.b + 2) * W2 + r.a + 2;
        s1[u] = C(r.sgn);
        st1[u] = (e < T::R1 && a >= 0 && a < TX && b >= 0 && b < TY) ? ((y0 + b) << lg) + x0 + a : -1;
    }
    // planes whose f is read: periodic all, Dirichlet the grid and one ghost plane on each side
    auto needf = [&](int q) { return bc || (q >= -1 && q <= n); };
    auto real = [&](int q) { return bc || (q >= 0 && q < n); };
    C fv[2][U2];  // f of two planes in flight
    auto fload = [&](int q, C (&v)[U2]) {
        int s = 1;
        const int64_t base = int64_t(bmap(q, n, bc, s)) * P;
        for (int u = 0; u < U2; ++u) v[u] = C(s) * sg[u] * St<S>::ld(f + base + src[u]);
    };
    auto fstore = [&](int q, const C (&v)[U2]) {
        for (int u = 0; u < U2; ++u) {
            const int e = t + u * NT;
            if (e < T::R2) St<S>::st(&Fr[fs(q)][e], v[u]);
        }
    };
    // stage 1: x2 on plane p (as k_sweep3's pass of the first two sweeps from zero)
    auto stage1 = [&](int p) {
        if (!real(p)) return;
        const bool own = p >= k0 && p < k0 + zc;
        const S *F0 = Fr[fs(p)], *Fm = Fr[fs(p - 1)], *Fp = Fr[fs(p + 1)];
        for (int u = 0; u < U1; ++u) {
            const int e = t + u * NT;
            if (e >= T::R1) break;
            const int c = c1[u];
            // each product a statement of its own, as the per-kernel path forms them
            const C fcv = St<S>::ld(F0 + c);
            const C xc = wdiag * fcv;
            const C xm = wdiag * St<S>::ld(F0 + c - 1);
            const C xp = wdiag * St<S>::ld(F0 + c + 1);
            const C ym = wdiag * St<S>::ld(F0 + c - W2);
            const C yp = wdiag * St<S>::ld(F0 + c + W2);
            const C zm = wdiag * St<S>::ld(Fm + c);
            const C zp = wdiag * St<S>::ld(Fp + c);
            const C t0 = ((xm + xp) + ym) + yp;
            const C s = (t0 + zm) + zp;
            const C r = fcv - (C(6) * xc - s) * inv_h2;
            const C v = s1[u] * st_round<S>(xc + wdiag * r);
            St<S>::st(&Xr[xs(p)][e], v);
            if (own && st1[u] >= 0) St<S>::st(xout + int64_t(p) * P + st1[u], v);
        }
    };
    // stage 2: the residuals of fine planes pa and pa + 1 and their restriction
    const int cx = t % CXN, cy = t / CXN;
    const int g2 = ((y0 + 2 * cy) << lg) + x0 + 2 * cx;  // in-plane offset of the first child
    C fr[2][2][2];  // f at the eight children [plane][row][column]
    auto fload2 = [&](int pa) {
        for (int z = 0; z < 2; ++z)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) fr[z][b][a] = St<S>::ld(f + int64_t(pa + z) * P + g2 + (b << lg) + a);
    };
    auto xr = [&](int q, int c) -> C {  // x2 ring value on plane q (Dirichlet ghost planes by the mirror)
        if (!bc && q < 0) return -St<S>::ld(&Xr[xs(0)][c]);
        if (!bc && q >= n) return -St<S>::ld(&Xr[xs(n - 1)][c]);
        return St<S>::ld(&Xr[xs(q)][c]);
    };
    auto resid = [&](int a, int b, int z, int pa) -> C {
        const int q = pa + z, c = (2 * cy + b + 1) * W1 + 2 * cx + a + 1;
        const S *X0 = Xr[xs(q)];
        const C xc = St<S>::ld(X0 + c);
        const C t0 = ((St<S>::ld(X0 + c - 1) + St<S>::ld(X0 + c + 1)) + St<S>::ld(X0 + c - W1)) + St<S>::ld(X0 + c + W1);
        const C s = (t0 + xr(q - 1, c)) + xr(q + 1, c);
        return fr[z][b][a] - (C(6) * xc - s) * inv_h2;
    };
    auto stage2 = [&](int pa) {
        C tsum;
        if constexpr (sizeof(S) == 2) {
            // k_restrict3 with two cells per thread: x pair, then z pair, then y pair
            C pr[2];
            for (int b = 0; b < 2; ++b) {
                C r0 = resid(0, b, 0, pa);
                r0 += resid(1, b, 0, pa);
                C r1 = resid(0, b, 1, pa);
                r1 += resid(1, b, 1, pa);
                C pair = r0;
                pair += r1;
                pr[b] = pair;
            }
            tsum = pr[0] + pr[1];
        } else {
            // one cell per thread: z pair per child column, then x, y
            C pz[2][2];
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    C pair = resid(a, b, 0, pa);
                    pair += resid(a, b, 1, pa);
                    pz[b][a] = pair;
                }
            tsum = ((pz[0][0] + pz[0][1]) + pz[1][0]) + pz[1][1];
        }
        const int lgc = lg - 1;
        const int64_t cc = (int64_t(pa >> 1) << (2 * lgc)) + (int64_t((y0 >> 1) + cy) << lgc) + (x0 >> 1) + cx;
        St<S>::st(fc + cc, tsum * C(0.125));
    };
    // stage 2 runs at steps p = k0 + 2, k0 + 4, ..., k0 + zc on the pair (p - 2, p - 1)
    auto two = [&](int p) { return p >= k0 + 2 && p <= k0 + zc && ((p - k0) & 1) == 0; };
    // prologue: f planes k0 - 2 .. k0 in the ring, plane k0 + 1 in flight
    for (int q = k0 - 2; q <= k0; ++q)
        if (needf(q)) {
            fload(q, fv[0]);
            fstore(q, fv[0]);
        }
    if (needf(k0 + 1)) fload(k0 + 1, fv[(k0 + 1) & 1]);
    __syncthreads();
    for (int p = k0 - 1; p <= k0 + zc; ++p) {
        // loads a step ahead: f plane p + 3 (stored at step p + 1), the children of step p + 1's stage 2
        const int qn = p + 3;
        if (qn <= k0 + zc + 1 && needf(qn)) fload(qn, fv[qn & 1]);
        if (two(p + 1)) fload2(p - 1);
        stage1(p);
        __syncthreads();
        if (two(p)) stage2(p - 2);
        // plane p + 2 (loaded a step ago) into the slot of plane p - 1, last read by stage 1 above
        if (p + 2 <= k0 + zc + 1 && needf(p + 2)) fstore(p + 2, fv[(p + 2) & 1]);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ up-leg
// xout = two weighted-Jacobi sweeps of A x = f from x' = x + P ec (the
// corrected iterate, cell-centred trilinear prolongation of the coarse
// correction ec).  Stage 0 forms x' on the tile and a two-cell ring (rounded
// to the storage precision as the per-kernel path stores it), stage 1 the
// first sweep on the tile and a one-cell ring, stage 2 the second sweep on
// the tile, each one plane behind the previous.  x' at a ring position outside
// the grid is formed at that position, from the raw iterate by the boundary
// rule and the correction from the coarse ghosts (as k_psweep3 forms its
// ghosts); the first sweep at a Dirichlet ring position outside the grid is
// minus that of its mirror (as the per-kernel second sweep reads it).  Rings
// in LDS: coarse planes (four), x' (three planes, two-cell ring), first sweep
// (three planes, one-cell ring).  zc even.  Equals k_psweep3<S> then
// k_sweep3<S, false> bit for bit.
template <class S, int TX, int TY>
__global__ __launch_bounds__((FTile<TX, TY>::NT)) void k_up2_3(const S *__restrict__ ec, const S *__restrict__ f,
                                                               const S *__restrict__ xin, S *__restrict__ xout,
                                                               int lg, int bc, int zc, typename St<S>::C inv_h2,
                                                               typename St<S>::C wdiag, const int *stop) {
    typedef typename St<S>::C C;
    typedef FTile<TX, TY> T;
    constexpr int NT = T::NT, W1 = T::W1, W2 = T::W2, U1 = T::U1, U2 = T::U2;
    constexpr int CW = TX / 2 + 4, CH = TY / 2 + 4, CR = CW * CH;  // coarse ring: tile +- 2 coarse cells
    constexpr int UC = (CR + NT - 1) / NT, U3 = TX * TY / NT;
    __shared__ S Er[4][CR];     // coarse planes, slot = plane mod 4
    __shared__ S Xr[3][T::R2];  // x', slot = plane mod 3
    __shared__ S Yr[3][T::R1];  // first sweep, slot = plane mod 3
    if (stop && *stop) return;
    const int n = 1 << lg, nc = n >> 1, lgc = lg - 1, ntx = n / TX, nty = n / TY;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
    const int x0 = bx * TX, y0 = by * TY, k0 = bz * zc, X0 = x0 >> 1, Y0 = y0 >> 1;
    const int64_t P = int64_t(1) << (2 * lg), Pc = int64_t(1) << (2 * lgc);
    const int t = int(threadIdx.x);
    auto es = [](int K) { return (K + 8) & 3; };
    auto rs = [](int q) { return (q + 6) % 3; };
    // coarse ring cells of this thread: in-plane source and sign
    int csrc[UC];
    C csg[UC];
    for (int u = 0; u < UC; ++u) {
        const int e = t + u * NT;
        int s = 1;
        const int gi = bmap(X0 + e % CW - 2, nc, bc, s), gj = bmap(Y0 + e / CW - 2, nc, bc, s);
        csrc[u] = e < CR ? (gj << lgc) + gi : 0;
        csg[u] = C(s);
    }
    C ev[UC];
    auto eload = [&](int K) {
        int s = 1;
        const int64_t base = int64_t(bmap(K, nc, bc, s)) * Pc;
        for (int u = 0; u < UC; ++u) ev[u] = C(s) * csg[u] * St<S>::ld(ec + base + csrc[u]);
    };
    auto estore = [&](int K) {
        for (int u = 0; u < UC; ++u) {
            const int e = t + u * NT;
            if (e < CR) St<S>::st(&Er[es(K)][e], ev[u]);
        }
    };
    // two-ring cells of this thread: raw-iterate source and sign, coarse ring columns and rows
    // (own and neighbour packed: columns 8 bits each, row offsets 16 bits each)
    int src[U2], ccol[U2], crow[U2];
    C sg[U2];
    for (int u = 0; u < U2; ++u) {
        const int e = t + u * NT, a = e % W2 - 2, b = e / W2 - 2;
        int s = 1;
        const int gi = bmap(x0 + a, n, bc, s), gj = bmap(y0 + b, n, bc, s);
        const bool in = e < T::R2;
        src[u] = in ? (gj << lg) + gi : 0;
        sg[u] = C(s);
        const int fx = x0 + a, fy = y0 + b;  // ghost positions keep their own coordinates
        const int lo = (fx >> 1) - X0 + 2, ro = (fy >> 1) - Y0 + 2;
        ccol[u] = in ? lo | ((lo + ((fx & 1) ? 1 : -1)) << 8) : 0;
        crow[u] = in ? (ro * CW) | (((ro + ((fy & 1) ? 1 : -1)) * CW) << 16) : 0;
    }
    C xv[2][U2];  // raw iterate of two planes in flight
    auto xload = [&](int q, C (&v)[U2]) {
        int s = 1;
        const int64_t base = int64_t(bmap(q, n, bc, s)) * P;
        for (int u = 0; u < U2; ++u) v[u] = C(s) * sg[u] * St<S>::ld(xin + base + src[u]);
    };
    // stage 0: x' on plane q from the raw values v (k_psweep3's correction of a loaded value)
    auto stage0 = [&](int q, const C (&v)[U2]) {
        const int K = q >> 1, Kn = K + ((q & 1) ? 1 : -1);
        const S *Eo = Er[es(K)], *En = Er[es(Kn)];
        for (int u = 0; u < U2; ++u) {
            const int e = t + u * NT;
            if (e >= T::R2) break;
            const int lo = ccol[u] & 255, ln = ccol[u] >> 8, ro = crow[u] & 0xffff, rn = crow[u] >> 16;
            const C eo = wpair(wpair(St<S>::ld(Eo + ro + lo), St<S>::ld(Eo + ro + ln)),
                               wpair(St<S>::ld(Eo + rn + lo), St<S>::ld(Eo + rn + ln)));
            const C en = wpair(wpair(St<S>::ld(En + ro + lo), St<S>::ld(En + ro + ln)),
                               wpair(St<S>::ld(En + rn + lo), St<S>::ld(En + rn + ln)));
            St<S>::st(&Xr[rs(q)][e], st_round<S>(v[u] + prolong_mix(eo, en)));
        }
    };
    // stage-1 cells: R2-frame index of the evaluated position, sign, f source (in-plane)
    int c1[U1], f1[U1];
    C s1[U1];
    for (int u = 0; u < U1; ++u) {
        const int e = t + u * NT;
        const RCell r = ring_cell(e < T::R1 ? e : 0, W1, 1, x0, y0, n, bc);
        c1[u] = (r.b + 2) * W2 + r.a + 2;
        s1[u] = C(r.sgn);
        int s = 1;
        const int gi = bmap(x0 + r.a, n, bc, s), gj = bmap(y0 + r.b, n, bc, s);
        f1[u] = (gj << lg) + gi;  // periodic: wrapped; Dirichlet: the mirror, inside the grid
    }
    C fv1[2][U1];  // f of the stage-1 cells on two planes
    auto f1load = [&](int p, C (&v)[U1]) {
        int s = 1;
        const int64_t base = int64_t(bmap(p, n, bc, s)) * P;  // Dirichlet: only planes of the grid are used
        for (int u = 0; u < U1; ++u) v[u] = St<S>::ld(f + base + f1[u]);
    };
    auto stage1 = [&](int p, const C (&fv)[U1]) {
        if (!bc && (p < 0 || p >= n)) return;  // a Dirichlet ghost plane is read as minus its mirror
        const S *Lm = Xr[rs(p - 1)], *L0 = Xr[rs(p)], *Lp = Xr[rs(p + 1)];
        for (int u = 0; u < U1; ++u) {
            const int e = t + u * NT;
            if (e >= T::R1) break;
            const int c = c1[u];
            const C xc = St<S>::ld(L0 + c);
            const C t0 = ((St<S>::ld(L0 + c - 1) + St<S>::ld(L0 + c + 1)) + St<S>::ld(L0 + c - W2)) +
                         St<S>::ld(L0 + c + W2);
            const C s = (t0 + St<S>::ld(Lm + c)) + St<S>::ld(Lp + c);
            const C r = fv[u] - (C(6) * xc - s) * inv_h2;
            St<S>::st(&Yr[rs(p)][e], s1[u] * st_round<S>(xc + wdiag * r));
        }
    };
    // stage 2: second sweep on plane p, tile cells (U3 per thread), stored
    C fv2[2][U3];
    auto f2load = [&](int p, C (&v)[U3]) {
        for (int u = 0; u < U3; ++u) {
            const int e = t + u * NT;
            v[u] = St<S>::ld(f + int64_t(p) * P + ((y0 + e / TX) << lg) + x0 + e % TX);
        }
    };
    auto stage2 = [&](int p, const C (&fv)[U3]) {
        const C sm = (!bc && p == 0) ? C(-1) : C(1), sp = (!bc && p == n - 1) ? C(-1) : C(1);
        const int qm = (!bc && p == 0) ? 0 : p - 1, qp = (!bc && p == n - 1) ? n - 1 : p + 1;
        const S *Lm = Yr[rs(qm)], *L0 = Yr[rs(p)], *Lp = Yr[rs(qp)];
        for (int u = 0; u < U3; ++u) {
            const int e = t + u * NT, a = e % TX, b = e / TX, c = (b + 1) * W1 + a + 1;
            const C xc = St<S>::ld(L0 + c);
            const C t0 = ((St<S>::ld(L0 + c - 1) + St<S>::ld(L0 + c + 1)) + St<S>::ld(L0 + c - W1)) +
                         St<S>::ld(L0 + c + W1);
            const C s = (t0 + sm * St<S>::ld(Lm + c)) + sp * St<S>::ld(Lp + c);
            const C r = fv[u] - (C(6) * xc - s) * inv_h2;
            St<S>::st(xout + int64_t(p) * P + ((y0 + b) << lg) + x0 + a, xc + wdiag * r);
        }
    };
    // highest coarse plane x'(q) reads: q / 2, plus one on odd planes
    auto khi = [](int q) { return (q >> 1) + ((q & 1) ? 1 : 0); };
    // prologue: coarse planes of x'(k0 - 2), x'(k0 - 1); those two planes; loads of the first step
    for (int K = (k0 >> 1) - 2; K <= khi(k0 - 1); ++K) {
        eload(K);
        estore(K);
    }
    int kload = khi(k0 - 1);
    xload(k0 - 2, xv[0]);
    xload(k0 - 1, xv[1]);
    __syncthreads();
    stage0(k0 - 2, xv[0]);
    stage0(k0 - 1, xv[1]);
    xload(k0, xv[k0 & 1]);
    f1load(k0 - 1, fv1[(k0 - 1) & 1]);
    bool epend = false;  // a coarse plane waits in ev, to be stored before the next stage 0
    if (khi(k0) > kload) {
        eload(khi(k0));
        epend = true;
    }
    for (int p = k0 - 1; p <= k0 + zc; ++p) {
        if (epend) {
            estore(++kload);
            epend = false;
        }
        // loads for the next steps: raw plane p + 2 and the coarse plane x'(p + 2) adds, f of
        // stage 1 on plane p + 1 and of stage 2 on plane p
        if (p + 2 <= k0 + zc + 1) {
            xload(p + 2, xv[(p + 2) & 1]);
            if (khi(p + 2) > kload) {
                eload(khi(p + 2));
                epend = true;
            }
        }
        if (p + 1 <= k0 + zc) f1load(p + 1, fv1[(p + 1) & 1]);
        if (p >= k0 && p < k0 + zc) f2load(p, fv2[p & 1]);
        __syncthreads();
        stage0(p + 1, xv[(p + 1) & 1]);
        __syncthreads();
        stage1(p, fv1[p & 1]);
        __syncthreads();
        if (p - 1 >= k0) stage2(p - 1, fv2[(p - 1) & 1]);
    }
}

}  // namespace np
