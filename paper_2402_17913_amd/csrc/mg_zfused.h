// Two Jacobi sweeps in one pass over a large 3D level (n >= 128) on z-marching
// tiles:
//   xout = sweep(sweep(x'))  with  x' = x + P ec  (CORR: the up-leg's
//   prolongation + correction and both post-sweeps) or x' = x (the down-leg's
//   two pre-sweeps; NORM: also the per-workgroup partial of |f - A x|^2, the
//   convergence check of the input iterate).
// A workgroup of kS3Threads threads owns a TX x TY column tile (32 threads per
// row, CPT cells each) and zc planes.  The first sweep is formed on the tile
// and on the one-cell ring around it one plane ahead of the second sweep, which
// reads that ring as in-plane neighbours.  Each thread holds its own cells'
// x' at z - 1, z, z + 1 and first sweep at z - 2 .. z in registers; the first
// waves also carry one cell each of the one-cell ring (x' at z - 1 .. z + 1 and
// f, first sweep formed there), the last waves one cell each of the two-cell
// ring (x' at z only, an in-plane neighbour of the first sweep): ring work
// falls on whole waves (lanes past the ring's end repeat its last cell, which
// writes the same value twice), so the roles branch on the wave, not on lanes.
// In-plane neighbours come from LDS.  The loop takes planes in odd/even pairs,
// so which coarse planes a correction mixes, and which LDS slot a plane uses,
// are fixed at compile time; plane indices map through the boundary rule
// without branches, values are loaded two steps before the end of the step that
// consumes (and signs) them, in two register sets named by the plane's parity,
// and Dirichlet ghosts of the second sweep are selected over unconditional LDS
// reads.
// Ring cells outside the grid take x' at that position from the raw iterate by
// the boundary rule plus the correction from the coarse ghosts, as k_psweep3
// forms its halo; the second sweep reads a Dirichlet ghost as minus the cell's
// own first-sweep value, as the per-kernel sweep does.  A correction is
// prolong_mix of two coarse planes' in-plane values at the cell; each coarse
// plane's value is formed once per position and kept while fine planes use it.
// Same arithmetic and term order as k_psweep3 (or k_sweep3) then k_sweep3: the
// result equals that pair bit for bit.  Offsets are 32-bit (n <= 1024).
#pragma once

#include "mg_level.h"
#include "mg_fused3.h"

namespace np {

template <class S> struct Z2Cfg {
    static constexpr int CPT = ZCfg<S>::CPT, TP = 32, TX = TP * CPT, TY = kS3Threads / TP;
    static constexpr int W1 = TX + 2, H1 = TY + 2, W2 = TX + 4, H2 = TY + 4;
    static constexpr int NR1 = 2 * (TX + 2) + 2 * TY;        // ring-1 cells
    static constexpr int NR2 = 2 * (TX + 4) + 2 * (TY + 2);  // ring-2 cells
    static constexpr int NW = kS3Threads / 64;               // waves per workgroup
    static constexpr int NW1 = (NR1 + 63) / 64, NW2 = (NR2 + 63) / 64;  // waves carrying ring 1 / ring 2
    static constexpr int CW = TX / 2 + 4, CH = TY / 2 + 4, CR = CW * CH;  // coarse cells the region reads
    static_assert(NW1 + NW2 <= NW, "ring-1 and ring-2 slots on distinct waves");
    static_assert(CR <= kS3Threads, "one coarse cell per thread");
    static_assert(TX * TY == kS3Threads * CPT, "tile of one cell group per thread");
};

// Tile position (a, b) of ring cell r of the ring at distance `ring` around a
// TX x TY tile: the row above, the row below (both with their corners), then
// the left and the right column.
template <int TX, int TY>
__device__ __forceinline__ void ring_pos(int r, int ring, int &a, int &b) {
    const int w = TX + 2 * ring, h = TY + 2 * (ring - 1);
    if (r < w) { a = r - ring; b = -ring; return; }
    r -= w;
    if (r < w) { a = r - ring; b = TY + ring - 1; return; }
    r -= w;
    if (r < h) { a = -ring; b = r - (ring - 1); return; }
    r -= h;
    a = TX + ring - 1;
    b = r - (ring - 1);
}

// LDS offsets, within a coarse plane tile, of the four coarse cells that the
// in-plane bilinear value at fine tile position (a, b) mixes (x0, y0 even).
template <int CW>
__device__ __forceinline__ void coarse_offsets(int a, int b, int (&o)[4]) {
    const int lo = (a >> 1) + 2, ln = lo + ((a & 1) ? 1 : -1);
    const int ro = ((b >> 1) + 2) * CW, rn = ro + ((b & 1) ? CW : -CW);
    o[0] = ro + lo;
    o[1] = ro + ln;
    o[2] = rn + lo;
    o[3] = rn + ln;
}

template <class C>
__device__ __forceinline__ C coarse_mix(const C *E, const int (&o)[4]) {
    return wpair(wpair(E[o[0]], E[o[1]]), wpair(E[o[2]], E[o[3]]));
}

// Plane q in [-n - 1, 2n - 2] of an n-plane axis by the boundary rule, without
// branches: periodic wraps; Dirichlet mirrors (-1 - q below, 2n - 1 - q above)
// and flips the sign.
__device__ __forceinline__ int plane_map(int q, int n, int bc, bool &flip) {
    const int kp = (q + n) & (n - 1);
    const int kd = min(max(q, -1 - q), 2 * n - 1 - q);
    flip = !bc && kd != q;
    return bc ? kp : kd;
}

// Planes per workgroup of k_sweep2z on an n^3 level: each chunk re-reads a few
// planes of x and f above and below it, so chunks are as long as still gives
// `wg` workgroups -- four per CU (1024), or two (512) for the kernels that fit
// fewer than four per CU (the up-leg in every precision and FP64's zero-start
// down-leg: at 256^3 one round of two per CU beat a second round at a third of
// the occupancy) -- and at least four planes (measured: at 128^3 BF16, 512
// workgroups of four planes beat 1024 of two); the tuning knob "zc3" overrides.
inline int z2_planes(int lg, int tx, int ty, int wg = 1024) {
    const int n = 1 << lg;
    const int64_t tiles = (int64_t(n) / tx) * (n / ty);
    int zc = 4;
    while (zc < n && tiles * (n / (2 * zc)) >= wg) zc *= 2;
    if (g_zc3 >= 2 && g_zc3 <= n) zc = g_zc3;
    return zc;
}
template <class S> inline int sweep2z_planes(int lg, int wg = 1024) {
    return z2_planes(lg, Z2Cfg<S>::TX, Z2Cfg<S>::TY, wg);
}

template <class S, bool CORR, bool NORM>
__global__ __launch_bounds__(kS3Threads) void k_sweep2z(const S *__restrict__ ec, const S *__restrict__ f,
                                                        const S *__restrict__ xin, S *__restrict__ xout,
                                                        double *__restrict__ partial, int lg, int bc, int zc,
                                                        typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                        const int *stop) {
    typedef typename St<S>::C C;
    typedef Z2Cfg<S> G;
    constexpr int TX = G::TX, TY = G::TY, CPT = G::CPT, TP = G::TP, W1 = G::W1, W2 = G::W2, CW = G::CW;
    constexpr int BS = G::H1 * W1;          // one first-sweep plane in LDS
    constexpr int AS = G::H2 * W2;          // one x' plane in LDS
    // one barrier per plane step, x' of planes z - 1 and z in two slots (the second sweep reads
    // the first sweep of the previous step).  Measured at 256^3 and 128^3 (average per launch):
    // FP32 up-leg 25.5 -> 24.5 us, BF16 up-leg 24.4 -> 23.4, BF16 down-leg 30.1 -> 28.8.  In FP64
    // it takes the up-leg past 128 VGPRs (one workgroup per CU): at 512 workgroups 47.8 against
    // 50.5 us, but launched as 256 workgroups (one round) the FP64 solve measured 5.99 -> 5.90 ms
    // (two barriers at 256: 5.92 ms)
    constexpr bool ONE = true;
    __shared__ C Ax[(ONE ? 2 : 1) * AS];    // x' of plane z (ONE: slot = plane & 1), tile and two-cell ring
    __shared__ C Bs[2 * BS];                // first sweep of planes z - 1, z (slot = plane & 1), tile and ring
    __shared__ C Ec[CORR ? 4 : 1][CORR ? G::CR + 1 : 1];  // coarse planes (slot = plane & 3), one spare cell
    if (stop && *stop) return;
    const int n = 1 << lg, nc = n >> 1, ntx = n / TX, nty = n / TY;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP, ai = CPT * tp;
    const int x0 = (blk % ntx) * TX, y0 = ((blk / ntx) % nty) * TY, k0 = (blk / (ntx * nty)) * zc;
    const int pl = 2 * lg;  // log2 of a plane's cells
    const uint32_t osrc = (uint32_t(y0 + ty) << lg) + uint32_t(x0 + ai);  // own cells, in-plane
    // ring role of this thread's wave: 1 (one-cell ring), 2 (two-cell ring) or none
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool r1 = wv < G::NW1, r2 = wv >= G::NW - G::NW2;
    int ra = 0, rb = 0;
    if (r1) ring_pos<TX, TY>(min(t, G::NR1 - 1), 1, ra, rb);
    if (r2) ring_pos<TX, TY>(min(t - 64 * (G::NW - G::NW2), G::NR2 - 1), 2, ra, rb);
    uint32_t rsrc;
    C rsg;
    {
        int s = 1;
        const int gi = bmap(x0 + ra, n, bc, s), gj = bmap(y0 + rb, n, bc, s);
        rsrc = (uint32_t(gj) << lg) + uint32_t(gi);
        rsg = C(s);
    }
    const int own_a = (ty + 2) * W2 + ai + 2;    // Ax offset of the first own cell
    const int own_b = (ty + 1) * W1 + ai + 1;    // Bs offset of the first own cell
    const int ring_a = (rb + 2) * W2 + ra + 2;   // Ax offset of the ring cell
    const int ring_b = (rb + 1) * W1 + ra + 1;   // Bs offset (ring 1)
    // Dirichlet walls next to the own cells (the second sweep's ghosts)
    bool dw[CPT], de[CPT];
    for (int c = 0; c < CPT; ++c) {
        dw[c] = !bc && x0 + ai + c == 0;
        de[c] = !bc && x0 + ai + c == n - 1;
    }
    const bool ds = !bc && y0 + ty == 0, dn = !bc && y0 + ty == n - 1;
    auto poff = [&](int q, C &sg) -> uint32_t {  // offset of plane q and the sign of its values
        bool flip;
        const int k = plane_map(q, n, bc, flip);
        sg = flip ? C(-1) : C(1);
        return uint32_t(k) << pl;
    };
    auto ld_own = [&](const S *base, C (&v)[CPT]) {
        if constexpr (CPT == 2) Pair<S>::ld(base + osrc, v[0], v[1]);
        else v[0] = St<S>::ld(base + osrc);
    };

    // coarse staging and the kept in-plane values: for a position corrected at fine plane q,
    // m0 / m1 hold coarse planes kk, kk + 1 with kk = floor((q - 1) / 2)
    int oco[CPT][4], rco[4];
    C m0[CPT], m1[CPT], rm0 = C(0), rm1 = C(0);
    uint32_t csrc = 0;
    C csg = C(1), ev = C(0);
    const int ce = min(t, G::CR);  // this thread's coarse cell (the spare cell past the region)
    if constexpr (CORR) {
        for (int c = 0; c < CPT; ++c) coarse_offsets<CW>(ai + c, ty, oco[c]);
        coarse_offsets<CW>(ra, rb, rco);
        int s = 1;
        const int gi = bmap((x0 >> 1) + t % CW - 2, nc, bc, s), gj = bmap((y0 >> 1) + t / CW - 2, nc, bc, s);
        csrc = t < G::CR ? (uint32_t(gj) << (lg - 1)) + uint32_t(gi) : 0u;
        csg = C(s);
    }
    auto eload = [&](int K) {  // this thread's cell of coarse plane K, in flight
        bool flip;
        const int k = plane_map(K, nc, bc, flip);
        ev = (flip ? -csg : csg) * St<S>::ld(ec + (uint32_t(k) << (pl - 2)) + csrc);
    };
    auto estore = [&](int K) { Ec[K & 3][ce] = ev; };
    // x' from a signed raw value at fine plane q: own coarse plane first (ODD: q odd)
    auto corr = [&](C v, C a0, C a1, auto odd) -> C {
        if constexpr (decltype(odd)::value) return st_round<S>(v + prolong_mix(a0, a1));
        else return st_round<S>(v + prolong_mix(a1, a0));
    };
    // a sweep at an LDS position of plane z (in-plane neighbours from Ax), z-neighbours given
    auto sweep1 = [&](const C *A, int q, C xc, C xm, C xp, C fv, C &r) -> C {
        const C t0 = ((A[q - 1] + A[q + 1]) + A[q - W2]) + A[q + W2];
        const C s = (t0 + xm) + xp;
        r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };

    // registers: own x' at z - 1, z, z + 1; first sweep at z - 2 .. z; f at z, z - 1; ring values
    C xo[3][CPT], so[2][CPT], fo[2][CPT];
    C rx0 = C(0), rx1 = C(0), rx2 = C(0), rf = C(0);  // ring 1: x' at z - 1 .. z + 1, f at z; ring 2: rx1
    // loads in flight for the step of parity u: own x(z + 2) and f(z + 1), ring x (z + 2 on ring 1,
    // z + 1 on ring 2) and f(z + 1) (ring 1)
    C pw[2][CPT], pf[2][CPT], prr[2] = {C(0), C(0)}, prf[2] = {C(0), C(0)};
    for (int c = 0; c < CPT; ++c) so[0][c] = so[1][c] = fo[1][c] = C(0);
    auto psign = [&](int q) -> C {  // sign of plane q's values by the boundary rule
        return (!bc && (q < 0 || q >= n)) ? C(-1) : C(1);
    };
    // the loads that the step at plane z consumes, into set u; past the last planes used (x up to
    // k0 + zc + 1, f and ring-2 x up to k0 + zc) the last one is read again, an L2 hit
    auto pload = [&](int z, auto u) {
        constexpr int U = decltype(u)::value;
        C sg;
        const uint32_t o2 = poff(min(z + 2, k0 + zc + 1), sg), o1 = poff(min(z + 1, k0 + zc), sg);
        ld_own(xin + o2, pw[U]);
        ld_own(f + o1, pf[U]);
        // every wave loads (a wave without a ring cell reads its tile's first cell, unused): a load
        // under a branch would keep the set's old value alive and cost register copies
        prr[U] = St<S>::ld(xin + (r1 ? o2 : o1) + rsrc);
        prf[U] = St<S>::ld(f + o1 + rsrc);
    };
    // ---------------------------------------------------------------- prologue
    const int K0 = k0 >> 1, Kmax = (k0 + zc + 2) >> 1;  // coarse planes the chunk's corrections use
    if constexpr (CORR) {
        for (int K = K0 - 2; K <= K0 + 1; ++K) {
            eload(K);
            estore(K);
        }
    }
    pload(k0 - 1, std::integral_constant<int, 1>{});
    for (int z = 0; z < 3; ++z) {
        C sg;
        const uint32_t o = poff(k0 - 2 + z, sg);
        ld_own(xin + o, xo[z]);
        for (int c = 0; c < CPT; ++c) xo[z][c] *= sg;
        if (r1) {
            const C v = sg * rsg * St<S>::ld(xin + o + rsrc);
            if (z == 0) rx0 = v;
            else if (z == 1) rx1 = v;
            else rx2 = v;
        }
    }
    {
        C sg;
        const uint32_t o = poff(k0 - 1, sg);
        if (r2) rx1 = sg * rsg * St<S>::ld(xin + o + rsrc);
        ld_own(f + o, fo[0]);
        if (r1) rf = St<S>::ld(f + o + rsrc);
    }
    if constexpr (CORR) {
        __syncthreads();
        // own and ring 1: planes k0 - 2 (coarse K0 - 2, K0 - 1), k0 - 1 and k0 (K0 - 1, K0)
        for (int c = 0; c < CPT; ++c) {
            m0[c] = coarse_mix(Ec[(K0 - 2) & 3], oco[c]);
            m1[c] = coarse_mix(Ec[(K0 - 1) & 3], oco[c]);
            xo[0][c] = corr(xo[0][c], m0[c], m1[c], std::false_type{});
            m0[c] = m1[c];
            m1[c] = coarse_mix(Ec[K0 & 3], oco[c]);
            xo[1][c] = corr(xo[1][c], m0[c], m1[c], std::true_type{});
            xo[2][c] = corr(xo[2][c], m0[c], m1[c], std::false_type{});
        }
        if (r1) {
            rm0 = coarse_mix(Ec[(K0 - 2) & 3], rco);
            rm1 = coarse_mix(Ec[(K0 - 1) & 3], rco);
            rx0 = corr(rx0, rm0, rm1, std::false_type{});
            rm0 = rm1;
            rm1 = coarse_mix(Ec[K0 & 3], rco);
            rx1 = corr(rx1, rm0, rm1, std::true_type{});
            rx2 = corr(rx2, rm0, rm1, std::false_type{});
        }
        if (r2) {  // plane k0 - 1 (coarse K0 - 1, K0)
            rm0 = coarse_mix(Ec[(K0 - 1) & 3], rco);
            rm1 = coarse_mix(Ec[K0 & 3], rco);
            rx1 = corr(rx1, rm0, rm1, std::true_type{});
        }
    }
    double acc = 0.0;
    // ------------------------------------------------------------------- march
    // one step: first sweep of plane z, second sweep of plane z - 1; ODD = z odd
    auto step = [&](int z, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        constexpr int U = ODD ? 1 : 0;
        typedef std::integral_constant<bool, !ODD> Even;
        if constexpr (CORR && ODD) {
            if (z > k0) estore((z + 3) >> 1);  // loaded two steps ago
            eload(min((z + 5) >> 1, Kmax));
        }
        pload(z + 1, std::integral_constant<int, 1 - U>{});  // for the next step
        // x' of plane z into LDS
        C *A = Ax + (ONE && ODD ? AS : 0);
        for (int c = 0; c < CPT; ++c) A[own_a + c] = xo[1][c];
        if (r1 || r2) A[ring_a] = rx1;
        __syncthreads();
        // first sweep of plane z: own cells and the ring-1 cell (values at Dirichlet ghosts are
        // formed too, and never selected)
        C *B = Bs + (ODD ? BS : 0);
        C sn[CPT];
        for (int c = 0; c < CPT; ++c) {
            C r;
            sn[c] = st_round<S>(sweep1(A, own_a + c, xo[1][c], xo[0][c], xo[2][c], fo[0][c], r));
            if (NORM && z >= k0 && z < k0 + zc) acc += double(r) * double(r);
            B[own_b + c] = sn[c];
        }
        if (r1) {
            C r;
            B[ring_b] = st_round<S>(sweep1(A, ring_a, rx1, rx0, rx2, rf, r));
        }
        if constexpr (!ONE) __syncthreads();
        // second sweep of plane z - 1, own cells (its first sweep was written by the previous step)
        if (z > k0) {
            const int p = z - 1;
            const C *L = Bs + (ODD ? 0 : BS);
            const bool dzl = !bc && p == 0, dzu = !bc && p == n - 1;
            C out[CPT];
            for (int c = 0; c < CPT; ++c) {
                const int q = own_b + c;
                const C xc = so[1][c];
                const C lw = L[q - 1], le = L[q + 1], ls = L[q - W1], ln = L[q + W1];
                // Dirichlet ghosts: minus the cell's own value
                const C xw = dw[c] ? -xc : lw;
                const C xe = de[c] ? -xc : le;
                const C ys = ds ? -xc : ls;
                const C yn = dn ? -xc : ln;
                const C zl = dzl ? -xc : so[0][c];
                const C zu = dzu ? -xc : sn[c];
                const C t0 = ((xw + xe) + ys) + yn;
                const C s = (t0 + zl) + zu;
                const C r = fo[1][c] - (C(6) * xc - s) * inv_h2;
                out[c] = xc + wdiag * r;
            }
            store_cells<S, CPT>(xout + (uint32_t(p) << pl) + osrc, out);
        }
        // slide: the first sweep, f, and x' (the loads signed and corrected now)
        const C sg2 = psign(z + 2), sg1 = psign(z + 1);
        for (int c = 0; c < CPT; ++c) {
            so[0][c] = so[1][c];
            so[1][c] = sn[c];
            fo[1][c] = fo[0][c];
            fo[0][c] = pf[U][c];
            xo[0][c] = xo[1][c];
            xo[1][c] = xo[2][c];
        }
        if constexpr (CORR) {
            if constexpr (ODD)  // x'(z + 2), z + 2 odd: coarse plane (z + 3) / 2 joins
                for (int c = 0; c < CPT; ++c) {
                    m0[c] = m1[c];
                    m1[c] = coarse_mix(Ec[((z + 3) >> 1) & 3], oco[c]);
                }
            for (int c = 0; c < CPT; ++c) xo[2][c] = corr(sg2 * pw[U][c], m0[c], m1[c], odd);
        } else {
            for (int c = 0; c < CPT; ++c) xo[2][c] = sg2 * pw[U][c];
        }
        if (r1) {
            rx0 = rx1;
            rx1 = rx2;
            rf = prf[U];
            const C v = (sg2 * rsg) * prr[U];
            if constexpr (CORR) {
                if constexpr (ODD) {
                    rm0 = rm1;
                    rm1 = coarse_mix(Ec[((z + 3) >> 1) & 3], rco);
                }
                rx2 = corr(v, rm0, rm1, odd);
            } else {
                rx2 = v;
            }
        }
        if (r2) {  // x'(z + 1), z + 1 odd when z is even: coarse plane (z + 2) / 2 joins
            const C v = (sg1 * rsg) * prr[U];
            if constexpr (CORR) {
                if constexpr (!ODD) {
                    rm0 = rm1;
                    rm1 = coarse_mix(Ec[((z + 2) >> 1) & 3], rco);
                }
                rx1 = corr(v, rm0, rm1, Even{});
            } else {
                rx1 = v;
            }
        }
    };
    // k0 even: pairs (odd, even); the last step loads nothing, the one before it no coarse plane
    for (int z = k0 - 1; z < k0 + zc; z += 2) {  // k0 even: pairs (odd, even)
        step(z, std::true_type{});
        step(z + 1, std::false_type{});
    }
    if constexpr (NORM) {
        acc = block_sum_n<kS3Threads>(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// The down-leg of a large 3D level (n >= 128) from a zero iterate in one pass on
// the same tiles: x2 = sweep(sweep(0)) and fc = R (f - A x2).  The first sweep
// from zero is x1 = w f (pointwise, unrounded, as the per-kernel sweep forms
// it); the second sweep is formed on the tile and the one-cell ring, one plane
// ahead of the residual, which needs that ring as in-plane neighbours; x2 is
// stored (rounded) and its residual summed over the 2 x 2 x 2 children of each
// coarse cell in k_restrict3's order -- the cell pair of a thread (CPT = 2),
// then the plane pair, then the row pair (and, CPT = 1, the column pair) by
// lane shuffles inside the wave (rows ty and ty + 1 are lanes 32 apart).  Same
// arithmetic and term order as k_sweep3 from zero then k_restrict3: both
// outputs equal that pair bit for bit.
template <class S>
__global__ __launch_bounds__(kS3Threads) void k_down0z(const S *__restrict__ f, S *__restrict__ xout,
                                                       S *__restrict__ fc, int lg, int bc, int zc,
                                                       typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                       const int *stop) {
    typedef typename St<S>::C C;
    typedef Z2Cfg<S> G;
    constexpr int TX = G::TX, TY = G::TY, CPT = G::CPT, TP = G::TP, W1 = G::W1, W2 = G::W2;
    constexpr int BS = G::H1 * W1;
    static_assert(TP == 32, "rows ty, ty + 1 are the two halves of a wave");
    __shared__ C Ax[G::H2 * W2];  // x1 = w f of plane z, tile and two-cell ring
    __shared__ C Bs[2 * BS];      // x2 of planes z - 1, z (slot = plane & 1), tile and ring
    if (stop && *stop) return;
    const int n = 1 << lg, ntx = n / TX, nty = n / TY, lgc = lg - 1;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP, ai = CPT * tp;
    const int x0 = (blk % ntx) * TX, y0 = ((blk / ntx) % nty) * TY, k0 = (blk / (ntx * nty)) * zc;
    const int pl = 2 * lg;
    const uint32_t osrc = (uint32_t(y0 + ty) << lg) + uint32_t(x0 + ai);
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool r1 = wv < G::NW1, r2 = wv >= G::NW - G::NW2;
    int ra = 0, rb = 0;
    if (r1) ring_pos<TX, TY>(min(t, G::NR1 - 1), 1, ra, rb);
    if (r2) ring_pos<TX, TY>(min(t - 64 * (G::NW - G::NW2), G::NR2 - 1), 2, ra, rb);
    uint32_t rsrc;
    C rsg;
    {
        int s = 1;
        const int gi = bmap(x0 + ra, n, bc, s), gj = bmap(y0 + rb, n, bc, s);
        rsrc = (uint32_t(gj) << lg) + uint32_t(gi);
        rsg = C(s);
    }
    const int own_a = (ty + 2) * W2 + ai + 2, own_b = (ty + 1) * W1 + ai + 1;
    const int ring_a = (rb + 2) * W2 + ra + 2, ring_b = (rb + 1) * W1 + ra + 1;
    bool dw[CPT], de[CPT];
    for (int c = 0; c < CPT; ++c) {
        dw[c] = !bc && x0 + ai + c == 0;
        de[c] = !bc && x0 + ai + c == n - 1;
    }
    const bool ds = !bc && y0 + ty == 0, dn = !bc && y0 + ty == n - 1;
    auto poff = [&](int q) -> uint32_t {
        bool flip;
        return uint32_t(plane_map(q, n, bc, flip)) << pl;
    };
    auto psign = [&](int q) -> C { return (!bc && (q < 0 || q >= n)) ? C(-1) : C(1); };
    auto ld_own = [&](const S *base, C (&v)[CPT]) {
        if constexpr (CPT == 2) Pair<S>::ld(base + osrc, v[0], v[1]);
        else v[0] = St<S>::ld(base + osrc);
    };
    auto sweep1 = [&](int q, C xc, C xm, C xp, C fv) -> C {
        const C t0 = ((Ax[q - 1] + Ax[q + 1]) + Ax[q - W2]) + Ax[q + W2];
        const C s = (t0 + xm) + xp;
        const C r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // registers: own f at z - 1 .. z + 1 and x1 = (signed) w f there; x2 at z - 2, z - 1;
    // ring 1: the same at its cell; ring 2: x1 at z
    C fo[3][CPT], xo[3][CPT], so[2][CPT];
    C rf[3] = {C(0), C(0), C(0)}, rx[3] = {C(0), C(0), C(0)};
    C pf[2][CPT], pr[2] = {C(0), C(0)};  // loads in flight (set = parity of the consuming step)
    for (int c = 0; c < CPT; ++c) so[0][c] = so[1][c] = C(0);
    // the step at plane z consumes own / ring-1 f(z + 2) and ring-2 f(z + 1); past the planes
    // used (up to k0 + zc + 1 and k0 + zc) the last one is read again, an L2 hit
    auto pload = [&](int z, auto u) {
        constexpr int U = decltype(u)::value;
        const uint32_t o2 = poff(min(z + 2, k0 + zc + 1)), o1 = poff(min(z + 1, k0 + zc));
        ld_own(f + o2, pf[U]);
        pr[U] = St<S>::ld(f + (r1 ? o2 : o1) + rsrc);
    };
    // prologue: f at k0 - 2 .. k0 (own, ring 1), k0 - 1 (ring 2)
    for (int z = 0; z < 3; ++z) {
        const int q = k0 - 2 + z;
        ld_own(f + poff(q), fo[z]);
        const C sg = psign(q);
        for (int c = 0; c < CPT; ++c) xo[z][c] = sg * (wdiag * fo[z][c]);
        if (r1) {
            rf[z] = St<S>::ld(f + poff(q) + rsrc);
            rx[z] = (sg * rsg) * (wdiag * rf[z]);
        }
    }
    if (r2) {
        const C v = St<S>::ld(f + poff(k0 - 1) + rsrc);
        rx[1] = (psign(k0 - 1) * rsg) * (wdiag * v);
    }
    pload(k0 - 1, std::integral_constant<int, 1>{});
    C pair = C(0);  // residual sum of the plane pair
    auto step = [&](int z, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        constexpr int U = ODD ? 1 : 0;
        pload(z + 1, std::integral_constant<int, 1 - U>{});
        // x1 of plane z into LDS (own cells at z are fo[1] / xo[1])
        for (int c = 0; c < CPT; ++c) Ax[own_a + c] = xo[1][c];
        if (r1 || r2) Ax[ring_a] = rx[1];
        __syncthreads();
        // second sweep at plane z: own cells and the ring-1 cell; own values stored
        C *B = Bs + (ODD ? BS : 0);
        C sn[CPT];
        for (int c = 0; c < CPT; ++c) {
            sn[c] = st_round<S>(sweep1(own_a + c, xo[1][c], xo[0][c], xo[2][c], fo[1][c]));
            B[own_b + c] = sn[c];
        }
        if (z >= k0 && z < k0 + zc) store_cells<S, CPT>(xout + (uint32_t(z) << pl) + osrc, sn);
        if (r1) B[ring_b] = st_round<S>(sweep1(ring_a, rx[1], rx[0], rx[2], rf[1]));
        __syncthreads();
        // residual of x2 at plane p = z - 1, own cells, summed into the coarse cells
        if (z > k0) {
            const int p = z - 1;
            const C *L = Bs + (ODD ? 0 : BS);
            const bool dzl = !bc && p == 0, dzu = !bc && p == n - 1;
            C r = C(0);
            for (int c = 0; c < CPT; ++c) {
                const int q = own_b + c;
                const C xc = so[1][c];
                const C lw = L[q - 1], le = L[q + 1], ls = L[q - W1], ln = L[q + W1];
                const C xw = dw[c] ? -xc : lw;
                const C xe = de[c] ? -xc : le;
                const C ys = ds ? -xc : ls;
                const C yn = dn ? -xc : ln;
                const C zl = dzl ? -xc : so[0][c];
                const C zu = dzu ? -xc : sn[c];
                const C t0 = ((xw + xe) + ys) + yn;
                const C s = (t0 + zl) + zu;
                const C rc = fo[0][c] - (C(6) * xc - s) * inv_h2;
                if (c == 0) r = rc;
                else r += rc;
            }
            if (ODD) {  // p even: the first plane of the pair
                pair = r;
            } else {
                pair += r;
                const uint32_t cc = (uint32_t(p >> 1) << (2 * lgc)) + (uint32_t((y0 + ty) >> 1) << lgc) +
                                    uint32_t((x0 + ai) >> 1);
                if constexpr (CPT == 2) {
                    const C o = __shfl_down(pair, 32);
                    if ((ty & 1) == 0) St<S>::st(fc + cc, (pair + o) * C(0.125));
                } else {
                    const C b = __shfl_down(pair, 1), cy = __shfl_down(pair, 32),
                            d = __shfl_down(pair, 33);
                    if (((tp | ty) & 1) == 0) St<S>::st(fc + cc, (((pair + b) + cy) + d) * C(0.125));
                }
            }
        }
        // slide
        const C sg2 = psign(z + 2), sg1 = psign(z + 1);
        for (int c = 0; c < CPT; ++c) {
            so[0][c] = so[1][c];
            so[1][c] = sn[c];
            fo[0][c] = fo[1][c];
            fo[1][c] = fo[2][c];
            fo[2][c] = pf[U][c];
            xo[0][c] = xo[1][c];
            xo[1][c] = xo[2][c];
            xo[2][c] = sg2 * (wdiag * pf[U][c]);
        }
        if (r1) {
            rf[0] = rf[1];
            rf[1] = rf[2];
            rf[2] = pr[U];
            rx[0] = rx[1];
            rx[1] = rx[2];
            rx[2] = (sg2 * rsg) * (wdiag * pr[U]);
        }
        if (r2) rx[1] = (sg1 * rsg) * (wdiag * pr[U]);
    };
    for (int z = k0 - 1; z < k0 + zc; z += 2) {  // k0 even: pairs (odd, even)
        step(z, std::true_type{});
        step(z + 1, std::false_type{});
    }
}

// k_down0z with one barrier per plane step: the second sweep runs one plane
// behind the first (at z - 1, reading x1 of that plane from the other of two
// LDS slots) and the residual one plane behind it (at z - 2, reading x2 from
// the slot the previous step filled), so every LDS read of a step comes from a
// slot written before the previous step's barrier.  Same tiles, arithmetic and
// term order: the outputs equal k_down0z's bit for bit.
template <class S>
__global__ __launch_bounds__(kS3Threads) void k_down0z1(const S *__restrict__ f, S *__restrict__ xout,
                                                        S *__restrict__ fc, int lg, int bc, int zc,
                                                        typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                        const int *stop) {
    typedef typename St<S>::C C;
    typedef Z2Cfg<S> G;
    constexpr int TX = G::TX, TY = G::TY, CPT = G::CPT, TP = G::TP, W1 = G::W1, W2 = G::W2;
    constexpr int AS = G::H2 * W2, BS = G::H1 * W1;
    static_assert(TP == 32, "rows ty, ty + 1 are the two halves of a wave");
    __shared__ C Ax[2 * AS];  // x1 = w f of planes z - 1, z (slot = plane & 1), tile and two-cell ring
    __shared__ C Bs[2 * BS];  // x2 of planes z - 2, z - 1 (slot = plane & 1), tile and ring
    if (stop && *stop) return;
    const int n = 1 << lg, ntx = n / TX, nty = n / TY, lgc = lg - 1;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP, ai = CPT * tp;
    const int x0 = (blk % ntx) * TX, y0 = ((blk / ntx) % nty) * TY, k0 = (blk / (ntx * nty)) * zc;
    const int pl = 2 * lg;
    const uint32_t osrc = (uint32_t(y0 + ty) << lg) + uint32_t(x0 + ai);
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool r1 = wv < G::NW1, r2 = wv >= G::NW - G::NW2;
    int ra = 0, rb = 0;
    if (r1) ring_pos<TX, TY>(min(t, G::NR1 - 1), 1, ra, rb);
    if (r2) ring_pos<TX, TY>(min(t - 64 * (G::NW - G::NW2), G::NR2 - 1), 2, ra, rb);
    uint32_t rsrc;
    C rsg;
    {
        int s = 1;
        const int gi = bmap(x0 + ra, n, bc, s), gj = bmap(y0 + rb, n, bc, s);
        rsrc = (uint32_t(gj) << lg) + uint32_t(gi);
        rsg = C(s);
    }
    const int own_a = (ty + 2) * W2 + ai + 2, own_b = (ty + 1) * W1 + ai + 1;
    const int ring_a = (rb + 2) * W2 + ra + 2, ring_b = (rb + 1) * W1 + ra + 1;
    bool dw[CPT], de[CPT];
    for (int c = 0; c < CPT; ++c) {
        dw[c] = !bc && x0 + ai + c == 0;
        de[c] = !bc && x0 + ai + c == n - 1;
    }
    const bool ds = !bc && y0 + ty == 0, dn = !bc && y0 + ty == n - 1;
    auto poff = [&](int q) -> uint32_t {
        bool flip;
        return uint32_t(plane_map(q, n, bc, flip)) << pl;
    };
    auto psign = [&](int q) -> C { return (!bc && (q < 0 || q >= n)) ? C(-1) : C(1); };
    auto ld_own = [&](const S *base, C (&v)[CPT]) {
        if constexpr (CPT == 2) Pair<S>::ld(base + osrc, v[0], v[1]);
        else v[0] = St<S>::ld(base + osrc);
    };
    auto sweep1 = [&](const C *A, int q, C xc, C xm, C xp, C fv) -> C {
        const C t0 = ((A[q - 1] + A[q + 1]) + A[q - W2]) + A[q + W2];
        const C s = (t0 + xm) + xp;
        const C r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // registers at the start of step z: own f and x1 = (signed) w f at z - 2 .. z, x2 at
    // z - 3, z - 2; ring cells (both rings) the same f and x1 at their cell
    C fo[3][CPT], xo[3][CPT], so[2][CPT];
    C rf[3] = {C(0), C(0), C(0)}, rx[3] = {C(0), C(0), C(0)};
    C pf[2][CPT], pr[2] = {C(0), C(0)};  // loads in flight (set = parity of the issuing step)
    for (int c = 0; c < CPT; ++c) so[0][c] = so[1][c] = fo[0][c] = xo[0][c] = C(0);
    // f of plane z (own and ring cells), consumed at the end of step z - 1; past the last
    // plane used (k0 + zc + 1) the last one is read again, an L2 hit
    auto pload = [&](int z, auto u) {
        constexpr int U = decltype(u)::value;
        const uint32_t o = poff(min(z, k0 + zc + 1));
        ld_own(f + o, pf[U]);
        pr[U] = St<S>::ld(f + o + rsrc);
    };
    // prologue: f and x1 at k0 - 2, k0 - 1
    for (int z = 1; z < 3; ++z) {
        const int q = k0 - 3 + z;
        ld_own(f + poff(q), fo[z]);
        rf[z] = St<S>::ld(f + poff(q) + rsrc);
        const C sg = psign(q);
        for (int c = 0; c < CPT; ++c) xo[z][c] = sg * (wdiag * fo[z][c]);
        rx[z] = (sg * rsg) * (wdiag * rf[z]);
    }
    pload(k0, std::integral_constant<int, 0>{});
    C pair = C(0);  // residual sum of the plane pair
    auto step = [&](int z, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        constexpr int U = ODD ? 1 : 0;
        pload(z + 2, std::integral_constant<int, U>{});
        // x1 of plane z into its slot
        C *A = Ax + (ODD ? AS : 0);
        for (int c = 0; c < CPT; ++c) A[own_a + c] = xo[2][c];
        if (r1 || r2) A[ring_a] = rx[2];
        C sn[CPT];
        if (z >= k0) {
            // second sweep at plane z - 1 from x1 there (the other slot): own cells and the ring-1 cell
            const C *Am = Ax + (ODD ? 0 : AS);
            C *B = Bs + (ODD ? 0 : BS);
            for (int c = 0; c < CPT; ++c) {
                sn[c] = st_round<S>(sweep1(Am, own_a + c, xo[1][c], xo[0][c], xo[2][c], fo[1][c]));
                B[own_b + c] = sn[c];
            }
            if (z > k0 && z <= k0 + zc) store_cells<S, CPT>(xout + (uint32_t(z - 1) << pl) + osrc, sn);
            if (r1) B[ring_b] = st_round<S>(sweep1(Am, ring_a, rx[1], rx[0], rx[2], rf[1]));
        } else {
            for (int c = 0; c < CPT; ++c) sn[c] = C(0);
        }
        // residual of x2 at plane p = z - 2 (its slot was filled before the last barrier),
        // own cells, summed into the coarse cells
        if (z >= k0 + 2) {
            const int p = z - 2;
            const C *L = Bs + (ODD ? BS : 0);
            const bool dzl = !bc && p == 0, dzu = !bc && p == n - 1;
            C r = C(0);
            for (int c = 0; c < CPT; ++c) {
                const int q = own_b + c;
                const C xc = so[1][c];
                const C lw = L[q - 1], le = L[q + 1], ls = L[q - W1], ln = L[q + W1];
                const C xw = dw[c] ? -xc : lw;
                const C xe = de[c] ? -xc : le;
                const C ys = ds ? -xc : ls;
                const C yn = dn ? -xc : ln;
                const C zl = dzl ? -xc : so[0][c];
                const C zu = dzu ? -xc : sn[c];
                const C t0 = ((xw + xe) + ys) + yn;
                const C s = (t0 + zl) + zu;
                const C rc = fo[0][c] - (C(6) * xc - s) * inv_h2;
                if (c == 0) r = rc;
                else r += rc;
            }
            if (!ODD) {  // p even: the first plane of the pair
                pair = r;
            } else {
                pair += r;
                const uint32_t cc = (uint32_t(p >> 1) << (2 * lgc)) + (uint32_t((y0 + ty) >> 1) << lgc) +
                                    uint32_t((x0 + ai) >> 1);
                if constexpr (CPT == 2) {
                    const C o = __shfl_down(pair, 32);
                    if ((ty & 1) == 0) St<S>::st(fc + cc, (pair + o) * C(0.125));
                } else {
                    const C b = __shfl_down(pair, 1), cy = __shfl_down(pair, 32),
                            d = __shfl_down(pair, 33);
                    if (((tp | ty) & 1) == 0) St<S>::st(fc + cc, (((pair + b) + cy) + d) * C(0.125));
                }
            }
        }
        __syncthreads();
        // slide: f of plane z + 1 (issued by step z - 1)
        const C sg1 = psign(z + 1);
        for (int c = 0; c < CPT; ++c) {
            so[0][c] = so[1][c];
            so[1][c] = sn[c];
            fo[0][c] = fo[1][c];
            fo[1][c] = fo[2][c];
            fo[2][c] = pf[1 - U][c];
            xo[0][c] = xo[1][c];
            xo[1][c] = xo[2][c];
            xo[2][c] = sg1 * (wdiag * pf[1 - U][c]);
        }
        if (r1 || r2) {
            rf[0] = rf[1];
            rf[1] = rf[2];
            rf[2] = pr[1 - U];
            rx[0] = rx[1];
            rx[1] = rx[2];
            rx[2] = (sg1 * rsg) * (wdiag * pr[1 - U]);
        }
    };
    step(k0 - 1, std::true_type{});  // k0 even: x1 of plane k0 - 1 only
    for (int z = k0; z < k0 + zc + 2; z += 2) {
        step(z, std::false_type{});
        step(z + 1, std::true_type{});
    }
}

// The down-leg of a large 3D level from a nonzero iterate in one pass (one cell
// per thread, 32 x 16 tiles, in every storage precision): x2 = sweep(sweep(x))
// and fc = R (f - A x2),
// with NORM the per-workgroup partials of |f - A x|^2 (the convergence check of
// the input iterate).  Three stages run one plane apart: the first sweep at
// plane z on the tile and a two-cell ring (reading x on a three-cell ring from
// LDS), the second at z - 1 on the tile and a one-cell ring, the residual of x2
// at z - 2 on the tile, summed over the children of each coarse cell in
// k_restrict3's order (the plane pair, then the column pair and the row pair by
// lane shuffles).  The second and third stages read what the previous plane
// step wrote (two LDS slots per stage), so in FP64, with the iterate's plane in
// two slots too, a step waits at one barrier, after that plane is stored (FP32
// keeps a barrier after each stage).  Ring cells go to whole
// waves as in k_sweep2z (ring 1 first,
// then ring 3, ring 2 last) and share one register set.  The second sweep and
// the residual read a Dirichlet ghost as minus the cell's own value, the first
// sweep reads the iterate's ghosts by the boundary rule, as the per-kernel
// kernels do: both outputs equal k_sweep3 twice then k_restrict3 bit for bit.
template <class S> struct Z3Cfg {
    static constexpr int TP = 32, TX = 32, TY = kS3Threads / TP;
    static constexpr int W1 = TX + 2, H1 = TY + 2, W2 = TX + 4, H2 = TY + 4, W3 = TX + 6, H3 = TY + 6;
    static constexpr int NR1 = 2 * (TX + 2) + 2 * TY, NR2 = 2 * (TX + 4) + 2 * (TY + 2),
                         NR3 = 2 * (TX + 6) + 2 * (TY + 4);
    static constexpr int NW = kS3Threads / 64;
    static constexpr int NW1 = (NR1 + 63) / 64, NW2 = (NR2 + 63) / 64, NW3 = (NR3 + 63) / 64;
    static_assert(NW1 + NW2 + NW3 <= NW, "ring slots on distinct waves");
};
template <class S> inline int down2z_planes(int lg) { return z2_planes(lg, Z3Cfg<S>::TX, Z3Cfg<S>::TY); }

template <class S, bool NORM>
__global__ __launch_bounds__(kS3Threads) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 4 : 2))) void k_down2z(const S *__restrict__ f, const S *__restrict__ xin,
                                                       S *__restrict__ xout, S *__restrict__ fc,
                                                       double *__restrict__ partial, int lg, int bc, int zc,
                                                       typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                       const int *stop) {
    typedef typename St<S>::C C;
    typedef Z3Cfg<S> G;
    constexpr int TX = G::TX, TY = G::TY, TP = G::TP, W1 = G::W1, W2 = G::W2, W3 = G::W3;
    constexpr int B1 = G::H1 * W1, B2 = G::H2 * W2, B3 = G::H3 * W3;
    // FP64: one barrier per plane step (the iterate's plane in two slots); FP32: three, which
    // measured faster there (4.19 against 4.23 ms per FP32-mixed 256^3 solve; FP64 6.60 -> 6.54)
    constexpr bool ONE = sizeof(S) == 8;
    __shared__ C XA[(ONE ? 2 : 1) * B3];  // x of plane z (ONE: planes z - 1, z, slot = plane & 1), tile and three-cell ring
    __shared__ C X1[2 * B2];      // first sweep of planes z - 1, z (slot = plane & 1), tile and two-cell ring
    __shared__ C X2[2 * B1];      // second sweep of planes z - 2, z - 1, tile and one-cell ring
    if (stop && *stop) return;
    const int n = 1 << lg, ntx = n / TX, nty = n / TY, lgc = lg - 1;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP;
    const int x0 = (blk % ntx) * TX, y0 = ((blk / ntx) % nty) * TY, k0 = (blk / (ntx * nty)) * zc;
    const int pl = 2 * lg;
    const uint32_t osrc = (uint32_t(y0 + ty) << lg) + uint32_t(x0 + tp);
    // ring role of this thread's wave: 1, 3 (after ring 1) or 2 (the last waves), or none
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool r1 = wv < G::NW1, r3 = wv >= G::NW1 && wv < G::NW1 + G::NW3, r2 = wv >= G::NW - G::NW2;
    const bool rr = r1 || r2 || r3;
    int ra = 0, rb = 0;
    if (r1) ring_pos<TX, TY>(min(t, G::NR1 - 1), 1, ra, rb);
    if (r3) ring_pos<TX, TY>(min(t - 64 * G::NW1, G::NR3 - 1), 3, ra, rb);
    if (r2) ring_pos<TX, TY>(min(t - 64 * (G::NW - G::NW2), G::NR2 - 1), 2, ra, rb);
    uint32_t rsrc;
    C rsg;
    {
        int s = 1;
        const int gi = bmap(x0 + ra, n, bc, s), gj = bmap(y0 + rb, n, bc, s);
        rsrc = (uint32_t(gj) << lg) + uint32_t(gi);
        rsg = C(s);
    }
    const int own_a = (ty + 3) * W3 + tp + 3, own_1 = (ty + 2) * W2 + tp + 2, own_2 = (ty + 1) * W1 + tp + 1;
    const int ring_a = (rb + 3) * W3 + ra + 3, ring_1 = (rb + 2) * W2 + ra + 2, ring_2 = (rb + 1) * W1 + ra + 1;
    // Dirichlet walls next to a position (the ghosts of the second sweep and the residual)
    auto wall = [&](int a, int b, bool &w, bool &e, bool &so, bool &no) {
        w = !bc && x0 + a == 0;
        e = !bc && x0 + a == n - 1;
        so = !bc && y0 + b == 0;
        no = !bc && y0 + b == n - 1;
    };
    bool ow, oe, os, on, qw, qe, qs, qn;
    wall(tp, ty, ow, oe, os, on);
    wall(ra, rb, qw, qe, qs, qn);
    auto poff = [&](int q) -> uint32_t {
        bool flip;
        return uint32_t(plane_map(q, n, bc, flip)) << pl;
    };
    auto psign = [&](int q) -> C { return (!bc && (q < 0 || q >= n)) ? C(-1) : C(1); };
    // a sweep at an LDS position with in-plane neighbours from frame L (row width W), z-neighbours
    // given; the residual r of the input
    auto sweepL = [&](const C *L, int W, int q, C xc, C xm, C xp, C fv, C &r) -> C {
        const C t0 = ((L[q - 1] + L[q + 1]) + L[q - W]) + L[q + W];
        const C s = (t0 + xm) + xp;
        r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // the same with Dirichlet ghosts selected as minus the centre value
    auto sweepD = [&](const C *L, int W, int q, C xc, C xm, C xp, C fv, bool w, bool e, bool so, bool no,
                      bool zl, bool zu, C &r) -> C {
        const C lw = L[q - 1], le = L[q + 1], ls = L[q - W], ln = L[q + W];
        const C xw = w ? -xc : lw, xe = e ? -xc : le, ys = so ? -xc : ls, yn = no ? -xc : ln;
        const C zm = zl ? -xc : xm, zp = zu ? -xc : xp;
        const C t0 = ((xw + xe) + ys) + yn;
        const C s = (t0 + zm) + zp;
        r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // registers: own x at z - 1 .. z + 1, x1 at z - 2 .. z, x2 at z - 3, z - 2, f at z, z - 1, z - 2;
    // ring (one set for every role): x at z - 1 .. z + 1 (ring 3: z only), x1 at z - 2 .. z (ring 1),
    // f at z, z - 1
    C xo[3], x1o[3], x2o[2], fo[3];
    C rx[3] = {C(0), C(0), C(0)}, r1x[3] = {C(0), C(0), C(0)}, rf[2] = {C(0), C(0)};
    C pw[2], pf[2], pr[2] = {C(0), C(0)}, pq[2] = {C(0), C(0)};  // loads in flight (set = step parity)
    for (int i = 0; i < 3; ++i) x1o[i] = fo[i] = C(0);
    x2o[0] = x2o[1] = C(0);
    // the step at plane z consumes x(z + 2), f(z + 1) at the own cell and the ring cell (ring 3:
    // x(z + 1)); past the planes used the last one is read again
    auto pload = [&](int z, auto u) {
        constexpr int U = decltype(u)::value;
        const uint32_t o2 = poff(min(z + 2, k0 + zc + 2)), o1 = poff(min(z + 1, k0 + zc + 1));
        pw[U] = St<S>::ld(xin + o2 + osrc);
        pf[U] = St<S>::ld(f + o1 + osrc);
        pr[U] = St<S>::ld(xin + (r3 ? o1 : o2) + rsrc);
        pq[U] = St<S>::ld(f + o1 + rsrc);
    };
    // prologue: x at k0 - 3 .. k0 - 1, f at k0 - 2 (own, rings 1 and 2); ring 3: x at k0 - 2
    for (int i = 0; i < 3; ++i) {
        const int q = k0 - 3 + i;
        xo[i] = psign(q) * St<S>::ld(xin + poff(q) + osrc);
        rx[i] = (psign(q) * rsg) * St<S>::ld(xin + poff(q) + rsrc);
    }
    fo[0] = St<S>::ld(f + poff(k0 - 2) + osrc);
    rf[0] = St<S>::ld(f + poff(k0 - 2) + rsrc);
    if (r3) rx[1] = (psign(k0 - 2) * rsg) * St<S>::ld(xin + poff(k0 - 2) + rsrc);
    pload(k0 - 2, std::integral_constant<int, 0>{});
    double acc = 0.0;
    C pair = C(0);
    auto step = [&](int z, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        constexpr int U = ODD ? 1 : 0;
        pload(z + 1, std::integral_constant<int, 1 - U>{});
        // x of plane z into LDS: own cell and the ring cell (every role).  With ONE, the step's one
        // barrier follows: stages B and C read what the previous step wrote, and every slot
        // written here was last read before it
        C *LA = XA + (ONE && ODD ? B3 : 0);
        LA[own_a] = xo[1];
        if (rr) LA[ring_a] = rx[1];
        __syncthreads();
        // stage A: first sweep at plane z, own cell, rings 1 and 2
        C *L1 = X1 + (ODD ? B2 : 0);
        {
            C r;
            const C v = st_round<S>(sweepL(LA, W3, own_a, xo[1], xo[0], xo[2], fo[0], r));
            if (NORM && z >= k0 && z < k0 + zc) acc += double(r) * double(r);
            L1[own_1] = v;
            x1o[2] = v;  // x1 at z (registers slide at the end of the step)
        }
        if (r1 || r2) {
            C r;
            const C v = st_round<S>(sweepL(LA, W3, ring_a, rx[1], rx[0], rx[2], rf[0], r));
            L1[ring_1] = v;
            r1x[2] = v;
        }
        if constexpr (!ONE) __syncthreads();
        // stage B: second sweep at plane z - 1 (x1 written by the previous step), own cell and ring 1
        const int p = z - 1;
        const C *M1 = X1 + (ODD ? 0 : B2);
        C *L2 = X2 + (ODD ? 0 : B1);
        const bool zl1 = !bc && p == 0, zu1 = !bc && p == n - 1;
        C x2n = C(0);
        if (z >= k0) {
            C r;
            x2n = st_round<S>(sweepD(M1, W2, own_1, x1o[1], x1o[0], x1o[2], fo[1], ow, oe, os, on, zl1, zu1, r));
            L2[own_2] = x2n;
            if (p >= k0 && p < k0 + zc) St<S>::st(xout + (uint32_t(p) << pl) + osrc, x2n);
            if (r1) {
                L2[ring_2] = st_round<S>(sweepD(M1, W2, ring_1, r1x[1], r1x[0], r1x[2], rf[1], qw, qe, qs, qn, zl1,
                                                zu1, r));
            }
        }
        if constexpr (!ONE) __syncthreads();
        // stage C: residual of x2 at plane z - 2 (written by the previous step), own cell, into the
        // coarse cells
        if (z >= k0 + 2) {
            const int pc = z - 2;
            const C *M2 = X2 + (ODD ? B1 : 0);
            const bool zl = !bc && pc == 0, zu = !bc && pc == n - 1;
            C r;
            (void)sweepD(M2, W1, own_2, x2o[1], x2o[0], x2n, fo[2], ow, oe, os, on, zl, zu, r);
            const uint32_t cc = (uint32_t(pc >> 1) << (2 * lgc)) + (uint32_t((y0 + ty) >> 1) << lgc) +
                                uint32_t((x0 + tp) >> 1);
            if constexpr (ZCfg<S>::CPT == 2) {
                // k_restrict3 with two cells per thread: the x-pair of each plane, the plane pair,
                // then the row pair
                const C rx = r + __shfl_down(r, 1);
                if (ODD) {
                    pair += rx;
                    const C o = __shfl_down(pair, 32);
                    if (((tp | ty) & 1) == 0) St<S>::st(fc + cc, (pair + o) * C(0.125));
                } else {
                    pair = rx;
                }
            } else {
                // one cell per thread: the plane pair, then the column pair and the row pair
                if (ODD) {  // pc odd: the second plane of the pair
                    pair += r;
                    const C b = __shfl_down(pair, 1), cy = __shfl_down(pair, 32), d = __shfl_down(pair, 33);
                    if (((tp | ty) & 1) == 0) St<S>::st(fc + cc, (((pair + b) + cy) + d) * C(0.125));
                } else {
                    pair = r;
                }
            }
        }
        // slide
        const C sg2 = psign(z + 2), sg1 = psign(z + 1);
        x2o[0] = x2o[1];
        x2o[1] = x2n;
        x1o[0] = x1o[1];
        x1o[1] = x1o[2];
        fo[2] = fo[1];
        fo[1] = fo[0];
        fo[0] = pf[U];
        xo[0] = xo[1];
        xo[1] = xo[2];
        xo[2] = sg2 * pw[U];
        r1x[0] = r1x[1];
        r1x[1] = r1x[2];
        rf[1] = rf[0];
        rf[0] = pq[U];
        if (r3) {
            rx[1] = (sg1 * rsg) * pr[U];
        } else {
            rx[0] = rx[1];
            rx[1] = rx[2];
            rx[2] = (sg2 * rsg) * pr[U];
        }
    };
    for (int z = k0 - 2; z < k0 + zc + 2; z += 2) {  // k0 even: pairs (even, odd)
        step(z, std::false_type{});
        step(z + 1, std::true_type{});
    }
    if constexpr (NORM) {
        acc = block_sum_n<kS3Threads>(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// k_down2z on two cells per thread: the 64 x 16 tiles of k_sweep2z (paired
// accesses), the same three stages one plane apart and one barrier per plane
// step (each stage's LDS plane in two slots).  Rings 1 and 2 take whole waves
// as in k_sweep2z; the three-cell ring, whose cells only carry the iterate of
// the plane into LDS, is a second slot of the ring-1 waves.  The residual's
// children are summed in k_restrict3's order (the cell pair, the plane pair,
// then the row pair by a lane shuffle).  Same values as k_down2z bit for bit.
template <class S> struct Z4Cfg {
    typedef Z2Cfg<S> G2;
    static constexpr int TP = G2::TP, TX = G2::TX, TY = G2::TY, CPT = G2::CPT;
    static constexpr int W1 = TX + 2, H1 = TY + 2, W2 = TX + 4, H2 = TY + 4, W3 = TX + 6, H3 = TY + 6;
    static constexpr int NR1 = G2::NR1, NR2 = G2::NR2, NR3 = 2 * (TX + 6) + 2 * (TY + 4);
    static constexpr int NW = G2::NW, NW1 = G2::NW1, NW2 = G2::NW2;
    static_assert(CPT == 2 && TP == 32, "two cells per thread, rows ty and ty + 1 in the two halves of a wave");
    static_assert(NR3 <= 64 * NW1, "the three-cell ring fits the ring-1 waves");
};

template <class S, bool NORM>
__global__ __launch_bounds__(kS3Threads) void k_down2z2(const S *__restrict__ f, const S *__restrict__ xin,
                                                        S *__restrict__ xout, S *__restrict__ fc,
                                                        double *__restrict__ partial, int lg, int bc, int zc,
                                                        typename St<S>::C inv_h2, typename St<S>::C wdiag,
                                                        const int *stop) {
    typedef typename St<S>::C C;
    typedef Z4Cfg<S> G;
    constexpr int TX = G::TX, TY = G::TY, TP = G::TP, W1 = G::W1, W2 = G::W2, W3 = G::W3;
    constexpr int B1 = G::H1 * W1, B2 = G::H2 * W2, B3 = G::H3 * W3;
    __shared__ C XA[2 * B3];  // x of planes z - 1, z (slot = plane & 1), tile and three-cell ring
    __shared__ C X1[2 * B2];  // first sweep of planes z - 1, z, tile and two-cell ring
    __shared__ C X2[2 * B1];  // second sweep of planes z - 2, z - 1, tile and one-cell ring
    if (stop && *stop) return;
    const int n = 1 << lg, ntx = n / TX, nty = n / TY, lgc = lg - 1;
    const int blk = int(xcd_block(blockIdx.x, gridDim.x));
    const int t = int(threadIdx.x), tp = t % TP, ty = t / TP, ai = 2 * tp;
    const int x0 = (blk % ntx) * TX, y0 = ((blk / ntx) % nty) * TY, k0 = (blk / (ntx * nty)) * zc;
    const int pl = 2 * lg;
    const uint32_t osrc = (uint32_t(y0 + ty) << lg) + uint32_t(x0 + ai);
    // ring roles of this thread's wave: ring 1 (also a three-cell-ring slot) on the first waves,
    // ring 2 on the last, none between
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool r1 = wv < G::NW1, r2 = wv >= G::NW - G::NW2, rr = r1 || r2;
    int ra = 0, rb = 0, ta = 0, tb = 0;
    if (r1) {
        ring_pos<TX, TY>(min(t, G::NR1 - 1), 1, ra, rb);
        ring_pos<TX, TY>(min(t, G::NR3 - 1), 3, ta, tb);
    }
    if (r2) ring_pos<TX, TY>(min(t - 64 * (G::NW - G::NW2), G::NR2 - 1), 2, ra, rb);
    uint32_t rsrc, tsrc;
    C rsg, tsg;
    {
        int s1 = 1, s3 = 1;
        const int gi = bmap(x0 + ra, n, bc, s1), gj = bmap(y0 + rb, n, bc, s1);
        rsrc = (uint32_t(gj) << lg) + uint32_t(gi);
        rsg = C(s1);
        const int hi = bmap(x0 + ta, n, bc, s3), hj = bmap(y0 + tb, n, bc, s3);
        tsrc = (uint32_t(hj) << lg) + uint32_t(hi);
        tsg = C(s3);
    }
    const int own_a = (ty + 3) * W3 + ai + 3, own_1 = (ty + 2) * W2 + ai + 2, own_2 = (ty + 1) * W1 + ai + 1;
    const int ring_a = (rb + 3) * W3 + ra + 3, ring_1 = (rb + 2) * W2 + ra + 2, ring_2 = (rb + 1) * W1 + ra + 1;
    const int r3_a = (tb + 3) * W3 + ta + 3;
    // Dirichlet walls next to a position (the ghosts of the second sweep and the residual)
    bool dw[2], de[2];
    for (int c = 0; c < 2; ++c) {
        dw[c] = !bc && x0 + ai + c == 0;
        de[c] = !bc && x0 + ai + c == n - 1;
    }
    const bool ds = !bc && y0 + ty == 0, dn = !bc && y0 + ty == n - 1;
    const bool qw = !bc && x0 + ra == 0, qe = !bc && x0 + ra == n - 1;
    const bool qs = !bc && y0 + rb == 0, qn = !bc && y0 + rb == n - 1;
    auto poff = [&](int q) -> uint32_t {
        bool flip;
        return uint32_t(plane_map(q, n, bc, flip)) << pl;
    };
    auto psign = [&](int q) -> C { return (!bc && (q < 0 || q >= n)) ? C(-1) : C(1); };
    auto ld2 = [&](const S *base, C (&v)[2]) { Pair<S>::ld(base + osrc, v[0], v[1]); };
    // a sweep at an LDS position with in-plane neighbours from frame L (row width W), z-neighbours
    // given; the residual r of the input
    auto sweepL = [&](const C *L, int W, int q, C xc, C xm, C xp, C fv, C &r) -> C {
        const C t0 = ((L[q - 1] + L[q + 1]) + L[q - W]) + L[q + W];
        const C s = (t0 + xm) + xp;
        r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // the same with Dirichlet ghosts selected as minus the centre value
    auto sweepD = [&](const C *L, int W, int q, C xc, C xm, C xp, C fv, bool w, bool e, bool so, bool no,
                      bool zl, bool zu, C &r) -> C {
        const C lw = L[q - 1], le = L[q + 1], ls = L[q - W], ln = L[q + W];
        const C xw = w ? -xc : lw, xe = e ? -xc : le, ys = so ? -xc : ls, yn = no ? -xc : ln;
        const C zm = zl ? -xc : xm, zp = zu ? -xc : xp;
        const C t0 = ((xw + xe) + ys) + yn;
        const C s = (t0 + zm) + zp;
        r = fv - (C(6) * xc - s) * inv_h2;
        return xc + wdiag * r;
    };
    // registers: own x at z - 1 .. z + 1, x1 at z - 2 .. z, x2 at z - 3, z - 2, f at z, z - 1, z - 2;
    // ring cell (rings 1 and 2): x at z - 1 .. z + 1, x1 at z - 2 .. z (ring 1), f at z, z - 1;
    // three-cell-ring slot: x at z
    C xo[3][2], x1o[3][2], x2o[2][2], fo[3][2];
    C rx[3] = {C(0), C(0), C(0)}, r1x[3] = {C(0), C(0), C(0)}, rf[2] = {C(0), C(0)}, r3x = C(0);
    C pw[2][2], pf[2][2], pr[2] = {C(0), C(0)}, pq[2] = {C(0), C(0)}, p3[2] = {C(0), C(0)};  // in flight
    for (int c = 0; c < 2; ++c) {
        for (int i = 0; i < 3; ++i) x1o[i][c] = fo[i][c] = C(0);
        x2o[0][c] = x2o[1][c] = C(0);
    }
    // the step at plane z consumes x(z + 2) and f(z + 1) at the own cells and the ring cell, and
    // x(z + 1) at the three-cell-ring slot; past the planes used the last one is read again
    auto pload = [&](int z, auto u) {
        constexpr int U = decltype(u)::value;
        const uint32_t o2 = poff(min(z + 2, k0 + zc + 2)), o1 = poff(min(z + 1, k0 + zc + 1));
        ld2(xin + o2, pw[U]);
        ld2(f + o1, pf[U]);
        pr[U] = St<S>::ld(xin + o2 + rsrc);
        pq[U] = St<S>::ld(f + o1 + rsrc);
        p3[U] = St<S>::ld(xin + o1 + tsrc);
    };
    // prologue: x at k0 - 3 .. k0 - 1, f at k0 - 2 (own, ring); three-cell ring: x at k0 - 2
    for (int i = 0; i < 3; ++i) {
        const int q = k0 - 3 + i;
        const C sg = psign(q);
        ld2(xin + poff(q), xo[i]);
        for (int c = 0; c < 2; ++c) xo[i][c] *= sg;
        rx[i] = (sg * rsg) * St<S>::ld(xin + poff(q) + rsrc);
    }
    ld2(f + poff(k0 - 2), fo[0]);
    rf[0] = St<S>::ld(f + poff(k0 - 2) + rsrc);
    r3x = (psign(k0 - 2) * tsg) * St<S>::ld(xin + poff(k0 - 2) + tsrc);
    pload(k0 - 2, std::integral_constant<int, 0>{});
    double acc = 0.0;
    C pair = C(0);
    auto step = [&](int z, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        constexpr int U = ODD ? 1 : 0;
        pload(z + 1, std::integral_constant<int, 1 - U>{});
        // x of plane z into its slot: own cells, the ring cell, the three-cell-ring slot.  The
        // step's one barrier follows: stages B and C read what the previous step wrote, and
        // every slot written here was last read before it
        C *LA = XA + (ODD ? B3 : 0);
        for (int c = 0; c < 2; ++c) LA[own_a + c] = xo[1][c];
        if (rr) LA[ring_a] = rx[1];
        if (r1) LA[r3_a] = r3x;
        __syncthreads();
        // stage A: first sweep at plane z, own cells, rings 1 and 2
        C *L1 = X1 + (ODD ? B2 : 0);
        for (int c = 0; c < 2; ++c) {
            C r;
            const C v = st_round<S>(sweepL(LA, W3, own_a + c, xo[1][c], xo[0][c], xo[2][c], fo[0][c], r));
            if (NORM && z >= k0 && z < k0 + zc) acc += double(r) * double(r);
            L1[own_1 + c] = v;
            x1o[2][c] = v;  // x1 at z (registers slide at the end of the step)
        }
        if (rr) {
            C r;
            const C v = st_round<S>(sweepL(LA, W3, ring_a, rx[1], rx[0], rx[2], rf[0], r));
            L1[ring_1] = v;
            r1x[2] = v;
        }
        // stage B: second sweep at plane z - 1 (x1 written by the previous step), own cells and ring 1
        const int p = z - 1;
        const C *M1 = X1 + (ODD ? 0 : B2);
        C *L2 = X2 + (ODD ? 0 : B1);
        const bool zl1 = !bc && p == 0, zu1 = !bc && p == n - 1;
        C x2n[2] = {C(0), C(0)};
        if (z >= k0) {
            C r;
            for (int c = 0; c < 2; ++c) {
                x2n[c] = st_round<S>(sweepD(M1, W2, own_1 + c, x1o[1][c], x1o[0][c], x1o[2][c], fo[1][c], dw[c],
                                            de[c], ds, dn, zl1, zu1, r));
                L2[own_2 + c] = x2n[c];
            }
            if (p >= k0 && p < k0 + zc) Pair<S>::st(xout + (uint32_t(p) << pl) + osrc, x2n[0], x2n[1]);
            if (r1) {
                L2[ring_2] = st_round<S>(sweepD(M1, W2, ring_1, r1x[1], r1x[0], r1x[2], rf[1], qw, qe, qs, qn, zl1,
                                                zu1, r));
            }
        }
        // stage C: residual of x2 at plane z - 2 (written by the previous step), own cells, into the
        // coarse cells: the cell pair, the plane pair, then the row pair
        if (z >= k0 + 2) {
            const int pc = z - 2;
            const C *M2 = X2 + (ODD ? B1 : 0);
            const bool zl = !bc && pc == 0, zu = !bc && pc == n - 1;
            C rc[2];
            for (int c = 0; c < 2; ++c)
                (void)sweepD(M2, W1, own_2 + c, x2o[1][c], x2o[0][c], x2n[c], fo[2][c], dw[c], de[c], ds, dn, zl, zu,
                             rc[c]);
            const C rxp = rc[0] + rc[1];
            if (ODD) {  // pc odd: the second plane of the pair
                pair += rxp;
                const uint32_t cc = (uint32_t(pc >> 1) << (2 * lgc)) + (uint32_t((y0 + ty) >> 1) << lgc) +
                                    uint32_t((x0 + ai) >> 1);
                const C o = __shfl_down(pair, 32);
                if ((ty & 1) == 0) St<S>::st(fc + cc, (pair + o) * C(0.125));
            } else {
                pair = rxp;
            }
        }
        // slide
        const C sg2 = psign(z + 2), sg1 = psign(z + 1);
        for (int c = 0; c < 2; ++c) {
            x2o[0][c] = x2o[1][c];
            x2o[1][c] = x2n[c];
            x1o[0][c] = x1o[1][c];
            x1o[1][c] = x1o[2][c];
            fo[2][c] = fo[1][c];
            fo[1][c] = fo[0][c];
            fo[0][c] = pf[U][c];
            xo[0][c] = xo[1][c];
            xo[1][c] = xo[2][c];
            xo[2][c] = sg2 * pw[U][c];
        }
        r1x[0] = r1x[1];
        r1x[1] = r1x[2];
        rf[1] = rf[0];
        rf[0] = pq[U];
        rx[0] = rx[1];
        rx[1] = rx[2];
        rx[2] = (sg2 * rsg) * pr[U];
        r3x = (sg1 * tsg) * p3[U];
    };
    for (int z = k0 - 2; z < k0 + zc + 2; z += 2) {  // k0 even: pairs (even, odd)
        step(z, std::false_type{});
        step(z + 1, std::true_type{});
    }
    if constexpr (NORM) {
        acc = block_sum_n<kS3Threads>(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

}  // namespace np
