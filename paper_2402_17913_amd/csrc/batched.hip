// Batched uneven-size 2D Poisson solves (mixed-precision refinement with
// batched V-cycles), one launch per level depth across all problems,
// refinement steps replayed from HIP graphs, per-problem convergence on the
// device, and an autotuner for the inner cycle count.
//
// Depths are counted from the coarsest grid: depth k has 4 * 2^k cells per
// axis, so every problem present at depth k has the same size there and one
// launch covers all of them.  Problem p (finest depth L_p) is present at
// depths 0..L_p; its fields at depth k live in slot slot[k] of that depth's
// pools.  Depths at or below kTailDepth run inside one workgroup per problem.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unistd.h>
#include <sys/stat.h>
#include <string>
#include <cstdlib>
#include <cstdio>
#include <map>
#include <mutex>
#include <vector>

#include "mg_kernels.h"
#include "mg_level.h"
#include "np_internal.h"

namespace np {

// Dense inverse of the 4^d coarsest operator (defined in mg.hip).
bool coarse_inverse_host(int d, int bc, double hc, std::vector<double> &inv);

namespace {

constexpr int kMaxDepth = 12;                 // up to 16384^2
constexpr int kTailDepth = Tail<2>::LG - 2;   // 64^2 and below run in one workgroup
constexpr int kHist = 64;                     // residual history kept per problem

struct BProb {
    int L;                 // finest depth
    int first_block;       // first refinement block
    int nblocks;           // refinement blocks
    int ir_first, ir_nblocks;  // the same for the row-marching refinement blocks
    int slot[kMaxDepth + 1];
    double h;              // finest spacing
    double nf;             // ||f||_2
};

struct BState {            // per-problem controller
    int stop, k, pad0, pad1;
    double hist[kHist];
};

struct BGlobal {
    int stop;              // all problems stopped
    int fixed, maxc, pad;
    double tol;
};

template <class S> struct BPtrs {
    const double *const *f;  // FP64 right-hand sides
    const double *const *xa; // FP64 iterate read
    double *const *xb;       // FP64 iterate written
};

// ---------------------------------------------------------------- kernels
// Refinement blocks cover kIrCells consecutive cells of one problem.
struct BBlk {
    int p;
    int base;
};

__device__ __forceinline__ double depth_h(const BProb &P, int k) { return P.h * double(1 << (P.L - k)); }

// ||f||^2 partials per refinement block.
__global__ __launch_bounds__(kBlock) void kb_fnorm(const double *const *f, const BBlk *__restrict__ blk,
                                                   const BProb *__restrict__ P, double *__restrict__ partial) {
    const BBlk b = blk[blockIdx.x];
    const int lg = P[b.p].L + 2;
    const int64_t m = int64_t(1) << (2 * lg);
    const double *fp = f[b.p];
    double acc = 0.0;
    for (int u = 0; u < kIrCells / kBlock; ++u) {
        const int64_t c = int64_t(b.base) + u * kBlock + threadIdx.x;
        if (c < m) acc += fp[c] * fp[c];
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Sum of problem p's partials by one wavefront: lane l adds blocks l, l + 64,
// ...; then a fixed butterfly.  Deterministic; the result is in every lane.
__device__ __forceinline__ double prob_sum(const double *__restrict__ partial, int first, int nb) {
    const int lane = int(threadIdx.x) & 63;
    double s = 0.0;
    for (int b = lane; b < nb; b += 64) s += partial[first + b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// nf[p] = sqrt(sum of its partials); zero right-hand sides stop at once.  One
// wavefront per problem.
__global__ __launch_bounds__(1024) void kb_nf(const double *__restrict__ partial, BProb *__restrict__ P,
                                              BState *__restrict__ st, int nprob) {
    const int w = int(threadIdx.x) >> 6, nw = int(blockDim.x) >> 6;
    for (int p = w; p < nprob; p += nw) {
        const double s = prob_sum(partial, P[p].first_block, P[p].nblocks);
        if ((threadIdx.x & 63) == 0) {
            P[p].nf = sqrt(s);
            st[p].stop = s == 0.0 ? kConverged : kRunning;
            st[p].k = 0;
            st[p].hist[0] = 0.0;
        }
    }
}

// x_p = 0 for every problem (through the pointer table).
__global__ __launch_bounds__(kBlock) void kb_zero(double *const *x, const BBlk *__restrict__ blk,
                                                  const BProb *__restrict__ P) {
    const BBlk b = blk[blockIdx.x];
    const int64_t m = int64_t(1) << (2 * (P[b.p].L + 2));
    double *xp = x[b.p];
    for (int u = 0; u < kIrCells / kBlock; ++u) {
        const int64_t c = int64_t(b.base) + u * kBlock + threadIdx.x;
        if (c < m) xp[c] = 0.0;
    }
}

// Copies pool -> caller buffer for problems whose last checked iterate is in
// the pool (odd number of updates).
__global__ __launch_bounds__(kBlock) void kb_final_copy(const double *const *y, double *const *x,
                                                        const BBlk *__restrict__ blk, const BProb *__restrict__ P,
                                                        const BState *__restrict__ st) {
    const BBlk b = blk[blockIdx.x];
    if (!(st[b.p].k & 1)) return;
    const int64_t m = int64_t(1) << (2 * (P[b.p].L + 2));
    const double *yp = y[b.p];
    double *xp = x[b.p];
    for (int u = 0; u < kIrCells / kBlock; ++u) {
        const int64_t c = int64_t(b.base) + u * kBlock + threadIdx.x;
        if (c < m) xp[c] = yp[c];
    }
}

// FP64 refinement step per problem: x_b = x_a + e (has_e), r = f - A x_b in
// FP64, r_lo = round(r) into the problem's finest-depth rhs slot, partials.
template <class SL>
__global__ __launch_bounds__(kBlock) void kb_ir(BPtrs<SL> ptr, SL *const *epool, SL *const *rpool,
                                                const BBlk *__restrict__ blk, const BProb *__restrict__ P,
                                                const BState *__restrict__ st, const BGlobal *__restrict__ g,
                                                double *__restrict__ partial, int has_e) {
    const BBlk b = blk[blockIdx.x];
    if (g->stop || st[b.p].stop) return;
    const BProb &pp = P[b.p];
    const int lg = pp.L + 2;
    const int64_t m = int64_t(1) << (2 * lg);
    const double inv_h2 = 1.0 / (pp.h * pp.h);
    const int64_t so = int64_t(pp.slot[pp.L]) * m;
    const SL *e = epool[pp.L] + so;
    SL *rlo = rpool[pp.L] + so;
    const double *x = ptr.xa[b.p], *f = ptr.f[b.p];
    double *xo = ptr.xb[b.p];
    struct {
        const double *x;
        const SL *e;
        int he;
        __device__ double operator()(int64_t q) const { return he ? x[q] + double(St<SL>::ld(e + q)) : x[q]; }
    } ldx{x, e, has_e};
    double acc = 0.0;
    for (int u = 0; u < kIrCells / kBlock; ++u) {
        const int64_t c = int64_t(b.base) + u * kBlock + threadIdx.x;
        if (c < m) {
            int i, j, k;
            decode<2>(c, lg, i, j, k);
            const double xc = ldx(c);
            const double s = nb_sum<2, double>(ldx, c, i, j, k, lg, 0, xc);
            const double r = f[c] - (4.0 * xc - s) * inv_h2;
            if (has_e) xo[c] = xc;
            St<SL>::st(rlo + c, typename St<SL>::C(r));
            acc += r * r;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Per-problem convergence check after a refinement residual: one wavefront
// per problem (grid: nprob / 4 workgroups of 4) sums its partials (of the
// row-marching refinement blocks when ir_blocks) and its first lane applies
// the stop rule.
__global__ __launch_bounds__(256) void kb_check(const double *__restrict__ partial, const BProb *__restrict__ P,
                                                BState *__restrict__ st, const BGlobal *__restrict__ g, int nprob,
                                                int ir_blocks) {
    if (g->stop) return;
    const int p = int(blockIdx.x) * 4 + (int(threadIdx.x) >> 6);
    if (p >= nprob) return;
    BState &s = st[p];
    if (s.stop) return;
    const double sum = ir_blocks ? prob_sum(partial, P[p].ir_first, P[p].ir_nblocks)
                                 : prob_sum(partial, P[p].first_block, P[p].nblocks);
    if (threadIdx.x & 63) return;
    const int k = s.k;
    const double rr = sqrt(sum) / P[p].nf;
    if (k < kHist) s.hist[k] = rr;
    int stp = kRunning;
    if (!(rr <= 1.0e300)) stp = kNonFinite;
    else if (g->fixed > 0) { if (k >= g->fixed) stp = kFixedDone; }
    else if (rr <= g->tol) stp = kConverged;
    else if (k >= g->maxc) stp = kMaxCycles;
    else if (k >= 3 && k < kHist && s.hist[k - 3] < s.hist[k - 2] && s.hist[k - 2] < s.hist[k - 1] &&
             s.hist[k - 1] < rr)
        stp = kDiverged;
    if (stp != kRunning) s.stop = stp;
    else s.k = k + 1;
}

// After kb_check: the whole batch stops once no problem is still running.
__global__ __launch_bounds__(1024) void kb_check_any(const BState *__restrict__ st, BGlobal *__restrict__ g,
                                                     int nprob) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (g->stop) return;
    for (int p = threadIdx.x; p < nprob; p += blockDim.x)
        if (st[p].stop == kRunning) any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && !any) g->stop = 1;
}

// One Jacobi sweep at depth k over every problem present there.  first: the
// first pre-smoothing sweep, which starts from zero unless this depth is the
// problem's finest and the inner cycle is not the first (cyc > 0).
template <class S>
__global__ __launch_bounds__(kBlock) void kb_sweep(const S *__restrict__ F, const S *__restrict__ Xin,
                                                   S *__restrict__ Xout, const int *__restrict__ slot_prob,
                                                   const BProb *__restrict__ P, const BState *__restrict__ st,
                                                   const BGlobal *__restrict__ g, int k, int first, int cyc,
                                                   double omega) {
    typedef typename St<S>::C C;
    const int lg = k + 2;
    const int64_t m = int64_t(1) << (2 * lg);
    const int bpp = int((m + kSweepCells - 1) / kSweepCells);
    const int slot = blockIdx.x / bpp;
    const int p = slot_prob[slot];
    if (g->stop || st[p].stop) return;
    const double h = depth_h(P[p], k);
    const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / 4.0);
    const bool zero = first && (k < P[p].L || cyc == 0);
    const int64_t so = int64_t(slot) * m;
    const S *f = F + so, *xin = Xin + so;
    S *xout = Xout + so;
    const int64_t base = int64_t(blockIdx.x % bpp) * kSweepCells;
    for (int u = 0; u < kSweepCells / kBlock; ++u) {
        const int64_t c = base + u * kBlock + threadIdx.x;
        if (c >= m) continue;
        const C fc = St<S>::ld(f + c);
        if (zero) {
            St<S>::st(xout + c, wdiag * fc);
        } else {
            int i, j, kk;
            decode<2>(c, lg, i, j, kk);
            const C xc = St<S>::ld(xin + c);
            const C s = nb_sum<2, C>(Ld<S>{xin}, c, i, j, kk, lg, 0, xc);
            St<S>::st(xout + c, xc + wdiag * (fc - (C(4) * xc - s) * inv_h2));
        }
    }
}

// Residual at depth k, averaged into depth k-1 (fine blocks of 128 x 2 cells).
template <class S>
__global__ __launch_bounds__(kBlock) void kb_restrict(const S *__restrict__ F, const S *__restrict__ X,
                                                      S *__restrict__ Fc, const int *__restrict__ slot_prob,
                                                      const BProb *__restrict__ P, const BState *__restrict__ st,
                                                      const BGlobal *__restrict__ g, int k) {
    typedef typename St<S>::C C;
    constexpr int FX = RBlk<2>::FX;
    __shared__ C r[kBlock];
    const int lg = k + 2, n = 1 << lg, nc = n >> 1;
    const int bxn = n / FX, bpp = bxn * nc;
    const int slot = blockIdx.x / bpp;
    const int p = slot_prob[slot];
    if (g->stop || st[p].stop) return;
    const double h = depth_h(P[p], k);
    const C inv_h2 = C(1.0 / (h * h));
    const int64_t m = int64_t(n) * n;
    const S *f = F + slot * m, *x = X + slot * m;
    S *fc = Fc + int64_t(P[p].slot[k - 1]) * (m / 4);
    const int b = blockIdx.x % bpp, tid = threadIdx.x;
    const int bx = b % bxn, J = b / bxn;
    const int a = tid % FX, yb = tid / FX;
    const int i = bx * FX + a, j = 2 * J + yb;
    const int64_t c = (int64_t(j) << lg) | i;
    r[tid] = resid_at<2, S>(f, x, c, i, j, 0, lg, 0, inv_h2);
    __syncthreads();
    if (tid < FX / 2) {
        C acc = C(0);
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) acc += r[cy * FX + 2 * tid + cx];
        St<S>::st(fc + (int64_t(J) * nc + bx * (FX / 2) + tid), acc * C(0.25));
    }
}

// x(depth k) += P e(depth k-1), one thread per fine cell.
template <class S>
__global__ __launch_bounds__(kBlock) void kb_prolong(const S *__restrict__ Ec, S *__restrict__ X,
                                                     const int *__restrict__ slot_prob, const BProb *__restrict__ P,
                                                     const BState *__restrict__ st, const BGlobal *__restrict__ g,
                                                     int k) {
    typedef typename St<S>::C C;
    const int lg = k + 2, lgc = lg - 1, nc = 1 << lgc;
    const int64_t m = int64_t(1) << (2 * lg);
    const int bpp = int(m / kBlock);
    const int slot = blockIdx.x / bpp;
    const int p = slot_prob[slot];
    if (g->stop || st[p].stop) return;
    const int64_t c = int64_t(blockIdx.x % bpp) * kBlock + threadIdx.x;
    const S *ec = Ec + int64_t(P[p].slot[k - 1]) * (m / 4);
    S *x = X + slot * m;
    int i, j, kk;
    decode<2>(c, lg, i, j, kk);
    int oi, ni, oj, nj;
    float si, sj;
    pro_axis(i, nc, 0, oi, ni, si);
    pro_axis(j, nc, 0, oj, nj, sj);
    C s = C(0);
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            const C w = C(a ? 0.25 : 0.75) * C(b ? 0.25 : 0.75) * C(1.0);
            const C sg = C((a ? si : 1.0f) * (b ? sj : 1.0f) * 1.0f);
            s += w * (sg * St<S>::ld(ec + ((int64_t(b ? nj : oj) << lgc) | (a ? ni : oi))));
        }
    St<S>::st(x + c, St<S>::ld(x + c) + s);
}

// ------------------------------------------------------- row-marching tiles
// Level kernels of the depths above the tail (n >= 128), marching along y: a
// workgroup of kRmT threads is G = kRmT / TT groups of TT = min(n, 2 kRmT) / 2
// threads; each thread owns two adjacent columns (one vector access per row)
// and a group marches ry consecutive rows of one problem's grid, keeping rows
// j - 1, j, j + 1 of its columns in registers.  Column neighbours come from a
// row published in LDS (one barrier per row, two alternating buffers); the
// strip's edge threads load the cell beyond the strip.  Same terms, signs and
// summation orders as kb_sweep, kb_restrict and kb_prolong (Dirichlet ghosts).
constexpr int kRmT = 256;
constexpr int kRmBuf = 2 * kRmT + 2 * (kRmT / 64);  // G <= 4 groups (n >= 128) of 2 tt + 2 values

struct RmTile {
    int lg, n, tt, grp, l, i0, j0, slot;
};

// ry rows per group; the grid is slots x strips x row blocks
__device__ __forceinline__ RmTile rm_tile(int k, int ry) {
    RmTile t;
    t.lg = k + 2;
    t.n = 1 << t.lg;
    const int tw = t.n < 2 * kRmT ? t.n : 2 * kRmT;  // columns per group
    t.tt = tw / 2;
    const int G = kRmT / t.tt, strips = t.n / tw, rblk = t.n / (G * ry), per = strips * rblk;
    t.slot = int(blockIdx.x) / per;
    const int b = int(blockIdx.x) % per, strip = b % strips, rb = b / strips;
    t.grp = int(threadIdx.x) / t.tt;
    t.l = int(threadIdx.x) % t.tt;
    t.i0 = strip * tw + 2 * t.l;
    t.j0 = (rb * G + t.grp) * ry;
    return t;
}

inline unsigned rm_grid(int k, int ry, unsigned nsl) {
    const int n = 1 << (k + 2), tw = n < 2 * kRmT ? n : 2 * kRmT, G = kRmT / (tw / 2);
    return nsl * unsigned(n / tw) * unsigned(n / (G * ry));
}

// Rows per group: the most (up to 32, at least 4) that still give `wg`
// workgroups, enough to fill the chip (the tile setting the autotuner picks).
inline int rm_rows(int k, unsigned nsl, int wg) {
    int ry = 32;
    while (rm_grid(k, ry, nsl) < unsigned(wg) && ry > 4) ry /= 2;
    return ry;
}

// Marching state of one thread: its two cells on rows j - 1, j, j + 1 and the
// value beyond the strip edge on row j (edge threads only).
// Loads of a level field in storage S for RmRow: a pair at an even index, one value.
template <class S> struct PairLd {
    const S *x;
    __device__ __forceinline__ void pair(int64_t q, typename St<S>::C &a, typename St<S>::C &b) const {
        Pair<S>::ld(x + q, a, b);
    }
    __device__ __forceinline__ typename St<S>::C one(int64_t q) const { return St<S>::ld(x + q); }
};

template <class C, class L> struct RmRow {
    L ld;
    int lg, last, i0, hcol;
    bool hl, hr;  // this thread loads the left / right edge value
    C hsg;
    C m0, m1, c0, c1, p0, p1, hv;     // rows j - 1, j, j + 1; edge value of row j
    C q0, q1, hn;                     // prefetched: row j + 2, edge value of row j + 1
    __device__ RmRow(const L &ld_, const RmTile &t) : ld(ld_), lg(t.lg), last(t.n - 1), i0(t.i0) {
        hl = t.l == 0;
        hr = t.l == t.tt - 1;
        int hc = hl ? i0 - 1 : i0 + 2;
        hsg = C(1);
        if (hc < 0 || hc > last) {  // Dirichlet ghost: the edge cell itself, negated
            hc = hc < 0 ? 0 : last;
            hsg = C(-1);
        }
        hcol = hc;
    }
    __device__ __forceinline__ int64_t at(int j) const { return (int64_t(j) << lg) + i0; }
    __device__ __forceinline__ C edge(int j) const {
        return (hl || hr) ? hsg * ld.one((int64_t(j) << lg) + hcol) : C(0);
    }
    __device__ __forceinline__ void start(int j0) {
        ld.pair(at(j0), c0, c1);
        C a, b;
        ld.pair(at(j0 > 0 ? j0 - 1 : j0), a, b);
        m0 = j0 > 0 ? a : -c0;
        m1 = j0 > 0 ? b : -c1;
        ld.pair(at(j0 < last ? j0 + 1 : j0), a, b);
        p0 = j0 < last ? a : -c0;
        p1 = j0 < last ? b : -c1;
        hv = edge(j0);
    }
    // loads for the row after j (row j + 2 and the edge value of row j + 1)
    __device__ __forceinline__ void prefetch(int j) {
        const int j2 = j + 2 <= last ? j + 2 : last, j1 = j + 1 <= last ? j + 1 : last;
        C a, b;
        ld.pair(at(j2), a, b);
        q0 = j + 2 <= last ? a : -p0;
        q1 = j + 2 <= last ? b : -p1;
        hn = edge(j1);
    }
    // publish row j into buf (tt + 1 pairs wide, pair index l + 1) and form the
    // neighbour sums of the two cells
    __device__ __forceinline__ void sums(C *buf, int l, int tt, C &s0, C &s1) const {
        buf[2 * l + 1] = c0;
        buf[2 * l + 2] = c1;
        if (hl) buf[0] = hv;
        if (hr) buf[2 * tt + 1] = hv;
        __syncthreads();
        s0 = ((buf[2 * l] + c1) + m0) + p0;
        s1 = ((c0 + buf[2 * l + 3]) + m1) + p1;
    }
    __device__ __forceinline__ void advance() {
        m0 = c0;
        m1 = c1;
        c0 = p0;
        c1 = p1;
        p0 = q0;
        p1 = q1;
        hv = hn;
    }
};

template <class S>
__global__ __launch_bounds__(kRmT) void kb_sweep_rm(const S *__restrict__ F, const S *__restrict__ Xin,
                                                    S *__restrict__ Xout, const int *__restrict__ slot_prob,
                                                    const BProb *__restrict__ P, const BState *__restrict__ st,
                                                    const BGlobal *__restrict__ g, int k, int first, int cyc,
                                                    double omega, int ry) {
    typedef typename St<S>::C C;
    __shared__ C buf[2][kRmBuf];  // two alternating rows per workgroup; group g at offset g (2 tt + 2)
    const RmTile t = rm_tile(k, ry);
    const int p = slot_prob[t.slot];
    if (g->stop || st[p].stop) return;
    const double h = depth_h(P[p], k);
    const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / 4.0);
    const bool zero = first && (k < P[p].L || cyc == 0);
    const int64_t so = int64_t(t.slot) << (2 * t.lg);
    const S *f = F + so;
    S *xout = Xout + so;
    if (zero) {
        for (int j = t.j0; j < t.j0 + ry; ++j) {
            const int64_t c = (int64_t(j) << t.lg) + t.i0;
            C a, b;
            Pair<S>::ld(f + c, a, b);
            Pair<S>::st(xout + c, wdiag * a, wdiag * b);
        }
        return;
    }
    RmRow<C, PairLd<S>> r(PairLd<S>{Xin + so}, t);
    r.start(t.j0);
    C f0, f1;
    Pair<S>::ld(f + r.at(t.j0), f0, f1);
    const int go = t.grp * (2 * t.tt + 2);
    for (int j = t.j0, q = 0; j < t.j0 + ry; ++j, q ^= 1) {
        r.prefetch(j);
        C g0, g1;
        Pair<S>::ld(f + r.at(j + 1 <= r.last ? j + 1 : r.last), g0, g1);
        C s0, s1;
        r.sums(buf[q] + go, t.l, t.tt, s0, s1);
        const C o0 = r.c0 + wdiag * (f0 - (C(4) * r.c0 - s0) * inv_h2);
        const C o1 = r.c1 + wdiag * (f1 - (C(4) * r.c1 - s1) * inv_h2);
        Pair<S>::st(xout + r.at(j), o0, o1);
        f0 = g0;
        f1 = g1;
        r.advance();
    }
}

// Residual at depth k averaged into depth k - 1: each thread's column pair is
// one coarse column, each pair of rows one coarse row.  ry even.
template <class S>
__global__ __launch_bounds__(kRmT) void kb_restrict_rm(const S *__restrict__ F, const S *__restrict__ X,
                                                       S *__restrict__ Fc, const int *__restrict__ slot_prob,
                                                       const BProb *__restrict__ P, const BState *__restrict__ st,
                                                       const BGlobal *__restrict__ g, int k, int ry) {
    typedef typename St<S>::C C;
    __shared__ C buf[2][kRmBuf];
    const RmTile t = rm_tile(k, ry);
    const int p = slot_prob[t.slot];
    if (g->stop || st[p].stop) return;
    const double h = depth_h(P[p], k);
    const C inv_h2 = C(1.0 / (h * h));
    const int64_t so = int64_t(t.slot) << (2 * t.lg);
    const S *f = F + so;
    const int lgc = t.lg - 1;
    S *fc = Fc + (int64_t(P[p].slot[k - 1]) << (2 * lgc));
    RmRow<C, PairLd<S>> r(PairLd<S>{X + so}, t);
    r.start(t.j0);
    C f0, f1;
    Pair<S>::ld(f + r.at(t.j0), f0, f1);
    const int go = t.grp * (2 * t.tt + 2);
    C acc = C(0);
    for (int j = t.j0, q = 0; j < t.j0 + ry; ++j, q ^= 1) {
        r.prefetch(j);
        C g0, g1;
        Pair<S>::ld(f + r.at(j + 1 <= r.last ? j + 1 : r.last), g0, g1);
        C s0, s1;
        r.sums(buf[q] + go, t.l, t.tt, s0, s1);
        const C r0 = f0 - (C(4) * r.c0 - s0) * inv_h2;
        const C r1 = f1 - (C(4) * r.c1 - s1) * inv_h2;
        if (!(j & 1)) acc = C(0);
        acc += r0;
        acc += r1;
        if (j & 1) St<S>::st(fc + ((int64_t(j >> 1) << lgc) + (t.i0 >> 1)), acc * C(0.25));
        f0 = g0;
        f1 = g1;
        r.advance();
    }
}

// x(depth k) += P e(depth k - 1): each thread's column pair shares its own
// coarse column; coarse rows J - 1, J, J + 1 (three values each: columns
// I - 1, I, I + 1, clamped; ghost signs applied per term) stay in registers.
template <class S>
__global__ __launch_bounds__(kRmT) void kb_prolong_rm(const S *__restrict__ Ec, S *__restrict__ X,
                                                      const int *__restrict__ slot_prob, const BProb *__restrict__ P,
                                                      const BState *__restrict__ st, const BGlobal *__restrict__ g,
                                                      int k, int ry) {
    typedef typename St<S>::C C;
    const RmTile t = rm_tile(k, ry);
    const int p = slot_prob[t.slot];
    if (g->stop || st[p].stop) return;
    const int lgc = t.lg - 1, nc = t.n >> 1, I = t.i0 >> 1;
    const S *ec = Ec + (int64_t(P[p].slot[k - 1]) << (2 * lgc));
    S *x = X + (int64_t(t.slot) << (2 * t.lg));
    // columns: own I; left neighbour (ghost at I = 0: own, sign -1); right (ghost at nc - 1)
    const int cl = I > 0 ? I - 1 : 0, cr = I < nc - 1 ? I + 1 : nc - 1;
    const float sl = I > 0 ? 1.0f : -1.0f, sr = I < nc - 1 ? 1.0f : -1.0f;
    auto row = [&](int J, C &a, C &b, C &c) {
        const S *e = ec + (int64_t(J) << lgc);
        a = St<S>::ld(e + cl);
        b = St<S>::ld(e + I);
        c = St<S>::ld(e + cr);
    };
    const int J0 = t.j0 >> 1;
    C ma, mb, mc, ca, cb, cc, pa, pb, pc;
    row(J0 > 0 ? J0 - 1 : 0, ma, mb, mc);
    row(J0, ca, cb, cc);
    row(J0 < nc - 1 ? J0 + 1 : nc - 1, pa, pb, pc);
    const C w00 = C(0.75) * C(0.75) * C(1.0), w10 = C(0.25) * C(0.75) * C(1.0);
    const C w01 = C(0.75) * C(0.25) * C(1.0), w11 = C(0.25) * C(0.25) * C(1.0);
    for (int J = J0; J < J0 + ry / 2; ++J) {
        C na = C(0), nb = C(0), ncv = C(0);
        if (J + 1 < J0 + ry / 2) row(J + 2 <= nc - 1 ? J + 2 : nc - 1, na, nb, ncv);
        for (int dy = 0; dy < 2; ++dy) {
            const int j = 2 * J + dy;
            // neighbour coarse row and its sign
            const bool ghost = dy ? J == nc - 1 : J == 0;
            const float sj = ghost ? -1.0f : 1.0f;
            const C ra = dy ? pa : ma, rb = dy ? pb : mb, rc = dy ? pc : mc;
            C v0, v1;
            Pair<S>::ld(x + ((int64_t(j) << t.lg) + t.i0), v0, v1);
            // left fine cell: own column I, neighbour I - 1
            C s = C(0);
            s += w00 * (C(1.0f * 1.0f * 1.0f) * cb);
            s += w10 * (C(sl * 1.0f * 1.0f) * ca);
            s += w01 * (C(1.0f * sj * 1.0f) * rb);
            s += w11 * (C(sl * sj * 1.0f) * ra);
            // right fine cell: own column I, neighbour I + 1
            C u = C(0);
            u += w00 * (C(1.0f * 1.0f * 1.0f) * cb);
            u += w10 * (C(sr * 1.0f * 1.0f) * cc);
            u += w01 * (C(1.0f * sj * 1.0f) * rb);
            u += w11 * (C(sr * sj * 1.0f) * rc);
            Pair<S>::st(x + ((int64_t(j) << t.lg) + t.i0), v0 + s, v1 + u);
        }
        // rows J, J + 1, J + 2 become J - 1, J, J + 1 (a ghost row J + 1 = J at the top is J itself)
        const bool top = J + 1 == nc - 1;
        ma = ca; mb = cb; mc = cc;
        ca = pa; cb = pb; cc = pc;
        pa = top ? ca : na; pb = top ? cb : nb; pc = top ? cc : ncv;
    }
}

// Refinement blocks of kb_ir_rm: on a problem with n >= 128 a row-marching
// tile (strip a, row block b: G groups of kIrRows rows), else kIrCells
// consecutive cells from a (b = -1).
struct BIr {
    int p, a, b;
};
constexpr int kIrRows = 16;

// x_b = x_a + e (has_e) in FP64, as kb_ir forms it.
template <class SL> struct IrLd {
    const double *x;
    const SL *e;
    int he;
    __device__ __forceinline__ double one(int64_t q) const { return he ? x[q] + double(St<SL>::ld(e + q)) : x[q]; }
    __device__ __forceinline__ double operator()(int64_t q) const { return one(q); }
    __device__ __forceinline__ void pair(int64_t q, double &a, double &b) const {
        Pair<double>::ld(x + q, a, b);
        if (he) {
            typename St<SL>::C u, v;
            Pair<SL>::ld(e + q, u, v);
            a = a + double(u);
            b = b + double(v);
        }
    }
};

// kb_ir on row-marching tiles (problems with n >= 128; smaller ones as kb_ir):
// the same values per cell; one partial per block.
template <class SL>
__global__ __launch_bounds__(kBlock) void kb_ir_rm(BPtrs<SL> ptr, SL *const *epool, SL *const *rpool,
                                                   const BIr *__restrict__ blk, const BProb *__restrict__ P,
                                                   const BState *__restrict__ st, const BGlobal *__restrict__ g,
                                                   double *__restrict__ partial, int has_e) {
    static_assert(kBlock == kRmT, "row-marching refinement tiles use the level kernels' workgroup");
    __shared__ double buf[2][kRmBuf];
    const BIr bk = blk[blockIdx.x];
    if (g->stop || st[bk.p].stop) return;
    const BProb &pp = P[bk.p];
    const int lg = pp.L + 2, n = 1 << lg;
    const int64_t m = int64_t(1) << (2 * lg);
    const double inv_h2 = 1.0 / (pp.h * pp.h);
    const int64_t so = int64_t(pp.slot[pp.L]) * m;
    const SL *e = epool[pp.L] + so;
    SL *rlo = rpool[pp.L] + so;
    const double *f = ptr.f[bk.p];
    double *xo = ptr.xb[bk.p];
    const IrLd<SL> ldx{ptr.xa[bk.p], e, has_e};
    double acc = 0.0;
    if (n < 128) {
        for (int u = 0; u < kIrCells / kBlock; ++u) {
            const int64_t c = int64_t(bk.a) + u * kBlock + threadIdx.x;
            if (c < m) {
                int i, j, k;
                decode<2>(c, lg, i, j, k);
                const double xc = ldx(c);
                const double s = nb_sum<2, double>(ldx, c, i, j, k, lg, 0, xc);
                const double r = f[c] - (4.0 * xc - s) * inv_h2;
                if (has_e) xo[c] = xc;
                St<SL>::st(rlo + c, typename St<SL>::C(r));
                acc += r * r;
            }
        }
    } else {
        RmTile t;
        t.lg = lg;
        t.n = n;
        const int tw = n < 2 * kRmT ? n : 2 * kRmT, G = kRmT / (tw / 2);
        t.tt = tw / 2;
        t.grp = int(threadIdx.x) / t.tt;
        t.l = int(threadIdx.x) % t.tt;
        t.i0 = bk.a * tw + 2 * t.l;
        t.j0 = (bk.b * G + t.grp) * kIrRows;
        t.slot = 0;
        RmRow<double, IrLd<SL>> r(ldx, t);
        r.start(t.j0);
        double f0, f1;
        Pair<double>::ld(f + r.at(t.j0), f0, f1);
        const int go = t.grp * (2 * t.tt + 2);
        for (int j = t.j0, q = 0; j < t.j0 + kIrRows; ++j, q ^= 1) {
            r.prefetch(j);
            double g0, g1;
            Pair<double>::ld(f + r.at(j + 1 <= r.last ? j + 1 : r.last), g0, g1);
            double s0, s1;
            r.sums(buf[q] + go, t.l, t.tt, s0, s1);
            const double r0 = f0 - (4.0 * r.c0 - s0) * inv_h2;
            const double r1 = f1 - (4.0 * r.c1 - s1) * inv_h2;
            if (has_e) Pair<double>::st(xo + r.at(j), r.c0, r.c1);
            Pair<SL>::st(rlo + r.at(j), typename St<SL>::C(r0), typename St<SL>::C(r1));
            acc += r0 * r0;
            acc += r1 * r1;
            f0 = g0;
            f1 = g1;
            r.advance();
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Depths min(L_p, kTailDepth) .. 0 of every problem, one workgroup each.
template <class S>
__global__ __launch_bounds__(Tail<2>::NT_B) void kb_tail(S *const *Xpool, S *const *Fpool, const double *__restrict__ Minv1,
                                                       const BProb *__restrict__ P, const BState *__restrict__ st,
                                                       const BGlobal *__restrict__ g, int cyc, double omega, int nu1,
                                                       int nu2) {
    typedef typename St<S>::C C;
    __shared__ C xs[Tail<2>::levels_sum()];
    __shared__ C fs[Tail<2>::levels_sum()];
    __shared__ C ts[Tail<2>::cells(Tail<2>::LG)];
    const int p = blockIdx.x;
    if (g->stop || st[p].stop) return;
    const BProb &pp = P[p];
    const int t = min(pp.L, kTailDepth);
    const int64_t m = int64_t(1) << (2 * (t + 2));
    S *x = Xpool[t] + int64_t(pp.slot[t]) * m;
    const S *f = Fpool[t] + int64_t(pp.slot[t]) * m;
    const bool warm = t == pp.L && cyc > 0;
    const double h = depth_h(pp, t);
    // Minv1 is the inverse for unit coarsest spacing; the coarsest spacing here
    // is h * 2^t, and the Dirichlet operator scales as 1/h^2.
    const double hc = h * double(1 << t);
    __shared__ double Ms[16 * 16];
    for (int q = threadIdx.x; q < 256; q += blockDim.x) Ms[q] = Minv1[q] * (hc * hc);
    __syncthreads();
    tail_cycle<2, S, Tail<2>::NT_B>(xs, fs, ts, f, x, warm ? x : nullptr, Ms, t + 2, 0, h, omega, nu1, nu2);
}

// ----------------------------------------------------------------- plan
struct Plan {
    int dev = 0, nprob = 0, K = 0;
    np_prec prec = NP_FP32;
    size_t es = 4;
    std::vector<int> L;                        // finest depth per problem
    std::vector<std::vector<int>> slots;       // per depth: problems present
    std::vector<void *> X, F, T;               // per depth pools
    std::vector<int *> d_slot_prob;            // per depth
    void **d_Xpool = nullptr, **d_Fpool = nullptr;
    BProb *d_P = nullptr;
    BState *d_st = nullptr, *h_st = nullptr;
    BGlobal *d_g = nullptr, *h_g = nullptr;
    BBlk *d_blk = nullptr;
    int nblk = 0;
    BIr *d_irblk = nullptr;
    int nirblk = 0;
    double *d_partial = nullptr;
    double *d_Minv1 = nullptr;
    double *ypool = nullptr;                   // second FP64 iterate of every problem
    const double **d_f = nullptr;
    double **d_x = nullptr, **d_y = nullptr;
    std::vector<double *> y;                   // host copy of the pool pointers
    std::vector<double> h;                     // finest spacing per problem (for graph keys)
    double omega_tune = 2.0 / 3.0;             // relaxation weight of the autotuner's trials
    hipStream_t cap = nullptr;
    std::map<std::tuple<int, int, int, int, int, int, int>, hipGraphExec_t> graphs;  // (kind, inner, nu1, nu2, omega bits, rm, wg)
    std::mutex mu;
};

std::mutex g_plan_mu;
std::map<std::vector<int64_t>, Plan *> g_plans;

// Settings of a batched solve chosen by the autotuner: inner cycles per
// refinement step, sweeps per level (nu1 = nu2 = nu) and the level-kernel
// tiles (row-marching on/off, workgroups a row-marching launch aims for), with
// the tuned batch's time.
struct BTuned {
    int inner = 0, nu = 2, rm = 1, wg = 4096;
    double ms = 0.0;
};
std::map<std::string, BTuned> g_tuned;  // cache key -> settings (this process)

np_status dmalloc(void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of %zu bytes failed", bytes);
        return NP_ENOMEM;
    }
    return NP_OK;
}

void free_plan(Plan *B) {
    for (auto &kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto *p : B->X) (void)hipFree(p);
    for (auto *p : B->F) (void)hipFree(p);
    for (auto *p : B->T) (void)hipFree(p);
    for (auto *p : B->d_slot_prob) (void)hipFree(p);
    void *q[] = {B->d_Xpool, B->d_Fpool, B->d_P, B->d_st, B->d_g, B->d_blk, B->d_irblk, B->d_partial, B->d_Minv1,
                 B->ypool, (void *)B->d_f, B->d_x, B->d_y};
    for (auto *p : q) if (p) (void)hipFree(p);
    if (B->h_st) (void)hipHostFree(B->h_st);
    if (B->h_g) (void)hipHostFree(B->h_g);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
}

template <class T> np_status upload(T **d, const std::vector<T> &h) {
    NP_TRY(dmalloc((void **)d, sizeof(T) * std::max<size_t>(1, h.size())));
    NP_HIP_TRY(hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return NP_OK;
}

np_status build_plan(const std::vector<int> &lgs, const std::vector<double> &hs, np_prec prec, Plan *B) {
    const int np_ = int(lgs.size());
    B->nprob = np_;
    B->prec = prec;
    B->es = prec_bytes(prec);
    B->h = hs;
    B->L.resize(np_);
    int K = 0;
    for (int p = 0; p < np_; ++p) {
        B->L[p] = lgs[p] - 2;
        K = std::max(K, B->L[p]);
    }
    B->K = K;
    B->slots.assign(K + 1, {});
    std::vector<BProb> P(np_);
    for (int p = 0; p < np_; ++p) {
        std::memset(&P[p], 0, sizeof(BProb));
        P[p].L = B->L[p];
        P[p].h = hs[p];
        for (int k = 0; k <= kMaxDepth; ++k) P[p].slot[k] = -1;
        for (int k = 0; k <= B->L[p]; ++k) {
            P[p].slot[k] = int(B->slots[k].size());
            B->slots[k].push_back(p);
        }
    }
    B->X.assign(K + 1, nullptr);
    B->F.assign(K + 1, nullptr);
    B->T.assign(K + 1, nullptr);
    B->d_slot_prob.assign(K + 1, nullptr);
    for (int k = 0; k <= K; ++k) {
        const size_t bytes = B->slots[k].size() * (size_t(1) << (2 * (k + 2))) * B->es;
        NP_TRY(dmalloc(&B->X[k], bytes));
        NP_TRY(dmalloc(&B->F[k], bytes));
        NP_TRY(dmalloc(&B->T[k], bytes));
        NP_TRY(upload(&B->d_slot_prob[k], B->slots[k]));
    }
    // refinement blocks
    std::vector<BBlk> blk;
    for (int p = 0; p < np_; ++p) {
        const int64_t m = int64_t(1) << (2 * lgs[p]);
        P[p].first_block = int(blk.size());
        for (int64_t b = 0; b < m; b += kIrCells) blk.push_back(BBlk{p, int(b)});
        P[p].nblocks = int(blk.size()) - P[p].first_block;
    }
    B->nblk = int(blk.size());
    NP_TRY(upload(&B->d_blk, blk));
    std::vector<BIr> irb;
    for (int p = 0; p < np_; ++p) {
        const int n = 1 << lgs[p];
        P[p].ir_first = int(irb.size());
        if (n >= 128) {
            const int tw = std::min(n, 2 * kRmT), G = kRmT / (tw / 2);
            for (int b = 0; b < n / (G * kIrRows); ++b)
                for (int a = 0; a < n / tw; ++a) irb.push_back(BIr{p, a, b});
        } else {
            for (int64_t c = 0; c < int64_t(n) * n; c += kIrCells) irb.push_back(BIr{p, int(c), -1});
        }
        P[p].ir_nblocks = int(irb.size()) - P[p].ir_first;
    }
    B->nirblk = int(irb.size());
    NP_TRY(upload(&B->d_irblk, irb));
    NP_TRY(upload(&B->d_P, P));
    NP_TRY(upload(&B->d_Xpool, B->X));
    NP_TRY(upload(&B->d_Fpool, B->F));
    NP_TRY(dmalloc((void **)&B->d_partial, sizeof(double) * std::max(B->nblk, B->nirblk)));
    NP_TRY(dmalloc((void **)&B->d_st, sizeof(BState) * np_));
    NP_TRY(dmalloc((void **)&B->d_g, sizeof(BGlobal)));
    if (hipHostMalloc((void **)&B->h_st, sizeof(BState) * np_, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&B->h_g, sizeof(BGlobal), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc failed");
        return NP_ENOMEM;
    }
    std::vector<double> inv;
    if (!coarse_inverse_host(2, NP_BC_DIRICHLET0, 1.0, inv)) {
        set_error("singular coarsest operator");
        return NP_EINVAL;
    }
    NP_TRY(upload(&B->d_Minv1, inv));
    int64_t ytot = 0;
    for (int p = 0; p < np_; ++p) ytot += int64_t(1) << (2 * lgs[p]);
    NP_TRY(dmalloc((void **)&B->ypool, sizeof(double) * ytot));
    B->y.resize(np_);
    int64_t o = 0;
    for (int p = 0; p < np_; ++p) {
        B->y[p] = B->ypool + o;
        o += int64_t(1) << (2 * lgs[p]);
    }
    NP_TRY(upload(&B->d_y, B->y));
    NP_TRY(dmalloc((void **)&B->d_f, sizeof(double *) * np_));
    NP_TRY(dmalloc((void **)&B->d_x, sizeof(double *) * np_));
    NP_HIP_TRY(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    return NP_OK;
}

struct BOpts {
    int nu1, nu2;
    double omega;
    int rm;  // row-marching level kernels above the tail depths (else one cell pair per thread)
    int wg;  // row-marching: workgroups a level launch aims for (sets the rows per group)
};

// One refinement step: kind 0 (x_a = caller x, no correction yet), 1 (x -> y),
// 2 (y -> x); then `inner` batched V-cycles on the rounded residuals.
template <class S>
np_status enqueue_step(Plan *B, int kind, int inner, const BOpts &o, hipStream_t s) {
    BPtrs<S> ptr;
    ptr.f = B->d_f;
    ptr.xa = kind == 2 ? (const double *const *)B->d_y : (const double *const *)B->d_x;
    ptr.xb = kind == 1 ? B->d_y : B->d_x;
    S *const *Xp = (S *const *)B->d_Xpool, *const *Fp = (S *const *)B->d_Fpool;
    if (o.rm)
        hipLaunchKernelGGL((kb_ir_rm<S>), dim3(B->nirblk), dim3(kBlock), 0, s, ptr, Xp, Fp, B->d_irblk, B->d_P,
                           B->d_st, B->d_g, B->d_partial, kind == 0 ? 0 : 1);
    else
        hipLaunchKernelGGL((kb_ir<S>), dim3(B->nblk), dim3(kBlock), 0, s, ptr, Xp, Fp, B->d_blk, B->d_P, B->d_st,
                           B->d_g, B->d_partial, kind == 0 ? 0 : 1);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(kb_check, dim3(unsigned((B->nprob + 3) / 4)), dim3(256), 0, s, B->d_partial, B->d_P, B->d_st,
                       B->d_g, B->nprob, o.rm);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(kb_check_any, dim3(1), dim3(1024), 0, s, B->d_st, B->d_g, B->nprob);
    NP_LAUNCH_CHECK();
    for (int c = 0; c < inner; ++c) {
        for (int k = B->K; k > kTailDepth; --k) {
            const unsigned nsl = unsigned(B->slots[k].size());
            const int64_t m = int64_t(1) << (2 * (k + 2));
            S *cur = (S *)B->X[k], *oth = (S *)B->T[k];
            const S *F = (const S *)B->F[k];
            const int ry = rm_rows(k, nsl, o.wg);
            for (int it = 0; it < o.nu1; ++it) {
                if (o.rm)
                    hipLaunchKernelGGL((kb_sweep_rm<S>), dim3(rm_grid(k, ry, nsl)), dim3(kRmT), 0, s, F, cur, oth,
                                       B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k, it == 0 ? 1 : 0, c, o.omega, ry);
                else
                    hipLaunchKernelGGL((kb_sweep<S>), dim3(unsigned(nsl * ((m + kSweepCells - 1) / kSweepCells))),
                                       dim3(kBlock), 0, s, F, cur, oth, B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k,
                                       it == 0 ? 1 : 0, c, o.omega);
                NP_LAUNCH_CHECK();
                std::swap(cur, oth);
            }
            const int n = 1 << (k + 2);
            if (o.rm)
                hipLaunchKernelGGL((kb_restrict_rm<S>), dim3(rm_grid(k, ry, nsl)), dim3(kRmT), 0, s, F, cur,
                                   (S *)B->F[k - 1], B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k, ry);
            else
                hipLaunchKernelGGL((kb_restrict<S>), dim3(unsigned(nsl * (n / RBlk<2>::FX) * (n / 2))), dim3(kBlock), 0,
                                   s, F, cur, (S *)B->F[k - 1], B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k);
            NP_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL((kb_tail<S>), dim3(B->nprob), dim3(Tail<2>::NT_B), 0, s, Xp, Fp, B->d_Minv1, B->d_P,
                           B->d_st, B->d_g, c, o.omega, o.nu1, o.nu2);
        NP_LAUNCH_CHECK();
        for (int k = kTailDepth + 1; k <= B->K; ++k) {
            const unsigned nsl = unsigned(B->slots[k].size());
            const int64_t m = int64_t(1) << (2 * (k + 2));
            // after an odd number of pre-sweeps the iterate sits in T
            S *cur = (o.nu1 & 1) ? (S *)B->T[k] : (S *)B->X[k];
            S *oth = (o.nu1 & 1) ? (S *)B->X[k] : (S *)B->T[k];
            const int ry = rm_rows(k, nsl, o.wg);
            if (o.rm)
                hipLaunchKernelGGL((kb_prolong_rm<S>), dim3(rm_grid(k, ry, nsl)), dim3(kRmT), 0, s,
                                   (const S *)B->X[k - 1], cur, B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k, ry);
            else
                hipLaunchKernelGGL((kb_prolong<S>), dim3(unsigned(nsl * (m / kBlock))), dim3(kBlock), 0, s,
                                   (const S *)B->X[k - 1], cur, B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k);
            NP_LAUNCH_CHECK();
            for (int it = 0; it < o.nu2; ++it) {
                if (o.rm)
                    hipLaunchKernelGGL((kb_sweep_rm<S>), dim3(rm_grid(k, ry, nsl)), dim3(kRmT), 0, s,
                                       (const S *)B->F[k], cur, oth, B->d_slot_prob[k], B->d_P, B->d_st, B->d_g, k, 0,
                                       c, o.omega, ry);
                else
                    hipLaunchKernelGGL((kb_sweep<S>), dim3(unsigned(nsl * ((m + kSweepCells - 1) / kSweepCells))),
                                       dim3(kBlock), 0, s, (const S *)B->F[k], cur, oth, B->d_slot_prob[k], B->d_P,
                                       B->d_st, B->d_g, k, 0, c, o.omega);
                NP_LAUNCH_CHECK();
                std::swap(cur, oth);
            }
        }
    }
    return NP_OK;
}

template <class S>
np_status run_step(Plan *B, int kind, int inner, const BOpts &o, hipStream_t s) {
    if (!g_batched_graphs) return enqueue_step<S>(B, kind, inner, o, s);
    int64_t ob;
    std::memcpy(&ob, &o.omega, sizeof ob);
    const auto key = std::make_tuple(kind, inner, o.nu1, o.nu2, int(ob ^ (ob >> 32)), o.rm, o.wg);
    auto it = B->graphs.find(key);
    if (it == B->graphs.end()) {
        NP_HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        np_status st = enqueue_step<S>(B, kind, inner, o, B->cap);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(B->cap, &graph);
        if (st != NP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return NP_EHIP;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(e));
            return NP_EHIP;
        }
        it = B->graphs.emplace(key, exec).first;
    }
    NP_HIP_TRY(hipGraphLaunch(it->second, s));
    return NP_OK;
}

// Full batched solve with a given inner cycle count.  Caller pointers are in
// the plan's pointer tables already.
template <class S>
np_status batched_run(Plan *B, int inner, const BOpts &o, const np_mg_opts &mo, double tol, hipStream_t s) {
    BGlobal *g = B->h_g;
    std::memset(g, 0, sizeof *g);
    g->fixed = mo.fixed_cycles;
    g->maxc = mo.max_cycles;
    g->tol = tol;
    NP_HIP_TRY(hipMemcpyAsync(B->d_g, g, sizeof *g, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(kb_zero, dim3(B->nblk), dim3(kBlock), 0, s, B->d_x, B->d_blk, B->d_P);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(kb_fnorm, dim3(B->nblk), dim3(kBlock), 0, s, (const double *const *)B->d_f, B->d_blk, B->d_P,
                       B->d_partial);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(kb_nf, dim3(1), dim3(1024), 0, s, B->d_partial, B->d_P, B->d_st, B->nprob);
    NP_LAUNCH_CHECK();
    NP_TRY(run_step<S>(B, 0, inner, o, s));
    int launched = 1, batch = mo.fixed_cycles > 0 ? mo.fixed_cycles : 4;
    for (;;) {
        for (int b = 0; b < batch; ++b, ++launched) NP_TRY(run_step<S>(B, (launched & 1) ? 1 : 2, inner, o, s));
        NP_HIP_TRY(hipMemcpyAsync(B->h_g, B->d_g, sizeof(BGlobal), hipMemcpyDeviceToHost, s));
        NP_HIP_TRY(hipStreamSynchronize(s));
        if (B->h_g->stop) break;
        batch = 2;
        if (launched > 4 * (mo.max_cycles + 2) + 16) {
            set_error("batched solve did not stop");
            return NP_ENOCONV;
        }
    }
    hipLaunchKernelGGL(kb_final_copy, dim3(B->nblk), dim3(kBlock), 0, s, (const double *const *)B->d_y, B->d_x,
                       B->d_blk, B->d_P, B->d_st);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipMemcpyAsync(B->h_st, B->d_st, sizeof(BState) * B->nprob, hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// ---------------------------------------------------- autotuning cache
// The tuned settings persist in a small JSON file keyed by (GPU architecture,
// precision, omega, the multiset of problem sizes): $NEUPHYS_TUNE_CACHE if set
// (empty: no file), else $XDG_CACHE_HOME/neuphys/batched_autotune.json, else
// $HOME/.cache/neuphys/batched_autotune.json.  One entry per line:
//   "<key>": {"inner": 4, "nu": 2, "rm": 1, "wg": 4096, "ms": 52.3},
// A missing or unreadable file is a cache miss; a failed write is ignored.
std::string tune_cache_path() {
    if (const char *e = std::getenv("NEUPHYS_TUNE_CACHE")) return std::string(e);
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/neuphys/batched_autotune.json";
    if (const char *h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/neuphys/batched_autotune.json";
    return std::string();
}

std::map<std::string, BTuned> read_tune_file(const std::string &path) {
    std::map<std::string, BTuned> out;
    if (path.empty()) return out;
    FILE *fp = std::fopen(path.c_str(), "r");
    if (!fp) return out;
    char line[4096];
    while (std::fgets(line, sizeof line, fp)) {
        const char *a = std::strchr(line, '"');
        const char *b = a ? std::strchr(a + 1, '"') : nullptr;
        if (!b || b[1] != ':') continue;
        BTuned t;
        if (std::sscanf(b + 1, ": {\"inner\": %d, \"nu\": %d, \"rm\": %d, \"wg\": %d, \"ms\": %lf}", &t.inner, &t.nu,
                        &t.rm, &t.wg, &t.ms) == 5 &&
            t.inner >= 1 && t.inner <= 16 && t.nu >= 1 && t.nu <= 16 && (t.rm == 0 || t.rm == 1) && t.wg >= 1)
            out[std::string(a + 1, b)] = t;
    }
    std::fclose(fp);
    return out;
}

void write_tune_file(const std::string &path, const std::string &key, const BTuned &t) {
    if (path.empty()) return;
    auto all = read_tune_file(path);
    all[key] = t;
    for (size_t i = 1; i < path.size(); ++i)  // parent directories
        if (path[i] == '/') (void)::mkdir(path.substr(0, i).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string(::getpid());
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\"neuphys_batched_autotune\": 1, \"entries\": {\n");
    size_t i = 0;
    for (const auto &kv : all)
        std::fprintf(fp, "\"%s\": {\"inner\": %d, \"nu\": %d, \"rm\": %d, \"wg\": %d, \"ms\": %.4f}%s\n",
                     kv.first.c_str(), kv.second.inner, kv.second.nu, kv.second.rm, kv.second.wg, kv.second.ms,
                     ++i < all.size() ? "," : "");
    std::fprintf(fp, "}}\n");
    const bool ok = std::fclose(fp) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}

// Cache key: architecture, precision, omega and the sorted multiset of sizes.
std::string tune_key(int dev, int prec, double omega, std::vector<int> lgs) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    else (void)hipGetLastError();
    std::sort(lgs.begin(), lgs.end());
    char buf[96];
    uint64_t ob;
    std::memcpy(&ob, &omega, sizeof ob);
    std::snprintf(buf, sizeof buf, "|%s|omega=%016llx|", prec == NP_FP32 ? "fp32" : "fp64", (unsigned long long)ob);
    std::string key = arch + buf;
    for (size_t i = 0; i < lgs.size();) {
        size_t j = i;
        while (j < lgs.size() && lgs[j] == lgs[i]) ++j;
        key += std::to_string(1 << lgs[i]) + "x" + std::to_string(j - i) + (j < lgs.size() ? "," : "");
        i = j;
    }
    return key;
}

// Picks the batch's settings by timing full solves of it: first the inner
// cycles and sweeps per level jointly (inner 1..4 x nu 1..3 on row-marching
// tiles aiming at 4096 workgroups), then the tiles for the winner (one cell
// pair per thread; row-marching aiming at 1024 or 16384 workgroups).  A
// candidate counts only if every problem converged; each runs once untimed
// (capturing its graphs) and is timed as the faster of two runs.
template <class Run>
np_status autotune(Plan *B, int nprob, hipStream_t s, Run &run, int default_inner, BTuned *out) {
    struct Ev {
        hipEvent_t a = nullptr, b = nullptr;
        ~Ev() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    NP_HIP_TRY(hipEventCreate(&ev.a));
    NP_HIP_TRY(hipEventCreate(&ev.b));
    BTuned best;
    best.ms = 1e300;
    bool found = false;
    auto trial = [&](const BTuned &c) -> np_status {
        const BOpts bo{c.nu, c.nu, B->omega_tune, c.rm, c.wg};
        NP_TRY(run(c.inner, bo));
        float tmin = 1e30f;
        for (int r = 0; r < 2; ++r) {
            NP_HIP_TRY(hipEventRecord(ev.a, s));
            NP_TRY(run(c.inner, bo));
            NP_HIP_TRY(hipEventRecord(ev.b, s));
            NP_HIP_TRY(hipEventSynchronize(ev.b));
            float ms = 0.0f;
            NP_HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
            tmin = std::min(tmin, ms);
        }
        bool ok = true;
        for (int p = 0; p < nprob; ++p) ok = ok && B->h_st[p].stop == kConverged;
        if (ok && tmin < best.ms) {
            best = c;
            best.ms = tmin;
            found = true;
        }
        return NP_OK;
    };
    for (int nu = 1; nu <= 3; ++nu)
        for (int inner = 1; inner <= 4; ++inner) {
            BTuned c;
            c.inner = inner;
            c.nu = nu;
            c.rm = 1;
            c.wg = 4096;
            NP_TRY(trial(c));
        }
    if (found) {
        const BTuned w = best;
        const int tiles[3][2] = {{0, 4096}, {1, 1024}, {1, 16384}};
        for (auto &tl : tiles) {
            BTuned c = w;
            c.rm = tl[0];
            c.wg = tl[1];
            NP_TRY(trial(c));
        }
        *out = best;
    } else {
        BTuned d;
        d.inner = default_inner;
        *out = d;
    }
    return NP_OK;
}

}  // namespace

int g_batched_graphs = 1;
int g_batched_autotune = 1;
int g_batched_rm = 1;
int g_batched_wg = 4096;
static thread_local int g_last_tune_inner = 0;
static thread_local double g_last_tune_ms = 0.0;
static thread_local int g_last_settings[6] = {0, 0, 0, 0, 0, 0};  // inner, nu1, nu2, rm, wg, source

void release_batched_cache() {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto &kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    g_tuned.clear();
}

}  // namespace np

using namespace np;

extern "C" np_status mg_poisson_solve_batched(int nprob, const np_dims *dims, const double *h, np_bc bc,
                                              const double *const *rhs, double *const *x, double tol,
                                              const np_mg_opts *opts, np_mg_stats *stats) {
    clear_error();
    if (nprob <= 0 || nprob > 65536 || !dims || !h || !rhs || !x) {
        set_error("bad batch arguments");
        return NP_EINVAL;
    }
    if (bc != NP_BC_DIRICHLET0) { set_error("batched solves support zero Dirichlet boundaries only"); return NP_EINVAL; }
    np_mg_opts o;
    np_default_opts(&o);
    if (opts) o = *opts;
    if (o.smooth_prec != NP_FP32 && o.smooth_prec != NP_FP64) {
        set_error("batched solves run FP32 (or FP64) inner cycles");
        return NP_EINVAL;
    }
    if (o.warm_start != 0) { set_error("batched solves start from zero"); return NP_EINVAL; }
    if (o.cycle != 0 || o.prolong != 0) { set_error("batched solves run V-cycles"); return NP_EINVAL; }
    if (o.nu1 < 1 || o.nu2 < 0 || ((o.nu1 + o.nu2) & 1) || o.nu1 > 16 || o.nu2 > 16 ||
        !(o.omega > 0.0 && o.omega < 2.0) || o.inner_cycles < 0 || o.inner_cycles > 16 || o.max_cycles < 0 ||
        o.fixed_cycles < 0 || o.max_cycles > 100000 || o.fixed_cycles > 100000) {
        set_error("bad cycle settings (batched: nu1 >= 1, nu1 + nu2 even)");
        return NP_EINVAL;
    }
    if (o.fixed_cycles <= 0 && !(tol > 0.0)) { set_error("tol must be positive"); return NP_EINVAL; }
    std::vector<int> lgs(nprob);
    std::vector<double> hs(nprob);
    for (int p = 0; p < nprob; ++p) {
        if (dims[p].ndim != 2 || dims[p].n[0] != dims[p].n[1] || !is_pow2(dims[p].n[0]) || dims[p].n[0] < 4 ||
            dims[p].n[0] > (int64_t(4) << kMaxDepth)) {
            set_error("problem %d: batched grids are 2D, n x n, n a power of two in [4, %d]", p, 4 << kMaxDepth);
            return NP_EINVAL;
        }
        if (!(h[p] > 0.0) || !rhs[p] || !x[p]) { set_error("problem %d: bad h or null pointer", p); return NP_EINVAL; }
        lgs[p] = ilog2(dims[p].n[0]);
        hs[p] = h[p];
    }
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    std::vector<int64_t> key;
    key.push_back(dev);
    key.push_back(o.smooth_prec);
    for (int p = 0; p < nprob; ++p) {
        key.push_back(lgs[p]);
        int64_t hb;
        std::memcpy(&hb, &hs[p], sizeof hb);
        key.push_back(hb);
    }
    Plan *B = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            B = it->second;
        } else {
            B = new Plan;
            B->dev = dev;
            np_status st = build_plan(lgs, hs, o.smooth_prec, B);
            if (st != NP_OK) {
                free_plan(B);
                return st;
            }
            g_plans[key] = B;
        }
    }
    std::lock_guard<std::mutex> lk(B->mu);
    hipStream_t s = (hipStream_t)o.stream;
    NP_HIP_TRY(hipMemcpyAsync(B->d_f, rhs, sizeof(double *) * nprob, hipMemcpyHostToDevice, s));
    NP_HIP_TRY(hipMemcpyAsync(B->d_x, x, sizeof(double *) * nprob, hipMemcpyHostToDevice, s));
    auto run = [&](int inner_, const BOpts &bo_) -> np_status {
        return o.smooth_prec == NP_FP32 ? batched_run<float>(B, inner_, bo_, o, tol, s)
                                        : batched_run<double>(B, inner_, bo_, o, tol, s);
    };
    BOpts bo{o.nu1, o.nu2, o.omega, g_batched_rm, g_batched_wg};
    int inner = o.inner_cycles, source = 0;
    g_last_tune_inner = 0;
    g_last_tune_ms = 0.0;
    if (inner == 0) {
        // the autotuner's settings for this batch: from this process's cache,
        // else the file cache, else timed full solves of this batch
        const std::string key = tune_key(dev, o.smooth_prec, o.omega, lgs);
        const std::string path = tune_cache_path();
        BTuned t;
        {
            std::lock_guard<std::mutex> lk2(g_plan_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                t = it->second;
                source = 2;
            } else {
                auto file = read_tune_file(path);
                auto jt = file.find(key);
                if (jt != file.end()) {
                    t = jt->second;
                    g_tuned[key] = t;
                    source = 3;
                }
            }
        }
        if (source == 0 && g_batched_autotune && o.fixed_cycles == 0) {
            const auto t0 = std::chrono::steady_clock::now();
            B->omega_tune = o.omega;
            NP_TRY(autotune(B, nprob, s, run, o.smooth_prec == NP_FP32 ? 3 : 1, &t));
            g_last_tune_inner = t.inner;
            g_last_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            {
                std::lock_guard<std::mutex> lk2(g_plan_mu);
                g_tuned[key] = t;
                write_tune_file(path, key, t);
            }
            source = 1;
        }
        if (source != 0) {
            inner = t.inner;
            bo = BOpts{t.nu, t.nu, o.omega, t.rm, t.wg};
        } else {
            inner = o.smooth_prec == NP_FP32 ? 3 : 1;
        }
    }
    const int set[6] = {inner, bo.nu1, bo.nu2, bo.rm, bo.wg, source};
    std::memcpy(g_last_settings, set, sizeof set);
    NP_TRY(run(inner, bo));
    np_status st = NP_OK;
    for (int p = 0; p < nprob; ++p) {
        const BState &b = B->h_st[p];
        if (stats) {
            np_mg_stats &q = stats[p];
            std::memset(&q, 0, sizeof q);
            q.outer_iters = b.k;
            q.cycles = b.k * inner;
            const int n = std::min(b.k + 1, kHist);
            for (int i = 0; i < n; ++i) q.hist[i] = b.hist[i];
            q.rel_res = b.hist[std::min(b.k, kHist - 1)];
            q.rho_est = (b.k > 0 && q.hist[0] > 0.0 && q.rel_res > 0.0) ? std::pow(q.rel_res / q.hist[0], 1.0 / b.k) : 0.0;
        }
        if (b.stop == kNonFinite) st = NP_ENAN;
        else if ((b.stop == kMaxCycles || b.stop == kDiverged) && st == NP_OK) st = NP_ENOCONV;
    }
    if (st == NP_ENAN) set_error("non-finite residual in a batched problem");
    else if (st == NP_ENOCONV) set_error("a batched problem did not reach the tolerance");
    return st;
}

extern "C" np_status np_last_batched_settings(int *inner_cycles, int *nu1, int *nu2, int *row_marching,
                                              int *workgroups, int *source) {
    int *dst[6] = {inner_cycles, nu1, nu2, row_marching, workgroups, source};
    for (int i = 0; i < 6; ++i)
        if (dst[i]) *dst[i] = g_last_settings[i];
    return NP_OK;
}

extern "C" np_status np_last_autotune(int *inner_cycles, double *ms) {
    if (inner_cycles) *inner_cycles = g_last_tune_inner;
    if (ms) *ms = g_last_tune_ms;
    return NP_OK;
}
