// Projection time step (Section 2.4) and the scalar advection-diffusion
// predictor-corrector (Section 2.1) on the GPU.
//
// Staggered periodic grid: p at cell centres, q_c[idx] on the face idx + e_c/2.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "np_internal.h"

namespace np {

np_status poisson_solve(np_dims dims, double h, np_bc bc, const double *rhs, double *x, double tol,
                        const np_mg_opts *opts, np_mg_stats *stats);

namespace {

// Periodic neighbour offset along axis a (0 = x, 1 = y, 2 = z) for a grid of
// n = 2^lg cells per axis: returns the linear index of (idx + s e_a).
__device__ __forceinline__ int64_t wrap_off(int64_t c, int coord, int s, int a, int lg) {
    const int n = 1 << lg;
    const int64_t st = int64_t(1) << (a * lg);
    int q = coord + s;
    if (q < 0) return c + int64_t(n - 1) * st;
    if (q >= n) return c - int64_t(n - 1) * st;
    return c + s * st;
}

struct Vel {
    const double *q[3];
};

// Momentum rate F_c of component c at face idx (coords co) for the field `in`
// (the component being advanced, possibly the half-step average of two
// arrays), advected by a (= u^n), with pressure gradient of p:
//   F_c = sum_e a_e^(c) (in[+e] - in[-e]) / (2h) - nu Lap(in) + (p[+e_c] - p) / h,
// a_e^(c) = a_c itself for e == c, else the mean of the four e-faces around
// the c-face: idx, idx + e_c, idx - e_e, idx + e_c - e_e.
template <int D, class IN>
__device__ __forceinline__ double mom_rate(const IN &in, const Vel &a, const double *__restrict__ p, int c,
                                           int64_t idx, const int co[3], int lg, double inv_2h,
                                           double nu_inv_h2, double inv_h) {
    const double qc = in(idx);
    double adv = 0.0, lap = -2.0 * D * qc;
    const int64_t pc = wrap_off(idx, co[c], 1, c, lg);  // idx + e_c
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const int64_t ip = wrap_off(idx, co[e], 1, e, lg), im = wrap_off(idx, co[e], -1, e, lg);
        const double qp = in(ip), qm = in(im);
        double ae;
        if (e == c) {
            ae = a.q[e][idx];
        } else {
            // idx + e_c - e_e: step -e_e from idx + e_c (coordinates of idx + e_c along e are co[e])
            const int64_t pcm = wrap_off(pc, co[e], -1, e, lg);
            ae = 0.25 * (a.q[e][idx] + a.q[e][pc] + a.q[e][im] + a.q[e][pcm]);
        }
        adv += ae * (qp - qm) * inv_2h;
        lap += qp + qm;
    }
    return adv - nu_inv_h2 * lap + (p[pc] - p[idx]) * inv_h;
}

struct LdArr {
    const double *p;
    __device__ __forceinline__ double operator()(int64_t q) const { return p[q]; }
};
struct LdHalf {
    const double *a, *b;
    __device__ __forceinline__ double operator()(int64_t q) const { return 0.5 * (a[q] + b[q]); }
};

// Predictor (STAGE 0): out_c = q^n_c - dt F_c(q^n).  Corrector (STAGE 1):
// out_c = q^n_c - dt F_c((qt_c + q^n_c)/2).  One thread per cell, all
// components.
template <int D, int STAGE>
__global__ __launch_bounds__(kBlock) void k_mom_stage(Vel qn, Vel qt, double *__restrict__ o0,
                                                      double *__restrict__ o1, double *__restrict__ o2,
                                                      const double *__restrict__ p, int lg, double dt,
                                                      double nu, double h) {
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m) return;
    const int n = 1 << lg;
    const int co[3] = {int(idx & (n - 1)), int((idx >> lg) & (n - 1)), D == 3 ? int(idx >> (2 * lg)) : 0};
    const double inv_2h = 0.5 / h, nu_inv_h2 = nu / (h * h), inv_h = 1.0 / h;
    double *out[3] = {o0, o1, o2};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double F;
        if (STAGE == 0) F = mom_rate<D>(LdArr{qn.q[c]}, qn, p, c, idx, co, lg, inv_2h, nu_inv_h2, inv_h);
        else F = mom_rate<D>(LdHalf{qt.q[c], qn.q[c]}, qn, p, c, idx, co, lg, inv_2h, nu_inv_h2, inv_h);
        out[c][idx] = qn.q[c][idx] - dt * F;
    }
}

// rhs = -(1/dt) D q: D q at a cell = sum_c (q_c[idx] - q_c[idx - e_c]) / h.
template <int D>
__global__ __launch_bounds__(kBlock) void k_div_rhs(Vel q, double *__restrict__ rhs, int lg, double scale) {
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m) return;
    const int n = 1 << lg;
    const int co[3] = {int(idx & (n - 1)), int((idx >> lg) & (n - 1)), D == 3 ? int(idx >> (2 * lg)) : 0};
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) s += q.q[c][idx] - q.q[c][wrap_off(idx, co[c], -1, c, lg)];
    rhs[idx] = s * scale;
}

// q_c = qs_c - dt (dp[idx + e_c] - dp[idx]) / h; p += dp.
template <int D>
__global__ __launch_bounds__(kBlock) void k_correct(Vel qs, double *__restrict__ o0, double *__restrict__ o1,
                                                    double *__restrict__ o2, double *__restrict__ p,
                                                    const double *__restrict__ dp, int lg, double dt_over_h) {
    const int64_t m = int64_t(1) << (D * lg);
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m) return;
    const int n = 1 << lg;
    const int co[3] = {int(idx & (n - 1)), int((idx >> lg) & (n - 1)), D == 3 ? int(idx >> (2 * lg)) : 0};
    double *out[3] = {o0, o1, o2};
    const double dc = dp[idx];
#pragma unroll
    for (int c = 0; c < D; ++c) out[c][idx] = qs.q[c][idx] - dt_over_h * (dp[wrap_off(idx, co[c], 1, c, lg)] - dc);
    p[idx] += dc;
}

// ---------------------------------------------------------- scalar AD step
// Any n >= 3 (not necessarily a power of two).  Ghost rule as the solver's.
struct Gen {
    int64_t n;
    int bc;
    __device__ __forceinline__ int64_t at(int i, int j, int k, int D) const {
        return (D == 3 ? (int64_t(k) * n + j) * n : int64_t(j) * n) + i;
    }
};

template <int D, class IN>
__device__ __forceinline__ double ad_rate(const IN &T, const double *const *a, const Gen &g, int i, int j, int k,
                                          double inv_2h, double nu_inv_h2) {
    const int64_t c = g.at(i, j, k, D);
    const double tc = T(c);
    const int co[3] = {i, j, k};
    double lap = -2.0 * D * tc, adv = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        int pp[3] = {i, j, k}, mm[3] = {i, j, k};
        pp[e] += 1;
        mm[e] -= 1;
        double tp, tm;
        if (pp[e] < g.n) tp = T(g.at(pp[0], pp[1], pp[2], D));
        else if (g.bc) { pp[e] = 0; tp = T(g.at(pp[0], pp[1], pp[2], D)); }
        else tp = -tc;
        if (mm[e] >= 0) tm = T(g.at(mm[0], mm[1], mm[2], D));
        else if (g.bc) { mm[e] = int(g.n - 1); tm = T(g.at(mm[0], mm[1], mm[2], D)); }
        else tm = -tc;
        (void)co;
        lap += tp + tm;
        if (a) adv += a[e][c] * (tp - tm) * inv_2h;
    }
    return adv - nu_inv_h2 * lap;
}

struct APtrs {
    const double *a[3];
    int has;
};

template <int D, int STAGE>
__global__ __launch_bounds__(kBlock) void k_ad_stage(const double *__restrict__ T, const double *__restrict__ Tt,
                                                     double *__restrict__ out, APtrs ap, Gen g, double dt,
                                                     double inv_2h, double nu_inv_h2) {
    const int64_t m = D == 3 ? g.n * g.n * g.n : g.n * g.n;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int i = int(c % g.n), j = int((c / g.n) % g.n), k = D == 3 ? int(c / (g.n * g.n)) : 0;
    const double *const *a = ap.has ? ap.a : nullptr;
    double R;
    if (STAGE == 0) R = ad_rate<D>(LdArr{T}, a, g, i, j, k, inv_2h, nu_inv_h2);
    else R = ad_rate<D>(LdHalf{Tt, T}, a, g, i, j, k, inv_2h, nu_inv_h2);
    out[c] = T[c] - dt * R;
}

// ------------------------------------- explicit step, filter families
// The filters of Section 2.1 and Appendix A on any n >= 3 (all axes equal):
// scheme 0 central (3-point first differences, 5-/7-point diffusion), 1
// first-order upwind advection (the upstream value: backward difference for a
// positive velocity component) with the same diffusion, 2 the finite-element
// (bilinear / trilinear) filters: first derivatives averaged across the other
// axes with weights (1, 4, 1)/6, diffusion 16 delta - (1,2,1)x(1,2,1) over
// 4 h^2 (2D) or 88 / -6 / -3 / -2 on the centre, faces, edges and corners over
// 26 h^2 (3D).  Boundary rule bc: 0 Dirichlet-0 (ghost = -value), 1 periodic,
// 2 zero normal derivative (ghost = value, the copy padding of Section 2.4).

// Index along one axis of the cell q (at most one cell outside [0, n)) and the
// sign its value takes.
__device__ __forceinline__ int adx_res(int q, int n, int bc, double &sg) {
    sg = 1.0;
    if (q < 0) {
        if (bc == 1) return n - 1;
        if (bc == 0) sg = -1.0;
        return 0;
    }
    if (q >= n) {
        if (bc == 1) return 0;
        if (bc == 0) sg = -1.0;
        return n - 1;
    }
    return q;
}

constexpr int kAdxX = 64, kAdxY = 4;  // workgroup: 64 cells along x, 4 rows

// The 3^d neighbourhood v[dz + 1][dy + 1][dx + 1] of cell (i, j, k) of F
// (HALF: of (F + G)/2) with the boundary rule; the 5/7-point families load
// the face neighbours only (the other entries stay zero).
template <int D, int SCHEME, bool HALF>
__device__ __forceinline__ void adx_gather(const double *__restrict__ F, const double *__restrict__ G, int i, int j,
                                           int k, int n, int bc, double (&v)[3][3][3]) {
    const int64_t nn = n;
    int ix[3];
    double sx[3];
    for (int o = 0; o < 3; ++o) ix[o] = adx_res(i + o - 1, n, bc, sx[o]);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        if (D == 2 && dz != 0) continue;
        double sz = 1.0;
        const int kk = D == 3 ? adx_res(k + dz, n, bc, sz) : 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            double sy;
            const int jj = adx_res(j + dy, n, bc, sy);
            const int64_t row = (int64_t(kk) * nn + jj) * nn;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (SCHEME != 2 && (dx != 0) + (dy != 0) + (dz != 0) > 1) continue;  // 5/7-point only
                const int64_t q = row + ix[dx + 1];
                const double t = HALF ? 0.5 * (G[q] + F[q]) : F[q];
                v[dz + 1][dy + 1][dx + 1] = sx[dx + 1] * sy * sz * t;
            }
        }
    }
}

// First derivative along axis e of the gathered field: the finite-element
// filter (scheme 2) or the central difference.
template <int D, int SCHEME>
__device__ __forceinline__ double adx_deriv(const double (&v)[3][3][3], int e, double h) {
    if (SCHEME == 2) {
        const double w[3] = {1.0, 4.0, 1.0};
        double g = 0.0;
        if (D == 2) {
#pragma unroll
            for (int p = 0; p < 3; ++p) g += w[p] * (e == 0 ? v[1][p][2] - v[1][p][0] : v[1][2][p] - v[1][0][p]);
            return g / (12.0 * h);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                g += w[p] * w[q] *
                     (e == 0 ? v[p][q][2] - v[p][q][0] : (e == 1 ? v[p][2][q] - v[p][0][q] : v[2][p][q] - v[0][p][q]));
        return g / (72.0 * h);
    }
    const double xm = e == 0 ? v[1][1][0] : (e == 1 ? v[1][0][1] : v[0][1][1]);
    const double xp = e == 0 ? v[1][1][2] : (e == 1 ? v[1][2][1] : v[2][1][1]);
    return (xp - xm) / (2.0 * h);
}

// Advection + diffusion rate of the gathered field, a the velocity at the
// cell (used when has_a).
template <int D, int SCHEME>
__device__ __forceinline__ double adx_rate_at(const double (&v)[3][3][3], const double (&a)[3], bool has_a, double nu,
                                              double h) {
    const double v0 = v[1][1][1];
    double adv = 0.0, dif;
    if (SCHEME == 2) {
        if (D == 2) {
            const double b[3] = {1.0, 2.0, 1.0};
            double sm = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) sm += b[p] * b[q] * v[1][p][q];
            dif = (16.0 * v0 - sm) / (4.0 * h * h);
        } else {
            const double cw[4] = {88.0, -6.0, -3.0, -2.0};  // by the number of nonzero offsets
            double sm = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int r = 0; r < 3; ++r) sm += cw[(p != 1) + (q != 1) + (r != 1)] * v[p][q][r];
            dif = sm / (26.0 * h * h);
        }
        if (has_a)
#pragma unroll
            for (int e = 0; e < D; ++e) adv += a[e] * adx_deriv<D, 2>(v, e, h);
    } else {
        const double xm[3] = {v[1][1][0], v[1][0][1], v[0][1][1]}, xp[3] = {v[1][1][2], v[1][2][1], v[2][1][1]};
        double lap = 0.0;
#pragma unroll
        for (int e = 0; e < D; ++e) {
            lap += (v0 - xm[e]) + (v0 - xp[e]);
            if (!has_a) continue;
            if (SCHEME == 0) adv += a[e] * (xp[e] - xm[e]) / (2.0 * h);
            else adv += a[e] >= 0.0 ? a[e] * (v0 - xm[e]) / h : a[e] * (xp[e] - v0) / h;
        }
        dif = lap / (h * h);
    }
    return adv + nu * dif;
}

// STAGE 0: out = T - dt R(T), and tcopy = T (so that the corrector can write
// the caller's array); STAGE 1: out = T - dt R((Tt + T)/2).  One thread per
// cell; the 3^d neighbourhood is gathered with the boundary rule, then every
// filter of the family reads it.
template <int D, int SCHEME, int STAGE>
__global__ __launch_bounds__(kAdxX * kAdxY) void k_adx_stage(const double *__restrict__ T,
                                                             const double *__restrict__ Tt,
                                                             double *__restrict__ out, double *__restrict__ tcopy,
                                                             APtrs ap, int n, int bc, double dt, double nu,
                                                             double h) {
    const int i = int(blockIdx.x) * kAdxX + int(threadIdx.x), j = int(blockIdx.y) * kAdxY + int(threadIdx.y);
    const int k = D == 3 ? int(blockIdx.z) : 0;
    if (i >= n || j >= n) return;
    double v[3][3][3] = {};
    adx_gather<D, SCHEME, STAGE == 1>(T, Tt, i, j, k, n, bc, v);
    const int64_t c = (int64_t(k) * n + j) * n + i;
    double a[3] = {0.0, 0.0, 0.0};
    if (ap.has)
#pragma unroll
        for (int e = 0; e < D; ++e) a[e] = ap.a[e][c];
    out[c] = T[c] - dt * adx_rate_at<D, SCHEME>(v, a, ap.has != 0, nu, h);
    if (STAGE == 0) tcopy[c] = T[c];
}

// 2D grids with n >= 1024, n a multiple of kAx2: row-marching tiles.  A
// workgroup of kAx2 threads owns kAx2 consecutive columns and ry rows; each
// step publishes the next row of the stage input (ghost rule and signs
// applied, the strip's edge threads adding the cells beyond it) into a ring
// of four LDS rows, so one barrier per row suffices, and every thread reads
// its 3 x 3 (or 5-point) neighbourhood from rows j - 1, j, j + 1.  The values
// and the rate are those of k_adx_stage, so the results are bit-identical.
constexpr int kAx2 = 256;

inline int adx_rows2(int n) {
    int ry = 32;
    while (int64_t(n / kAx2) * (n / ry) < 2048 && ry > 4) ry /= 2;
    return ry;
}

template <int SCHEME, int STAGE>
__global__ __launch_bounds__(kAx2) void k_adx_stage2r(const double *__restrict__ T, const double *__restrict__ Tt,
                                                      double *__restrict__ out, double *__restrict__ tcopy,
                                                      APtrs ap, int n, int bc, int ry, double dt, double nu,
                                                      double h) {
    __shared__ double rows[4][kAx2 + 2];
    const int strips = n / kAx2, tid = int(threadIdx.x);
    const int x0 = (int(blockIdx.x) % strips) * kAx2, j0 = (int(blockIdx.x) / strips) * ry;
    const int i = x0 + tid;
    // the edge threads also publish the column beyond the strip (ghost rule)
    const bool hl = tid == 0, hr = tid == kAx2 - 1;
    double hsx = 1.0;
    const int hi = (hl || hr) ? adx_res(hl ? x0 - 1 : x0 + kAx2, n, bc, hsx) : 0;
    const int64_t nn = n;
    auto tv = [&](int64_t q) { return STAGE == 1 ? 0.5 * (Tt[q] + T[q]) : T[q]; };
    // row jr of the stage input (jr may be -1 or n): own column and edge value;
    // raw: T at the own column of that row (the corrector's T^n, kept for later)
    auto fetch = [&](int jr, double &own, double &edge, double &raw) {
        double sy;
        const int jj = adx_res(jr < n ? jr : n, n, bc, sy);
        const int64_t q = int64_t(jj) * nn + i;
        raw = T[q];
        own = (1.0 * sy * 1.0) * (STAGE == 1 ? 0.5 * (Tt[q] + raw) : raw);
        edge = (hl || hr) ? (hsx * sy * 1.0) * tv(int64_t(jj) * nn + hi) : 0.0;
    };
    auto publish = [&](int jr, double own, double edge) {
        double *r = rows[jr & 3];
        r[tid + 1] = own;
        if (hl) r[0] = edge;
        if (hr) r[kAx2 + 1] = edge;
    };
    double o, e, r;
    fetch(j0 - 1, o, e, r);
    publish(j0 - 1, o, e);
    fetch(j0, o, e, r);
    publish(j0, o, e);
    double rc = r;  // T at the own column of row j
    double no, ne, nr;
    fetch(j0 + 1, no, ne, nr);
    for (int j = j0; j < j0 + ry; ++j) {
        publish(j + 1, no, ne);
        const int64_t c = int64_t(j) * nn + i;
        double a[3] = {0.0, 0.0, 0.0};
        if (ap.has)
#pragma unroll
            for (int q = 0; q < 2; ++q) a[q] = ap.a[q][c];
        const double tc = rc;
        rc = nr;
        __syncthreads();
        if (j + 1 < j0 + ry) fetch(j + 2, no, ne, nr);
        double v[3][3][3] = {};
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (SCHEME != 2 && (dx != 0) + (dy != 0) > 1) continue;  // 5-point families
                v[1][dy + 1][dx + 1] = rows[(j + dy) & 3][tid + 1 + dx];
            }
        // the stage input of the predictor is T itself: its own value is in the ring
        const double t0 = STAGE == 1 ? tc : v[1][1][1];
        out[c] = t0 - dt * adx_rate_at<2, SCHEME>(v, a, ap.has != 0, nu, h);
        if (STAGE == 0) tcopy[c] = t0;
    }
}

// 3D levels on z-marching tiles: a workgroup of kZx x TY threads owns a
// kZx x TY column tile and zc planes; planes z - 1, z, z + 1 of the stage
// input (with its halo ring, ghost rule applied) sit in a ring of three LDS
// buffers, and each thread loads its share of plane z + 2 into registers
// before computing plane z.  Every filter family reads its 3^3 (or 7-point)
// neighbourhood from LDS; the velocity is read per cell.  Any n >= 3.
constexpr int kZx = 64;
}  // namespace
int g_zmarch_explicit = 1;  // tuning knob "zmarch_explicit"
int g_mom_rows = 4;         // tuning knob "mom_rows": tile rows of the staggered corrector stage (4 or 8)
int g_mom_ring = 2;         // tuning knob "mom_ring": planes per field in the staggered stages' LDS rings (2 or 3)
namespace {
// Tile rows per workgroup: 4 for the 27-point finite-element stages (their
// register footprint leaves room for more, smaller workgroups per CU: measured
// faster), 8 otherwise.
constexpr int zrows(int scheme) { return scheme == 2 ? 4 : 8; }

// Plane ring of NF fields on a z-marching tile of kZx x TY columns: each
// thread owns PER slots of the (kZx + 2) x (TY + 2) plane (the tile and its
// halo ring, ghost rule along x and y applied through the slot's source offset
// and sign).
template <int NF, int TY>
struct ZRing {
    static constexpr int T = kZx * TY;                          // threads
    static constexpr int SLOTS = (kZx + 2) * (TY + 2);
    static constexpr int PER = (SLOTS + T - 1) / T;             // plane values loaded per thread
    typedef double Plane[3][TY + 2][kZx + 2];
    int tx, ty, x0, y0, z0, z1, n, bc;
    int64_t P;
    int64_t off[PER];
    double sg[PER];
    int ly[PER], lx[PER];
    bool own[PER];
    double nx[NF][PER];  // plane z + 1 (then z + 2) in flight
    __device__ ZRing(int n_, int bc_, int zc) : n(n_), bc(bc_) {
        tx = int(threadIdx.x) % kZx;
        ty = int(threadIdx.x) / kZx;
        const int ntx = (n + kZx - 1) / kZx, nty = (n + TY - 1) / TY;
        // XCD-contiguous tiles, so that a tile's halo rows and planes (its neighbours' own cells)
        // are read through the same L2: the three-plane momentum stages read 1.07x / 1.10x their
        // algorithmic bytes so, 1.94x / 1.62x in launch order
        const int blk = int(xcd_block(blockIdx.x, gridDim.x));
        x0 = (blk % ntx) * kZx;
        y0 = ((blk / ntx) % nty) * TY;
        z0 = (blk / (ntx * nty)) * zc;
        z1 = min(z0 + zc, n);
        P = int64_t(n) * n;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int sidx = int(threadIdx.x) + r * T;
            own[r] = sidx < SLOTS;
            const int t = own[r] ? sidx : 0;
            ly[r] = t / (kZx + 2);
            lx[r] = t % (kZx + 2);
            double s1, s2;
            const int gi = adx_res(min(x0 + lx[r] - 1, n), n, bc, s1);
            const int gj = adx_res(min(y0 + ly[r] - 1, n), n, bc, s2);
            off[r] = int64_t(gj) * n + gi;
            sg[r] = s1 * s2;
        }
    }
    // load plane z of every field into nx; ld(f, q) is field f at index q
    template <class LD>
    __device__ __forceinline__ void load(const LD &ld, int z) {
        double sz;
        const int64_t kk = adx_res(z, n, bc, sz);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < PER; ++r) nx[f][r] = sz * sg[r] * ld(f, kk * P + off[r]);
    }
    __device__ __forceinline__ void store(Plane *pl, int z) {
        const int slot = (z + 3) % 3;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < PER; ++r)
                if (own[r]) pl[f][slot][ly[r]][lx[r]] = nx[f][r];
    }
    // planes z0 - 1, z0 into LDS, plane z0 + 1 in flight
    template <class LD>
    __device__ __forceinline__ void start(const LD &ld, Plane *pl) {
        load(ld, z0 - 1);
        store(pl, z0 - 1);
        load(ld, z0);
        store(pl, z0);
        load(ld, z0 + 1);
    }
    // The marching loop: plane z + 1 is stored, then plane z + 2 is issued
    // before body(z) computes plane z; two barriers per plane (the store is
    // visible; every read of the oldest buffer is done before it is overwritten).
    template <class LD, class BODY>
    __device__ __forceinline__ void march(const LD &ld, Plane *pl, const BODY &body) {
        start(ld, pl);
        for (int z = z0; z < z1; ++z) {
            store(pl, z + 1);
            __syncthreads();
            if (z + 2 <= z1) load(ld, z + 2);
            body(z);
            __syncthreads();
        }
    }
    // the thread's 3^3 (SCHEME != 2: 7-point) neighbourhood of field f at plane z
    template <int SCHEME>
    __device__ __forceinline__ void gather(const Plane &pf, int z, double (&v)[3][3][3]) const {
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const int sl = (z + dz + 3) % 3;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (SCHEME != 2 && (dx != 0) + (dy != 0) + (dz != 0) > 1) continue;
                    v[dz + 1][dy + 1][dx + 1] = pf[sl][ty + 1 + dy][tx + 1 + dx];
                }
        }
    }
};

template <int SCHEME, int STAGE>
__global__ __launch_bounds__(kZx * zrows(SCHEME)) void k_adx_stage3z(const double *__restrict__ T,
                                                                     const double *__restrict__ Tt,
                                                                     double *__restrict__ out,
                                                                     double *__restrict__ tcopy, APtrs ap, int n,
                                                                     int bc, int zc, double dt, double nu, double h) {
    typedef ZRing<1, zrows(SCHEME)> Ring;
    __shared__ typename Ring::Plane pl[1];
    Ring R(n, bc, zc);
    auto ld = [&](int, int64_t q) { return STAGE == 0 ? T[q] : 0.5 * (Tt[q] + T[q]); };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    R.march(ld, pl, [&](int z) {
        if (i < n && j < n) {
            double v[3][3][3] = {};
            R.template gather<SCHEME>(pl[0], z, v);
            const int64_t c = int64_t(z) * R.P + int64_t(j) * n + i;
            double a[3] = {0.0, 0.0, 0.0};
            if (ap.has)
#pragma unroll
                for (int e = 0; e < 3; ++e) a[e] = ap.a[e][c];
            const double tc = T[c];
            out[c] = tc - dt * adx_rate_at<3, SCHEME>(v, a, ap.has != 0, nu, h);
            if (STAGE == 0) tcopy[c] = tc;
        }
    });
}

// Collocated momentum stage (as k_nsc_stage) on z-marching tiles: the three
// components' stage input and the pressure in LDS rings.
template <int SCHEME, int STAGE>
__global__ __launch_bounds__(kZx * zrows(SCHEME)) void k_nsc_stage3z(Vel qn, Vel qt, double *__restrict__ o0,
                                                                     double *__restrict__ o1, double *__restrict__ o2,
                                                                     const double *__restrict__ p, int n, int zc,
                                                                     double dt, double nu, double h) {
    typedef ZRing<4, zrows(SCHEME)> Ring;
    __shared__ typename Ring::Plane pl[4];
    Ring R(n, 1, zc);
    auto ld = [&](int f, int64_t q) {
        if (f == 3) return p[q];
        return STAGE == 0 ? qn.q[f][q] : 0.5 * (qt.q[f][q] + qn.q[f][q]);
    };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    double *out[3] = {o0, o1, o2};
    R.march(ld, pl, [&](int z) {
        if (i < n && j < n) {
            const int64_t c = int64_t(z) * R.P + int64_t(j) * n + i;
            // the velocity at the node: in the predictor it is the ring's own value
            double a[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) a[e] = STAGE == 0 ? pl[e][(z + 3) % 3][R.ty + 1][R.tx + 1] : qn.q[e][c];
            // the pressure gradient first, so that one 3^3 neighbourhood is live at a time
            double gp[3];
            {
                double vp[3][3][3] = {};
                R.template gather<SCHEME>(pl[3], z, vp);
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) gp[comp] = adx_deriv<3, SCHEME>(vp, comp, h);
            }
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                double v[3][3][3] = {};
                R.template gather<SCHEME>(pl[comp], z, v);
                const double Rr = adx_rate_at<3, SCHEME>(v, a, true, nu, h) + gp[comp];
                out[comp][c] = a[comp] - dt * Rr;
            }
        }
    });
}

// rhs = scale * sum_e D_e q_e on z-marching tiles.
template <int SCHEME>
__global__ __launch_bounds__(kZx * 8) void k_nsc_div3z(Vel q, double *__restrict__ rhs, int n, int zc, double h,
                                                       double scale) {
    __shared__ ZRing<3, 8>::Plane pl[3];
    ZRing<3, 8> R(n, 1, zc);
    auto ld = [&](int f, int64_t x) { return q.q[f][x]; };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    R.march(ld, pl, [&](int z) {
        if (i < n && j < n) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                double v[3][3][3] = {};
                R.template gather<SCHEME>(pl[e], z, v);
                s += adx_deriv<3, SCHEME>(v, e, h);
            }
            rhs[int64_t(z) * R.P + int64_t(j) * n + i] = s * scale;
        }
    });
}

// q_c = qs_c - dt D_c dp; p += dp, on z-marching tiles.
template <int SCHEME>
__global__ __launch_bounds__(kZx * 8) void k_nsc_correct3z(Vel qs, double *__restrict__ o0, double *__restrict__ o1,
                                                           double *__restrict__ o2, double *__restrict__ p,
                                                           const double *__restrict__ dp, int n, int zc, double dt,
                                                           double h) {
    __shared__ ZRing<1, 8>::Plane pl[1];
    ZRing<1, 8> R(n, 1, zc);
    auto ld = [&](int, int64_t x) { return dp[x]; };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    double *out[3] = {o0, o1, o2};
    R.march(ld, pl, [&](int z) {
        if (i < n && j < n) {
            const int64_t c = int64_t(z) * R.P + int64_t(j) * n + i;
            double v[3][3][3] = {};
            R.template gather<SCHEME>(pl[0], z, v);
#pragma unroll
            for (int e = 0; e < 3; ++e) out[e][c] = qs.q[e][c] - dt * adx_deriv<3, SCHEME>(v, e, h);
            p[c] += v[1][1][1];
        }
    });
}

// MAC momentum stage (as k_mom_stage, the same terms in the same order) on
// z-marching tiles of kZx x TY columns: the advecting velocity q^n (three
// components), the advanced field (the predictor's q^n itself; the
// corrector's half-step average (q~ + q^n) / 2, fields 3..5) and p sit in
// LDS rings of three planes with their halo ring, so every face average of the
// advecting velocity (idx, idx + e_c, idx - e_e, idx + e_c - e_e) and every
// neighbour of the advanced field is an LDS read.  Periodic.
template <int STAGE, int TY>
__global__ __launch_bounds__(kZx * TY) void k_mom_stage3z(Vel qn, Vel qt, double *__restrict__ o0,
                                                          double *__restrict__ o1, double *__restrict__ o2,
                                                          const double *__restrict__ p, int n, int zc, double dt,
                                                          double nu, double h) {
    constexpr int NF = STAGE == 0 ? 4 : 7, FP = NF - 1;
    typedef ZRing<NF, TY> Ring;
    __shared__ typename Ring::Plane pl[NF];
    Ring R(n, 1, zc);
    auto ld = [&](int f, int64_t q) -> double {
        if (f < 3) return qn.q[f][q];
        if (STAGE == 1 && f < 6) return 0.5 * (qt.q[f - 3][q] + qn.q[f - 3][q]);
        return p[q];
    };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    const double inv_2h = 0.5 / h, nu_inv_h2 = nu / (h * h), inv_h = 1.0 / h;
    double *out[3] = {o0, o1, o2};
    R.march(ld, pl, [&](int z) {
        if (i < n && j < n) {
            const int sl[3] = {(z + 2) % 3, z % 3, (z + 1) % 3};  // planes z - 1, z, z + 1
            auto at = [&](int f, int dx, int dy, int dz) -> double {
                return pl[f][sl[dz + 1]][R.ty + 1 + dy][R.tx + 1 + dx];
            };
            const int64_t c = int64_t(z) * R.P + int64_t(j) * n + i;
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                const int fin = STAGE == 0 ? comp : 3 + comp;
                const int cx = comp == 0, cy = comp == 1, cz = comp == 2;  // e_c
                const double qc = at(fin, 0, 0, 0);
                double adv = 0.0, lap = -2.0 * 3 * qc;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int ex = e == 0, ey = e == 1, ez = e == 2;
                    const double qp = at(fin, ex, ey, ez), qm = at(fin, -ex, -ey, -ez);
                    double ae;
                    if (e == comp) {
                        ae = at(e, 0, 0, 0);
                    } else {
                        ae = 0.25 * (at(e, 0, 0, 0) + at(e, cx, cy, cz) + at(e, -ex, -ey, -ez) +
                                     at(e, cx - ex, cy - ey, cz - ez));
                    }
                    adv += ae * (qp - qm) * inv_2h;
                    lap += qp + qm;
                }
                const double F = adv - nu_inv_h2 * lap + (at(FP, cx, cy, cz) - at(FP, 0, 0, 0)) * inv_h;
                out[comp][c] = at(comp, 0, 0, 0) - dt * F;
            }
        }
    });
}

// LDS rings of two planes per field for the MAC momentum stage (periodic), on
// tiles of X x TY columns.  While plane z is computed, field f holds planes
// z + mom_lo(f) and z + mom_lo(f) + 1 (slot = plane & 1): mom_lo = 0 for the
// fields read off the own column only up to z + 1 (the x and y velocity, the
// advanced field, p), mom_lo = -1 for the z velocity (its face averages reach
// z - 1 off the own column).  The one z-neighbour outside that pair is only ever
// read at the thread's own column, so it sits in a register: plane z - 1 (saved
// from LDS a step earlier) for mom_lo = 0, plane z + 1 (prefetched two steps
// ahead) for the z velocity.
// Slot order: the tile's TY + 2 rows of X interior columns first, one row per
// wave when X = 64 (so every wave-wide load covers whole aligned 128-byte lines),
// then the two halo columns of each row; slots past the end repeat the last one
// (the same value to the same place), so no lane is masked.
__host__ __device__ constexpr int mom_lo(int f) { return f == 2 ? -1 : 0; }

template <int NF, int X, int TY>
struct ZRing2 {
    static constexpr int T = X * TY;
    static constexpr int SLOTS = (X + 2) * (TY + 2);
    static constexpr int PER = (SLOTS + T - 1) / T;
    typedef double Plane[2][TY + 2][X + 2];
    typedef double Regs[NF][PER];  // one plane of every field, in flight
    int tx, ty, x0, y0, z0, z1, n;
    int64_t P;
    int64_t off[PER];
    int ly[PER], lx[PER];
    __device__ ZRing2(int n_, int zc) : n(n_) {
        tx = int(threadIdx.x) % X;
        ty = int(threadIdx.x) / X;
        const int ntx = (n + X - 1) / X, nty = (n + TY - 1) / TY;
        const int blk = int(xcd_block(blockIdx.x, gridDim.x));
        x0 = (blk % ntx) * X;
        y0 = ((blk / ntx) % nty) * TY;
        z0 = (blk / (ntx * nty)) * zc;
        z1 = min(z0 + zc, n);
        P = int64_t(n) * n;
        constexpr int NI = X * (TY + 2);  // interior slots
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int t = min(int(threadIdx.x) + r * T, SLOTS - 1);
            ly[r] = t < NI ? t / X : (t - NI) >> 1;
            lx[r] = t < NI ? t % X + 1 : (((t - NI) & 1) ? X + 1 : 0);
            double s1, s2;
            const int gi = adx_res(min(x0 + lx[r] - 1, n), n, 1, s1);
            const int gj = adx_res(min(y0 + ly[r] - 1, n), n, 1, s2);
            off[r] = int64_t(gj) * n + gi;
        }
    }
    __device__ __forceinline__ int64_t plane(int z) const {
        double sz;
        return int64_t(adx_res(z, n, 1, sz)) * P;
    }
    template <class LD>
    __device__ __forceinline__ void load(const LD &ld, Regs &v, int f, int z) const {
        const int64_t kk = plane(z);
#pragma unroll
        for (int r = 0; r < PER; ++r) v[f][r] = ld(f, kk + off[r]);
    }
    __device__ __forceinline__ void store(Plane &pf, const Regs &v, int f, int z) const {
#pragma unroll
        for (int r = 0; r < PER; ++r) pf[z & 1][ly[r]][lx[r]] = v[f][r];
    }
};

// MAC momentum stage on z-marching tiles with two-plane LDS rings (ZRing2): the
// same terms in the same order as k_mom_stage (and k_mom_stage3z), so the step
// is bit-identical.  Fields: 0..2 q^n (the advecting velocity; the predictor's
// advanced field too), the corrector's half-step average (q~ + q^n) / 2
// (3..5), p (last).  The predictor stores that average, formed exactly as the
// per-cell corrector forms it, instead of q~ (which nothing else reads): the
// corrector then reads seven fields, not nine.  Periodic.
template <int STAGE, int X, int TY>
__global__ __launch_bounds__(X * TY) __attribute__((amdgpu_waves_per_eu(STAGE == 0 ? 4 : 1))) void k_mom_stage3r(
    Vel qn, Vel qa, double *__restrict__ o0, double *__restrict__ o1, double *__restrict__ o2,
    const double *__restrict__ p, int n, int zc, double dt, double nu, double h) {
    constexpr int NF = STAGE == 0 ? 4 : 7, FP = NF - 1;
    typedef ZRing2<NF, X, TY> Ring;
    __shared__ typename Ring::Plane pl[NF];
    const Ring R(n, zc);
    const int zc0 = R.z0, zc1 = R.z1;
    auto ld = [&](int f, int64_t q) -> double {
        if (f < 3) return qn.q[f][q];
        if (STAGE == 1 && f < 6) return qa.q[f - 3][q];
        return p[q];
    };
    const int i = R.x0 + R.tx, j = R.y0 + R.ty;
    const bool act = i < n && j < n;
    const int64_t col = int64_t(min(j, n - 1)) * n + min(i, n - 1);
    const double inv_2h = 0.5 / h, nu_inv_h2 = nu / (h * h), inv_h = 1.0 / h;
    double *out[3] = {o0, o1, o2};
    // Two planes of every field in flight (parity-named register sets, so the
    // wait before a store leaves the other set's loads outstanding), and the own
    // column's out-of-ring z-neighbours in registers: plane z - 1 of the
    // mom_lo = 0 fields (prev), plane z + 1 of the z velocity (the predictor
    // reads it: its advanced field is q^n itself), prefetched two steps ahead.
    typename Ring::Regs sa, sb;
    double prev[NF], wa = 0.0, wb = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        R.load(ld, sa, f, zc0 + mom_lo(f));
        prev[f] = mom_lo(f) == 0 ? ld(f, R.plane(zc0 - 1) + col) : 0.0;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) R.store(pl[f], sa, f, zc0 + mom_lo(f));
    // issued in the order the loop issues them (set a, then set b), so that the
    // loop's waits leave the second set in flight
#pragma unroll
    for (int f = 0; f < NF; ++f) R.load(ld, sa, f, zc0 + 1 + mom_lo(f));
    if (STAGE == 0) wa = ld(2, R.plane(zc0 + 1) + col);
#pragma unroll
    for (int f = 0; f < NF; ++f) R.load(ld, sb, f, zc0 + 2 + mom_lo(f));
    if (STAGE == 0) wb = ld(2, R.plane(zc0 + 2) + col);
    // plane z: the set sv holds planes z + 1 + mom_lo, w the z velocity's own plane z + 1.
    // The loads two steps ahead are unconditional (no branch for the wait counts to
    // merge over): past the chunk's end they repeat plane z1 + mom_lo.
    // The z velocity's own plane z + 1 passes through LDS (the thread's own word), so
    // that its register is free before the next load into it: kept in a register
    // while that load is in flight, it costs a copy at the loop's back edge and
    // with it a wait for every load.
    __shared__ double wst[STAGE == 0 ? TY : 1][X];
    auto step = [&](int z, typename Ring::Regs &sv, double &w) {
#pragma unroll
        for (int f = 0; f < NF; ++f) R.store(pl[f], sv, f, z + 1 + mom_lo(f));
        if (STAGE == 0) wst[R.ty][R.tx] = w;
        __syncthreads();
        const double wz = STAGE == 0 ? wst[R.ty][R.tx] : 0.0;
        const int za = min(z + 3, zc1);
#pragma unroll
        for (int f = 0; f < NF; ++f) R.load(ld, sv, f, za + mom_lo(f));
        if (STAGE == 0) w = ld(2, R.plane(za) + col);
        if (act) {
            auto at = [&](int f, int dx, int dy, int dz) -> double {
                if (dz == -1 && mom_lo(f) == 0) return prev[f];  // own column only
                if (dz == 1 && mom_lo(f) == -1) return wz;       // own column only (the z velocity)
                return pl[f][(z + dz) & 1][R.ty + 1 + dy][R.tx + 1 + dx];
            };
            const int64_t c = int64_t(z) * R.P + int64_t(j) * n + i;
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                const int fin = STAGE == 0 ? comp : 3 + comp;
                const int cx = comp == 0, cy = comp == 1, cz = comp == 2;  // e_c
                const double qc = at(fin, 0, 0, 0);
                double adv = 0.0, lap = -2.0 * 3 * qc;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int ex = e == 0, ey = e == 1, ez = e == 2;
                    const double qp = at(fin, ex, ey, ez), qm = at(fin, -ex, -ey, -ez);
                    double ae;
                    if (e == comp) {
                        ae = at(e, 0, 0, 0);
                    } else {
                        ae = 0.25 * (at(e, 0, 0, 0) + at(e, cx, cy, cz) + at(e, -ex, -ey, -ez) +
                                     at(e, cx - ex, cy - ey, cz - ez));
                    }
                    adv += ae * (qp - qm) * inv_2h;
                    lap += qp + qm;
                }
                const double F = adv - nu_inv_h2 * lap + (at(FP, cx, cy, cz) - at(FP, 0, 0, 0)) * inv_h;
                const double qs = at(comp, 0, 0, 0) - dt * F;
                out[comp][c] = STAGE == 0 ? 0.5 * (qs + at(comp, 0, 0, 0)) : qs;
            }
        }
        // the own values of plane z are plane z - 1 of the next step
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (mom_lo(f) == 0) prev[f] = pl[f][z & 1][R.ty + 1][R.tx + 1];
        __syncthreads();
    };
    // chunks of an even number of planes; the first pair outside the loop, so that the
    // loop's waits never see the prologue's own-column loads (issued last) as pending
    step(zc0, sa, wa);
    step(zc0 + 1, sb, wb);
    for (int z = zc0 + 2; z < zc1; z += 2) {
        step(z, sa, wa);
        step(z + 1, sb, wb);
    }
}

// planes per workgroup of a two-plane-ring momentum launch: the most (up to 32)
// that still gives 1024 workgroups; even
inline int mom_planes(int n, int x, int ty) {
    const int64_t tiles = int64_t((n + x - 1) / x) * ((n + ty - 1) / ty);
    int zc = 32;
    while (zc > 2 && tiles * ((n + zc - 1) / zc) < 1024) zc >>= 1;
    return min(zc, n);
}

inline unsigned mom_grid(int n, int x, int ty, int zc) {
    return unsigned(((n + x - 1) / x) * ((n + ty - 1) / ty) * ((n + zc - 1) / zc));
}

inline int adx_planes(int n, int ty) {
    const int64_t tiles = int64_t((n + kZx - 1) / kZx) * ((n + ty - 1) / ty);
    int zc = 32;
    while (zc > 4 && tiles * ((n + zc - 1) / zc) < 2048) zc >>= 1;
    return zc;
}

// workgroups of a z-marching launch with ty-row tiles and zc planes each
inline unsigned zgrid(int n, int ty, int zc) {
    return unsigned(((n + kZx - 1) / kZx) * ((n + ty - 1) / ty) * ((n + zc - 1) / zc));
}

// ----------------------------------------- collocated projection step
// Velocity components and pressure at the same nodes (Section 2.4), periodic.
// Momentum STAGE 0: out_c = q^n_c - dt (R_c(q^n_c) + D_c p); STAGE 1:
// out_c = q^n_c - dt (R_c((qt_c + q^n_c)/2) + D_c p); R advects with the
// lagged velocity q^n at the cell.  All components per thread.
template <int D, int SCHEME, int STAGE>
__global__ __launch_bounds__(kAdxX * kAdxY) void k_nsc_stage(Vel qn, Vel qt, double *__restrict__ o0,
                                                             double *__restrict__ o1, double *__restrict__ o2,
                                                             const double *__restrict__ p, int n, double dt,
                                                             double nu, double h) {
    const int i = int(blockIdx.x) * kAdxX + int(threadIdx.x), j = int(blockIdx.y) * kAdxY + int(threadIdx.y);
    const int k = D == 3 ? int(blockIdx.z) : 0;
    if (i >= n || j >= n) return;
    const int64_t c = (int64_t(k) * n + j) * n + i;
    double a[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < D; ++e) a[e] = qn.q[e][c];
    double vp[3][3][3] = {};
    adx_gather<D, SCHEME, false>(p, nullptr, i, j, k, n, 1, vp);
    double *out[3] = {o0, o1, o2};
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
        double v[3][3][3] = {};
        adx_gather<D, SCHEME, STAGE == 1>(qn.q[comp], qt.q[comp], i, j, k, n, 1, v);
        const double R = adx_rate_at<D, SCHEME>(v, a, true, nu, h) + adx_deriv<D, SCHEME>(vp, comp, h);
        out[comp][c] = a[comp] - dt * R;
    }
}

// rhs = scale * sum_e D_e q_e (scale = -1/dt).
template <int D, int SCHEME>
__global__ __launch_bounds__(kAdxX * kAdxY) void k_nsc_div(Vel q, double *__restrict__ rhs, int n, double h,
                                                           double scale) {
    const int i = int(blockIdx.x) * kAdxX + int(threadIdx.x), j = int(blockIdx.y) * kAdxY + int(threadIdx.y);
    const int k = D == 3 ? int(blockIdx.z) : 0;
    if (i >= n || j >= n) return;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        double v[3][3][3] = {};
        adx_gather<D, SCHEME, false>(q.q[e], nullptr, i, j, k, n, 1, v);
        s += adx_deriv<D, SCHEME>(v, e, h);
    }
    rhs[(int64_t(k) * n + j) * n + i] = s * scale;
}

// q_c = qs_c - dt D_c dp; p += dp.
template <int D, int SCHEME>
__global__ __launch_bounds__(kAdxX * kAdxY) void k_nsc_correct(Vel qs, double *__restrict__ o0,
                                                               double *__restrict__ o1, double *__restrict__ o2,
                                                               double *__restrict__ p, const double *__restrict__ dp,
                                                               int n, double dt, double h) {
    const int i = int(blockIdx.x) * kAdxX + int(threadIdx.x), j = int(blockIdx.y) * kAdxY + int(threadIdx.y);
    const int k = D == 3 ? int(blockIdx.z) : 0;
    if (i >= n || j >= n) return;
    const int64_t c = (int64_t(k) * n + j) * n + i;
    double v[3][3][3] = {};
    adx_gather<D, SCHEME, false>(dp, nullptr, i, j, k, n, 1, v);
    double *out[3] = {o0, o1, o2};
#pragma unroll
    for (int e = 0; e < D; ++e) out[e][c] = qs.q[e][c] - dt * adx_deriv<D, SCHEME>(v, e, h);
    p[c] += v[1][1][1];
}

// ------------------------------------------------------------- workspace
struct NsWork {
    int d = 0, lg = 0;
    double *buf = nullptr;  // 2*d face arrays + rhs + dp
    bool dp_valid = false;  // dp holds the increment of a converged step on this grid
    std::mutex mu;
};
std::mutex g_ns_mu;
std::map<std::tuple<int, int, int>, NsWork *> g_ns;
std::map<std::tuple<int, int64_t>, double *> g_ad;  // (dev, cells) -> 2 scratch fields
std::map<std::tuple<int, int, int>, NsWork *> g_nsc;  // collocated step: 2*d fields + rhs + dp

np_status ns_work(int d, int lg, NsWork **out, bool collocated = false) {
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ns_mu);
    auto key = std::make_tuple(dev, d, lg);
    auto &cache = collocated ? g_nsc : g_ns;
    auto it = cache.find(key);
    if (it != cache.end()) { *out = it->second; return NP_OK; }
    NsWork *W = new NsWork;
    W->d = d;
    W->lg = lg;
    const size_t m = size_t(1) << (d * lg);
    if (hipMalloc((void **)&W->buf, sizeof(double) * m * (2 * d + 2)) != hipSuccess) {
        (void)hipGetLastError();
        delete W;
        set_error("hipMalloc failed for the projection-step workspace");
        return NP_ENOMEM;
    }
    cache[key] = W;
    *out = W;
    return NP_OK;
}

}  // namespace

void release_ns_cache() {
    std::lock_guard<std::mutex> lk(g_ns_mu);
    for (auto &kv : g_ns) {
        (void)hipFree(kv.second->buf);
        delete kv.second;
    }
    g_ns.clear();
    for (auto &kv : g_nsc) {
        (void)hipFree(kv.second->buf);
        delete kv.second;
    }
    g_nsc.clear();
    for (auto &kv : g_ad) (void)hipFree(kv.second);
    g_ad.clear();
}

template <int D>
static np_status ns_step_impl(int lg, double h, double *u, double *v, double *w, double *p, double dt, double nu,
                              double tol, const np_mg_opts *opts, np_mg_stats *stats, double *rhs_out,
                              double *dp_out) {
    NsWork *W = nullptr;
    NP_TRY(ns_work(D, lg, &W));
    std::lock_guard<std::mutex> lk(W->mu);
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const int64_t m = int64_t(1) << (D * lg);
    double *qt[3] = {W->buf, W->buf + m, D == 3 ? W->buf + 2 * m : nullptr};
    double *qs[3] = {W->buf + D * m, W->buf + (D + 1) * m, D == 3 ? W->buf + (D + 2) * m : nullptr};
    double *rhs = W->buf + 2 * D * m, *dp = rhs + m;
    Vel qn{{u, v, w}}, vt{{qt[0], qt[1], qt[2]}}, vs{{qs[0], qs[1], qs[2]}};
    const unsigned nb = blocks_for(m);
    const int n = 1 << lg;
    if (D == 3 && n >= 32 && g_zmarch_explicit) {
        if (g_mom_ring == 2) {
            // two-plane rings: the predictor on 128 x 4 tiles (it stores the half-step average), the
            // corrector on 64 x 4 (or 64 x 8) tiles
            const int zp = mom_planes(n, 128, 4);
            hipLaunchKernelGGL((k_mom_stage3r<0, 128, 4>), dim3(mom_grid(n, 128, 4, zp)), dim3(512), 0, s, qn, vt,
                               qt[0], qt[1], qt[2], p, n, zp, dt, nu, h);
            NP_LAUNCH_CHECK();
            const int ty = g_mom_rows, zq = mom_planes(n, 64, ty);
            if (ty == 8)
                hipLaunchKernelGGL((k_mom_stage3r<1, 64, 8>), dim3(mom_grid(n, 64, 8, zq)), dim3(512), 0, s, qn, vt,
                                   qs[0], qs[1], qs[2], p, n, zq, dt, nu, h);
            else
                hipLaunchKernelGGL((k_mom_stage3r<1, 64, 4>), dim3(mom_grid(n, 64, 4, zq)), dim3(256), 0, s, qn, vt,
                                   qs[0], qs[1], qs[2], p, n, zq, dt, nu, h);
            NP_LAUNCH_CHECK();
        } else {
            // three-plane rings: 8 tile rows for the predictor's four fields, 4 (or 8) for the corrector's seven
            const int z8 = adx_planes(n, 8), z4 = adx_planes(n, 4);
            hipLaunchKernelGGL((k_mom_stage3z<0, 8>), dim3(zgrid(n, 8, z8)), dim3(kZx * 8), 0, s, qn, vt, qt[0],
                               qt[1], qt[2], p, n, z8, dt, nu, h);
            NP_LAUNCH_CHECK();
            if (g_mom_rows == 8)
                hipLaunchKernelGGL((k_mom_stage3z<1, 8>), dim3(zgrid(n, 8, z8)), dim3(kZx * 8), 0, s, qn, vt, qs[0],
                                   qs[1], qs[2], p, n, z8, dt, nu, h);
            else
                hipLaunchKernelGGL((k_mom_stage3z<1, 4>), dim3(zgrid(n, 4, z4)), dim3(kZx * 4), 0, s, qn, vt, qs[0],
                                   qs[1], qs[2], p, n, z4, dt, nu, h);
            NP_LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL((k_mom_stage<D, 0>), dim3(nb), dim3(kBlock), 0, s, qn, vt, qt[0], qt[1], qt[2], p, lg, dt,
                           nu, h);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_mom_stage<D, 1>), dim3(nb), dim3(kBlock), 0, s, qn, vt, qs[0], qs[1], qs[2], p, lg, dt,
                           nu, h);
        NP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_div_rhs<D>), dim3(nb), dim3(kBlock), 0, s, vs, rhs, lg, -1.0 / (dt * h));
    NP_LAUNCH_CHECK();
    np_mg_opts o;
    np_default_opts(&o);
    if (opts) o = *opts;
    np_dims dims{D, {int64_t(1) << lg, int64_t(1) << lg, D == 3 ? int64_t(1) << lg : 1}};
    // warm_start 2: the increment starts from the previous step's (held in the
    // workspace), or from zero when this grid has none yet
    if (o.warm_start == 2 && !W->dp_valid) o.warm_start = 0;
    W->dp_valid = false;
    np_status st = poisson_solve(dims, h, NP_BC_PERIODIC, rhs, dp, tol, &o, stats);
    if (st == NP_EINVAL || st == NP_EHIP || st == NP_ENOMEM) return st;
    W->dp_valid = st == NP_OK;
    if (rhs_out) NP_HIP_TRY(hipMemcpyAsync(rhs_out, rhs, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    if (dp_out) NP_HIP_TRY(hipMemcpyAsync(dp_out, dp, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_correct<D>), dim3(nb), dim3(kBlock), 0, s, vs, u, v, w, p, dp, lg, dt / h);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return st;
}

// Collocated projection step: momentum (two stages into qt, qs), rhs =
// -(1/dt) D.qs, the multigrid solve A dp = rhs (periodic), q = qs - dt D dp,
// p += dp.  Workspace as the staggered step's (own cache).
template <int D, int SCHEME>
static np_status nsc_step_impl(int lg, double h, double *u, double *v, double *w, double *p, double dt, double nu,
                               double tol, const np_mg_opts *opts, np_mg_stats *stats) {
    NsWork *W = nullptr;
    NP_TRY(ns_work(D, lg, &W, true));
    std::lock_guard<std::mutex> lk(W->mu);
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const int n = 1 << lg;
    const int64_t m = int64_t(1) << (D * lg);
    double *qt[3] = {W->buf, W->buf + m, D == 3 ? W->buf + 2 * m : nullptr};
    double *qs[3] = {W->buf + D * m, W->buf + (D + 1) * m, D == 3 ? W->buf + (D + 2) * m : nullptr};
    double *rhs = W->buf + 2 * D * m, *dp = rhs + m;
    Vel qn{{u, v, w}}, vt{{qt[0], qt[1], qt[2]}}, vs{{qs[0], qs[1], qs[2]}};
    const dim3 blk(kAdxX, kAdxY), grd(unsigned((n + kAdxX - 1) / kAdxX), unsigned((n + kAdxY - 1) / kAdxY),
                                      D == 3 ? unsigned(n) : 1u);
    // 3D from 32^3: z-marching tiles
    const bool zm = D == 3 && n >= 32 && g_zmarch_explicit;
    constexpr int tys = zrows(SCHEME);  // the momentum stages' tile rows; divergence and correction: 8
    const int zcs = adx_planes(n, tys), zc = adx_planes(n, 8);
    const unsigned nzs = zgrid(n, tys, zcs), nz3 = zgrid(n, 8, zc);
    if (zm) {
        hipLaunchKernelGGL((k_nsc_stage3z<SCHEME, 0>), dim3(nzs), dim3(kZx * tys), 0, s, qn, vt, qt[0], qt[1], qt[2],
                           p, n, zcs, dt, nu, h);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_nsc_stage3z<SCHEME, 1>), dim3(nzs), dim3(kZx * tys), 0, s, qn, vt, qs[0], qs[1], qs[2],
                           p, n, zcs, dt, nu, h);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_nsc_div3z<SCHEME>), dim3(nz3), dim3(kZx * 8), 0, s, vs, rhs, n, zc, h, -1.0 / dt);
    } else {
        hipLaunchKernelGGL((k_nsc_stage<D, SCHEME, 0>), grd, blk, 0, s, qn, vt, qt[0], qt[1], qt[2], p, n, dt, nu,
                           h);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_nsc_stage<D, SCHEME, 1>), grd, blk, 0, s, qn, vt, qs[0], qs[1], qs[2], p, n, dt, nu,
                           h);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_nsc_div<D, SCHEME>), grd, blk, 0, s, vs, rhs, n, h, -1.0 / dt);
    }
    NP_LAUNCH_CHECK();
    np_mg_opts o;
    np_default_opts(&o);
    if (opts) o = *opts;
    if (o.warm_start != 0) {
        set_error("the collocated step solves the pressure increment from zero (warm_start 0)");
        return NP_EINVAL;
    }
    np_dims dims{D, {int64_t(n), int64_t(n), D == 3 ? int64_t(n) : 1}};
    np_status st = poisson_solve(dims, h, NP_BC_PERIODIC, rhs, dp, tol, &o, stats);
    if (st == NP_EINVAL || st == NP_EHIP || st == NP_ENOMEM) return st;
    if (zm)
        hipLaunchKernelGGL((k_nsc_correct3z<SCHEME>), dim3(nz3), dim3(kZx * 8), 0, s, vs, u, v, w, p, dp, n, zc, dt,
                           h);
    else
        hipLaunchKernelGGL((k_nsc_correct<D, SCHEME>), grd, blk, 0, s, vs, u, v, w, p, dp, n, dt, h);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return st;
}

}  // namespace np

using namespace np;

extern "C" np_status ns_collocated_step(np_dims dims, double h, double *u, double *v, double *w, double *p,
                                        double dt, double nu, int scheme, double tol, const np_mg_opts *opts,
                                        np_mg_stats *stats) {
    clear_error();
    const int lg = check_grid(dims);
    if (lg < 0) return NP_EINVAL;
    if (!u || !v || !p || (dims.ndim == 3 && !w)) { set_error("null velocity or pressure array"); return NP_EINVAL; }
    if (!(h > 0.0) || !(dt > 0.0) || !(nu >= 0.0) || !std::isfinite(h) || !std::isfinite(dt) || !std::isfinite(nu)) {
        set_error("h, dt must be positive and nu non-negative");
        return NP_EINVAL;
    }
    if (scheme < 0 || scheme > 2) { set_error("scheme must be 0 (central), 1 (upwind) or 2 (finite element)"); return NP_EINVAL; }
    if (dims.ndim == 2) {
        if (scheme == 0) return nsc_step_impl<2, 0>(lg, h, u, v, nullptr, p, dt, nu, tol, opts, stats);
        if (scheme == 1) return nsc_step_impl<2, 1>(lg, h, u, v, nullptr, p, dt, nu, tol, opts, stats);
        return nsc_step_impl<2, 2>(lg, h, u, v, nullptr, p, dt, nu, tol, opts, stats);
    }
    if (scheme == 0) return nsc_step_impl<3, 0>(lg, h, u, v, w, p, dt, nu, tol, opts, stats);
    if (scheme == 1) return nsc_step_impl<3, 1>(lg, h, u, v, w, p, dt, nu, tol, opts, stats);
    return nsc_step_impl<3, 2>(lg, h, u, v, w, p, dt, nu, tol, opts, stats);
}

extern "C" np_status np_nsc_divergence(np_dims dims, double h, const double *u, const double *v, const double *w,
                                       int scheme, double *div, void *stream) {
    clear_error();
    const int lg = check_grid(dims);
    if (lg < 0) return NP_EINVAL;
    if (!u || !v || !div || (dims.ndim == 3 && !w) || !(h > 0.0)) { set_error("bad argument"); return NP_EINVAL; }
    if (scheme < 0 || scheme > 2) { set_error("scheme must be 0, 1 or 2"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const int n = 1 << lg;
    Vel q{{u, v, w}};
    const dim3 blk(kAdxX, kAdxY), grd(unsigned((n + kAdxX - 1) / kAdxX), unsigned((n + kAdxY - 1) / kAdxY),
                                      dims.ndim == 3 ? unsigned(n) : 1u);
    if (dims.ndim == 2) {
        if (scheme == 2) hipLaunchKernelGGL((k_nsc_div<2, 2>), grd, blk, 0, s, q, div, n, h, 1.0);
        else hipLaunchKernelGGL((k_nsc_div<2, 0>), grd, blk, 0, s, q, div, n, h, 1.0);
    } else {
        if (scheme == 2) hipLaunchKernelGGL((k_nsc_div<3, 2>), grd, blk, 0, s, q, div, n, h, 1.0);
        else hipLaunchKernelGGL((k_nsc_div<3, 0>), grd, blk, 0, s, q, div, n, h, 1.0);
    }
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status ns_projection_step_io(np_dims dims, double h, double *u, double *v, double *w, double *p,
                                           double dt, double nu, np_bc bc, double tol, const np_mg_opts *opts,
                                           np_mg_stats *stats, double *rhs_out, double *dp_out) {
    clear_error();
    const int lg = check_grid(dims);
    if (lg < 0) return NP_EINVAL;
    if (bc != NP_BC_PERIODIC) { set_error("the projection step supports periodic boundaries only"); return NP_EINVAL; }
    if (!u || !v || !p || (dims.ndim == 3 && !w)) { set_error("null velocity or pressure array"); return NP_EINVAL; }
    if (!(h > 0.0) || !(dt > 0.0) || !(nu >= 0.0) || !std::isfinite(dt) || !std::isfinite(nu)) {
        set_error("h, dt must be positive and nu non-negative");
        return NP_EINVAL;
    }
    if (opts && opts->smooth_prec != NP_FP64 && opts->smooth_prec != NP_FP32 && opts->smooth_prec != NP_BF16) {
        set_error("unknown smooth_prec");
        return NP_EINVAL;
    }
    if (dims.ndim == 2) return ns_step_impl<2>(lg, h, u, v, nullptr, p, dt, nu, tol, opts, stats, rhs_out, dp_out);
    return ns_step_impl<3>(lg, h, u, v, w, p, dt, nu, tol, opts, stats, rhs_out, dp_out);
}

extern "C" np_status ns_projection_step(np_dims dims, double h, double *u, double *v, double *w, double *p,
                                        double dt, double nu, np_bc bc, double tol, const np_mg_opts *opts,
                                        np_mg_stats *stats) {
    return ns_projection_step_io(dims, h, u, v, w, p, dt, nu, bc, tol, opts, stats, nullptr, nullptr);
}

// Two scratch fields of m cells for the explicit steps (cached per device and size).
static np_status ad_scratch(int64_t m, double **out) {
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ns_mu);
    auto key = std::make_tuple(dev, m);
    auto it = g_ad.find(key);
    if (it != g_ad.end()) {
        *out = it->second;
        return NP_OK;
    }
    double *scr = nullptr;
    if (hipMalloc((void **)&scr, sizeof(double) * 2 * m) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc failed");
        return NP_ENOMEM;
    }
    g_ad[key] = scr;
    *out = scr;
    return NP_OK;
}

extern "C" np_status np_ad_scalar_step(np_dims dims, double h, double *T, const double *const *a, double dt,
                                       double nu, np_bc bc, const np_mg_opts *opts) {
    clear_error();
    if (dims.ndim != 2 && dims.ndim != 3) { set_error("ndim must be 2 or 3"); return NP_EINVAL; }
    const int64_t n = dims.n[0];
    for (int e = 1; e < dims.ndim; ++e)
        if (dims.n[e] != n) { set_error("all axes must have the same size"); return NP_EINVAL; }
    if (n < 3 || n > (dims.ndim == 2 ? 16384 : 1024)) { set_error("n out of range"); return NP_EINVAL; }
    if (!T || !(h > 0.0) || !(dt > 0.0) || !(nu >= 0.0)) { set_error("bad argument"); return NP_EINVAL; }
    if (bc != NP_BC_DIRICHLET0 && bc != NP_BC_PERIODIC) { set_error("unknown bc"); return NP_EINVAL; }
    APtrs ap{{nullptr, nullptr, nullptr}, 0};
    if (a) {
        for (int e = 0; e < dims.ndim; ++e) {
            if (!a[e]) { set_error("null velocity component"); return NP_EINVAL; }
            ap.a[e] = a[e];
        }
        ap.has = 1;
    }
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const int64_t m = dims.ndim == 3 ? n * n * n : n * n;
    double *scr = nullptr;
    NP_TRY(ad_scratch(m, &scr));
    Gen g{n, (int)bc};
    const unsigned nb = blocks_for(m);
    const double inv_2h = 0.5 / h, nu_inv_h2 = nu / (h * h);
    if (dims.ndim == 2) {
        hipLaunchKernelGGL((k_ad_stage<2, 0>), dim3(nb), dim3(kBlock), 0, s, T, T, scr, ap, g, dt, inv_2h, nu_inv_h2);
        hipLaunchKernelGGL((k_ad_stage<2, 1>), dim3(nb), dim3(kBlock), 0, s, T, scr, scr + m, ap, g, dt, inv_2h,
                           nu_inv_h2);
    } else {
        hipLaunchKernelGGL((k_ad_stage<3, 0>), dim3(nb), dim3(kBlock), 0, s, T, T, scr, ap, g, dt, inv_2h, nu_inv_h2);
        hipLaunchKernelGGL((k_ad_stage<3, 1>), dim3(nb), dim3(kBlock), 0, s, T, scr, scr + m, ap, g, dt, inv_2h,
                           nu_inv_h2);
    }
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipMemcpyAsync(T, scr + m, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_ad_explicit_step(np_dims dims, double h, double *T, const double *const *a, double dt,
                                         double nu, np_bc bc, int scheme, const np_mg_opts *opts) {
    clear_error();
    if (dims.ndim != 2 && dims.ndim != 3) { set_error("ndim must be 2 or 3"); return NP_EINVAL; }
    const int64_t n = dims.n[0];
    for (int e = 1; e < dims.ndim; ++e)
        if (dims.n[e] != n) { set_error("all axes must have the same size"); return NP_EINVAL; }
    if (n < 3 || n > (dims.ndim == 2 ? 16384 : 1024)) { set_error("n out of range"); return NP_EINVAL; }
    if (!T || !(h > 0.0) || !(dt > 0.0) || !(nu >= 0.0) || !std::isfinite(h) || !std::isfinite(dt) ||
        !std::isfinite(nu)) {
        set_error("bad argument");
        return NP_EINVAL;
    }
    if (bc != NP_BC_DIRICHLET0 && bc != NP_BC_PERIODIC && bc != NP_BC_NEUMANN) { set_error("unknown bc"); return NP_EINVAL; }
    if (scheme < 0 || scheme > 2) { set_error("scheme must be 0 (central), 1 (upwind) or 2 (finite element)"); return NP_EINVAL; }
    APtrs ap{{nullptr, nullptr, nullptr}, 0};
    if (a) {
        for (int e = 0; e < dims.ndim; ++e) {
            if (!a[e]) { set_error("null velocity component"); return NP_EINVAL; }
            ap.a[e] = a[e];
        }
        ap.has = 1;
    }
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const int64_t m = dims.ndim == 3 ? n * n * n : n * n;
    double *scr = nullptr;
    NP_TRY(ad_scratch(m, &scr));
    const dim3 blk(kAdxX, kAdxY), grd(unsigned((n + kAdxX - 1) / kAdxX), unsigned((n + kAdxY - 1) / kAdxY),
                                      dims.ndim == 3 ? unsigned(n) : 1u);
    const int ni = int(n);
    // predictor: scr = T~, scr + m = T^n; corrector: T = T^n - dt R((T~ + T^n)/2)
#define NP_ADX(D, S)                                                                                              \
    do {                                                                                                          \
        hipLaunchKernelGGL((k_adx_stage<D, S, 0>), grd, blk, 0, s, T, T, scr, scr + m, ap, ni, int(bc), dt, nu,   \
                           h);                                                                                    \
        hipLaunchKernelGGL((k_adx_stage<D, S, 1>), grd, blk, 0, s, scr + m, scr, T, nullptr, ap, ni, int(bc), dt, \
                           nu, h);                                                                                \
    } while (0)
    // 3D: z-marching tiles (three LDS planes) from 32^3 up
#define NP_ADX3(S)                                                                                                \
    do {                                                                                                          \
        constexpr int ty = zrows(S);                                                                              \
        const int zc = adx_planes(ni, ty);                                                                        \
        const unsigned nz3 = zgrid(ni, ty, zc);                                                                   \
        hipLaunchKernelGGL((k_adx_stage3z<S, 0>), dim3(nz3), dim3(kZx * ty), 0, s, T, T, scr, scr + m, ap, ni,    \
                           int(bc), zc, dt, nu, h);                                                               \
        hipLaunchKernelGGL((k_adx_stage3z<S, 1>), dim3(nz3), dim3(kZx * ty), 0, s, scr + m, scr, T, nullptr, ap,  \
                           ni, int(bc), zc, dt, nu, h);                                                           \
    } while (0)
    // 2D: row-marching tiles from 1024^2 up (n a multiple of the strip width)
    const int ry2 = adx_rows2(ni);
    const unsigned nr2 = unsigned((ni / kAx2) * (ni / ry2));
#define NP_ADX2(S)                                                                                                \
    do {                                                                                                          \
        hipLaunchKernelGGL((k_adx_stage2r<S, 0>), dim3(nr2), dim3(kAx2), 0, s, T, T, scr, scr + m, ap, ni,        \
                           int(bc), ry2, dt, nu, h);                                                              \
        hipLaunchKernelGGL((k_adx_stage2r<S, 1>), dim3(nr2), dim3(kAx2), 0, s, scr + m, scr, T, nullptr, ap, ni,  \
                           int(bc), ry2, dt, nu, h);                                                              \
    } while (0)
    if (dims.ndim == 2 && ni >= 1024 && ni % kAx2 == 0 && g_zmarch_explicit) {
        if (scheme == 0) NP_ADX2(0);
        else if (scheme == 1) NP_ADX2(1);
        else NP_ADX2(2);
    } else if (dims.ndim == 2) {
        if (scheme == 0) NP_ADX(2, 0);
        else if (scheme == 1) NP_ADX(2, 1);
        else NP_ADX(2, 2);
    } else if (ni >= 32 && g_zmarch_explicit) {
        if (scheme == 0) NP_ADX3(0);
        else if (scheme == 1) NP_ADX3(1);
        else NP_ADX3(2);
    } else {
        if (scheme == 0) NP_ADX(3, 0);
        else if (scheme == 1) NP_ADX(3, 1);
        else NP_ADX(3, 2);
    }
#undef NP_ADX
#undef NP_ADX2
#undef NP_ADX3
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}
