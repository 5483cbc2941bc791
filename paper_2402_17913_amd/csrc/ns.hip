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

np_status ns_work(int d, int lg, NsWork **out) {
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ns_mu);
    auto key = std::make_tuple(dev, d, lg);
    auto it = g_ns.find(key);
    if (it != g_ns.end()) { *out = it->second; return NP_OK; }
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
    g_ns[key] = W;
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
    hipLaunchKernelGGL((k_mom_stage<D, 0>), dim3(nb), dim3(kBlock), 0, s, qn, vt, qt[0], qt[1], qt[2], p, lg, dt,
                       nu, h);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mom_stage<D, 1>), dim3(nb), dim3(kBlock), 0, s, qn, vt, qs[0], qs[1], qs[2], p, lg, dt,
                       nu, h);
    NP_LAUNCH_CHECK();
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

}  // namespace np

using namespace np;

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
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    double *scr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ns_mu);
        auto key = std::make_tuple(dev, m);
        auto it = g_ad.find(key);
        if (it == g_ad.end()) {
            if (hipMalloc((void **)&scr, sizeof(double) * 2 * m) != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc failed");
                return NP_ENOMEM;
            }
            g_ad[key] = scr;
        } else {
            scr = it->second;
        }
    }
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
