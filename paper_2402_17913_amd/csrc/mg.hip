// Multigrid Poisson solver: level hierarchy, V-cycle driver, FP64 solve,
// mixed-precision iterative refinement and the single-operator entry points.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "mg_kernels.h"
#include "np_internal.h"

namespace np {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

int check_grid(const np_dims &dims) {
    if (dims.ndim != 2 && dims.ndim != 3) {
        set_error("ndim must be 2 or 3 (got %d)", dims.ndim);
        return -1;
    }
    const int64_t n = dims.n[0];
    for (int a = 1; a < dims.ndim; ++a)
        if (dims.n[a] != n) {
            set_error("all axes must have the same size");
            return -1;
        }
    const int64_t nmax = dims.ndim == 2 ? 8192 : 1024;
    if (!is_pow2(n) || n < 4 || n > nmax) {
        set_error("n must be a power of two in [4, %lld] (got %lld)", (long long)nmax, (long long)n);
        return -1;
    }
    return ilog2(n);
}

// --------------------------------------------------------------- profiling
namespace {
struct ProfRec {
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_prof_mu;
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool prof_on() { return g_prof; }

np_status prof_begin(hipStream_t s, void **tok) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = take_event();
    if (!e) {
        set_error("hipEventCreate failed");
        return NP_EHIP;
    }
    NP_HIP_TRY(hipEventRecord(e, s));
    *tok = e;
    return NP_OK;
}

np_status prof_end(hipStream_t s, void *tok, double bytes) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = take_event();
    if (!e) {
        set_error("hipEventCreate failed");
        return NP_EHIP;
    }
    NP_HIP_TRY(hipEventRecord(e, s));
    g_prof_recs.push_back(ProfRec{(hipEvent_t)tok, e, bytes});
    return NP_OK;
}

// -------------------------------------------------------------- hierarchy
// Level l has n_l = n / 2^l cells per axis, l = 0..L with n_L = 4.  Level 0
// of the plain FP64 path uses the caller's x and rhs; t[0] is its ping-pong
// partner.  The mixed path keeps the correction e, the rounded residual and
// the ping-pong buffer of level 0 in x[0], f[0], t[0].
struct Hier {
    int dev = 0, d = 0, lg = 0, L = 0, bc = 0;
    np_prec prec = NP_FP64;
    size_t es = 8;
    std::vector<void *> x, f, t;
    double *Minv = nullptr;
    double Minv_h = -1.0;     // level-0 spacing Minv was built for
    double *red = nullptr;    // kRedBlocks partials followed by 8 scalar slots
    double *hred = nullptr;   // pinned host mirror of the scalar slots
    double *f64 = nullptr;    // FP64 copy of the rhs (periodic mean removal)
    double *x64 = nullptr;    // second FP64 solution buffer (mixed path)
    std::mutex mu;            // one solve at a time per workspace
};

namespace {
std::mutex g_cache_mu;
std::map<std::tuple<int, int, int, int, int>, Hier *> g_cache;

int64_t cells(int d, int lg) { return int64_t(1) << (d * lg); }

np_status dmalloc(void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of %zu bytes failed", bytes);
        return NP_ENOMEM;
    }
    return NP_OK;
}

void free_hier(Hier *H) {
    for (auto *p : H->x) if (p) (void)hipFree(p);
    for (auto *p : H->f) if (p) (void)hipFree(p);
    for (auto *p : H->t) if (p) (void)hipFree(p);
    if (H->Minv) (void)hipFree(H->Minv);
    if (H->red) (void)hipFree(H->red);
    if (H->hred) (void)hipHostFree(H->hred);
    if (H->f64) (void)hipFree(H->f64);
    if (H->x64) (void)hipFree(H->x64);
    delete H;
}

np_status alloc_hier(Hier *H) {
    const int L = H->L;
    H->x.assign(L + 1, nullptr);
    H->f.assign(L + 1, nullptr);
    H->t.assign(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) {
        const size_t bytes = size_t(cells(H->d, H->lg - l)) * H->es;
        const bool own0 = H->prec != NP_FP64;  // plain FP64 uses the caller's x, rhs on level 0
        if (l > 0 || own0) {
            NP_TRY(dmalloc(&H->x[l], bytes));
            NP_TRY(dmalloc(&H->f[l], bytes));
        }
        NP_TRY(dmalloc(&H->t[l], bytes));
    }
    NP_TRY(dmalloc((void **)&H->Minv, sizeof(double) * 64 * 64));
    NP_TRY(dmalloc((void **)&H->red, sizeof(double) * (kRedBlocks + 8)));
    if (hipHostMalloc((void **)&H->hred, sizeof(double) * 8, hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return NP_ENOMEM;
    }
    if (H->prec != NP_FP64) NP_TRY(dmalloc((void **)&H->x64, sizeof(double) * cells(H->d, H->lg)));
    return NP_OK;
}
}  // namespace

static np_status get_hier(int d, int lg, int bc, np_prec prec, Hier **out) {
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_tuple(dev, d, lg, bc, int(prec));
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *out = it->second;
        return NP_OK;
    }
    Hier *H = new Hier;
    H->dev = dev;
    H->d = d;
    H->lg = lg;
    H->L = lg - 2;
    H->bc = bc;
    H->prec = prec;
    H->es = prec_bytes(prec);
    np_status st = alloc_hier(H);
    if (st != NP_OK) {
        free_hier(H);
        return st;
    }
    g_cache[key] = H;
    *out = H;
    return NP_OK;
}

void release_mg_cache() {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto &kv : g_cache) free_hier(kv.second);
    g_cache.clear();
}

// Dense inverse of the coarsest (4^d) operator with spacing hc, assembled
// from the stencil and the ghost rule; periodic adds 1 1^T / m.  Gauss-Jordan
// elimination with partial pivoting in FP64 on the host.
static bool coarse_inverse(int d, int bc, double hc, std::vector<double> &inv) {
    const int n = 4, m = d == 3 ? 64 : 16;
    std::vector<double> A(m * m, 0.0);
    const double w = 1.0 / (hc * hc);
    for (int c = 0; c < m; ++c) {
        const int i = c % n, j = (c / n) % n, k = c / (n * n);
        A[c * m + c] += 2.0 * d * w;
        for (int a = 0; a < d; ++a)
            for (int s = -1; s <= 1; s += 2) {
                int q[3] = {i, j, k};
                q[a] += s;
                if (q[a] < 0 || q[a] >= n) {
                    if (bc == NP_BC_PERIODIC) q[a] = (q[a] + n) % n;
                    else { A[c * m + c] += w; continue; }
                }
                A[c * m + (q[2] * n + q[1]) * n + q[0]] -= w;
            }
    }
    if (bc == NP_BC_PERIODIC)
        for (auto &v : A) v += 1.0 / m;
    inv.assign(m * m, 0.0);
    for (int i = 0; i < m; ++i) inv[i * m + i] = 1.0;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(A[r * m + col]) > std::fabs(A[piv * m + col])) piv = r;
        if (A[piv * m + col] == 0.0) return false;
        if (piv != col)
            for (int q = 0; q < m; ++q) {
                std::swap(A[piv * m + q], A[col * m + q]);
                std::swap(inv[piv * m + q], inv[col * m + q]);
            }
        const double p = A[col * m + col];
        for (int q = 0; q < m; ++q) {
            A[col * m + q] /= p;
            inv[col * m + q] /= p;
        }
        for (int r = 0; r < m; ++r)
            if (r != col) {
                const double fct = A[r * m + col];
                if (fct != 0.0)
                    for (int q = 0; q < m; ++q) {
                        A[r * m + q] -= fct * A[col * m + q];
                        inv[r * m + q] -= fct * inv[col * m + q];
                    }
            }
    }
    return true;
}

static np_status ensure_coarse(Hier *H, double h, hipStream_t s) {
    if (H->Minv_h == h) return NP_OK;
    std::vector<double> inv;
    const double hc = h * double(int64_t(1) << H->L);
    if (!coarse_inverse(H->d, H->bc, hc, inv)) {
        set_error("singular coarsest operator");
        return NP_EINVAL;
    }
    NP_HIP_TRY(hipMemcpyAsync(H->Minv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    H->Minv_h = h;
    return NP_OK;
}

// ------------------------------------------------------------ launchers
struct CycleOpts {
    int nu1 = 2, nu2 = 2;
    double omega = 2.0 / 3.0;
};

template <int D, class S> struct Ops {
    typedef typename St<S>::C C;

    static np_status jacobi(const S *f, const S *xin, S *xout, int lg, int bc, double h, double omega,
                            bool zero, hipStream_t s, bool finest) {
        const int64_t m = cells(D, lg);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        void *tok = nullptr;
        const bool prof = finest && prof_on();
        if (prof) NP_TRY(prof_begin(s, &tok));
        if (zero)
            hipLaunchKernelGGL((k_jacobi<D, S, true>), dim3(blocks_for(m)), dim3(kBlock), 0, s, f, xin,
                               xout, lg, bc, inv_h2, wdiag);
        else
            hipLaunchKernelGGL((k_jacobi<D, S, false>), dim3(blocks_for(m)), dim3(kBlock), 0, s, f, xin,
                               xout, lg, bc, inv_h2, wdiag);
        NP_LAUNCH_CHECK();
        if (prof) NP_TRY(prof_end(s, tok, double(m) * sizeof(S) * (zero ? 2 : 3)));
        return NP_OK;
    }

    static np_status resid_restrict(const S *f, const S *x, S *fc, int lg, int bc, double h,
                                    hipStream_t s) {
        const int64_t mc = cells(D, lg - 1);
        hipLaunchKernelGGL((k_resid_restrict<D, S>), dim3(blocks_for(mc)), dim3(kBlock), 0, s, f, x, fc,
                           lg, bc, C(1.0 / (h * h)));
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    static np_status prolong_add(const S *ec, S *x, int lgc, int bc, hipStream_t s) {
        const int64_t m = cells(D, lgc + 1);
        hipLaunchKernelGGL((k_prolong_add<D, S>), dim3(blocks_for(m)), dim3(kBlock), 0, s, ec, x, lgc, bc);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    static np_status coarse(const S *f, S *x, const double *Minv, int bc, double hc, bool zero,
                            hipStream_t s) {
        hipLaunchKernelGGL((k_coarse<D, S>), dim3(1), dim3(64), 0, s, f, x, Minv, bc, 1.0 / (hc * hc),
                           zero ? 1 : 0);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    // red[kRedBlocks + slot] = ||f - A x||_2 (device).
    static np_status resid_norm(const S *f, const S *x, int lg, int bc, double h, double *red, int slot,
                                hipStream_t s) {
        const int64_t m = cells(D, lg);
        const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
        hipLaunchKernelGGL((k_resid_sq<D, S>), dim3(nb), dim3(kBlock), 0, s, f, x, red, lg, bc,
                           C(1.0 / (h * h)));
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, red, int(nb), red + kRedBlocks + slot, 1);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    // One V(nu1, nu2) cycle on the hierarchy.  Level 0 works on (x0, f0) with
    // t0 as ping-pong partner; zero0 means x0 is known to be zero on entry.
    // On return the level-0 iterate is in x0.
    static np_status vcycle(Hier *H, S *x0, const S *f0, S *t0, bool zero0, double h, const CycleOpts &o,
                            hipStream_t s) {
        const int L = H->L, bc = H->bc;
        std::vector<S *> cur(L + 1), oth(L + 1);
        std::vector<const S *> F(L + 1);
        for (int l = 0; l <= L; ++l) {
            cur[l] = l == 0 ? x0 : (S *)H->x[l];
            oth[l] = l == 0 ? t0 : (S *)H->t[l];
            F[l] = l == 0 ? f0 : (const S *)H->f[l];
        }
        double hl = h;
        for (int l = 0; l < L; ++l, hl *= 2.0) {
            const int lg = H->lg - l;
            bool zero = l > 0 || zero0;
            if (zero && o.nu1 == 0) {
                hipLaunchKernelGGL((k_zero<S>), dim3(blocks_for(cells(D, lg))), dim3(kBlock), 0, s, cur[l],
                                   cells(D, lg));
                NP_LAUNCH_CHECK();
                zero = false;
            }
            for (int it = 0; it < o.nu1; ++it) {
                NP_TRY(jacobi(F[l], cur[l], oth[l], lg, bc, hl, o.omega, zero && it == 0, s, l == 0));
                std::swap(cur[l], oth[l]);
            }
            NP_TRY(resid_restrict(F[l], cur[l], (S *)H->f[l + 1], lg, bc, hl, s));
        }
        // coarsest level: exact solve (zero guess unless the whole grid is 4^d)
        NP_TRY(coarse(F[L], cur[L], H->Minv, bc, hl, L > 0 || zero0, s));
        for (int l = L - 1; l >= 0; --l) {
            hl *= 0.5;
            const int lg = H->lg - l;
            NP_TRY(prolong_add(cur[l + 1], cur[l], lg - 1, bc, s));
            for (int it = 0; it < o.nu2; ++it) {
                NP_TRY(jacobi(F[l], cur[l], oth[l], lg, bc, hl, o.omega, false, s, l == 0));
                std::swap(cur[l], oth[l]);
            }
        }
        if (cur[0] != x0)
            NP_HIP_TRY(hipMemcpyAsync(x0, cur[0], sizeof(S) * cells(D, H->lg), hipMemcpyDeviceToDevice, s));
        return NP_OK;
    }
};

// --------------------------------------------------------- solve helpers
static np_status read_scalars(Hier *H, int count, hipStream_t s) {
    NP_HIP_TRY(hipMemcpyAsync(H->hred, H->red + kRedBlocks, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// Sum (square = 0) or squared norm (square = 1) of an FP64 field into red slot.
static np_status dsum(Hier *H, const double *v, int64_t m, int square, int slot, hipStream_t s) {
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
    hipLaunchKernelGGL((k_sum<double>), dim3(nb), dim3(kBlock), 0, s, v, m, square, H->red);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->red + kRedBlocks + slot,
                       square);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

static np_status remove_mean(Hier *H, double *v, int64_t m, hipStream_t s) {
    NP_TRY(dsum(H, v, m, 0, 7, s));
    hipLaunchKernelGGL(k_sub_scaled, dim3(blocks_for(m)), dim3(kBlock), 0, s, v, m, H->red + kRedBlocks + 7,
                       1.0 / double(m));
    NP_LAUNCH_CHECK();
    return NP_OK;
}

static void fill_opts(const np_mg_opts *opts, CycleOpts &co, np_mg_opts &o) {
    np_default_opts(&o);
    if (opts) o = *opts;
    co.nu1 = o.nu1;
    co.nu2 = o.nu2;
    co.omega = o.omega;
}

struct Track {
    np_mg_stats *st;
    int n = 0;
    double first = 0.0;
    void push(double rr) {
        if (n == 0) first = rr;
        if (st && n < 256) st->hist[n] = rr;
        ++n;
    }
};

static void finish_stats(np_mg_stats *st, const Track &tr, int cycles, int outer, double rr) {
    if (!st) return;
    st->cycles = cycles;
    st->outer_iters = outer;
    st->rel_res = rr;
    const int steps = tr.n - 1;
    st->rho_est = (steps > 0 && tr.first > 0.0 && rr > 0.0) ? std::pow(rr / tr.first, 1.0 / steps) : 0.0;
}

// Decides whether to stop after seeing rr with k cycles done.  Returns 1 to
// stop (status in *st), 0 to continue.
static int stop_rule(const np_mg_opts &o, double tol, double rr, int k, const Track &tr, double prev[3],
                     np_status *st) {
    if (!std::isfinite(rr)) {
        set_error("non-finite residual norm after %d cycles", k);
        *st = NP_ENAN;
        return 1;
    }
    if (o.fixed_cycles > 0) {
        if (k >= o.fixed_cycles) { *st = NP_OK; return 1; }
        return 0;
    }
    if (rr <= tol) { *st = NP_OK; return 1; }
    if (k >= o.max_cycles) {
        set_error("tolerance %.3g not reached in %d cycles (rel_res %.3g)", tol, k, rr);
        *st = NP_ENOCONV;
        return 1;
    }
    // divergence guard: the residual grew in three consecutive cycles
    if (tr.n >= 4 && prev[0] < prev[1] && prev[1] < prev[2] && prev[2] < rr) {
        set_error("residual grew in three consecutive cycles (rel_res %.3g)", rr);
        *st = NP_ENOCONV;
        return 1;
    }
    return 0;
}

template <int D>
static np_status solve_fp64(Hier *H, const double *f, double *x, double h, double tol, const np_mg_opts &o,
                            const CycleOpts &co, hipStream_t s, bool x_zero, double nf, np_mg_stats *stats) {
    typedef Ops<D, double> O;
    Track tr{stats};
    double prev[3] = {0, 0, 0};
    int k = 0;
    np_status st = NP_OK;
    double rr = 1.0;
    for (;;) {
        if (!(k == 0 && x_zero)) {
            NP_TRY(O::resid_norm(f, x, H->lg, H->bc, h, H->red, 0, s));
            NP_TRY(read_scalars(H, 1, s));
            rr = H->hred[0] / nf;
        } else {
            rr = 1.0;  // r = f exactly for a zero iterate
        }
        tr.push(rr);
        if (stop_rule(o, tol, rr, k, tr, prev, &st)) break;
        prev[0] = prev[1]; prev[1] = prev[2]; prev[2] = rr;
        NP_TRY(O::vcycle(H, x, f, (double *)H->t[0], k == 0 && x_zero, h, co, s));
        ++k;
    }
    finish_stats(stats, tr, k, k, rr);
    return st;
}

template <int D, class SL>
static np_status solve_mixed(Hier *H, const double *f, double *x, double h, double tol, const np_mg_opts &o,
                             const CycleOpts &co, hipStream_t s, double nf, np_mg_stats *stats) {
    typedef Ops<D, SL> O;
    const int64_t m = cells(D, H->lg);
    const int inner = o.inner_cycles > 0 ? o.inner_cycles : (H->prec == NP_BF16 ? 2 : 3);
    SL *e = (SL *)H->x[0], *rlo = (SL *)H->f[0], *tt = (SL *)H->t[0];
    double *xa = x, *xb = H->x64;
    Track tr{stats};
    double prev[3] = {0, 0, 0};
    int k = 0, cycles = 0;
    np_status st = NP_OK;
    double rr = 1.0;
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
    for (;;) {
        // x <- x + e (from the second step on), r = f - A x, r_lo = round(r), ||r||
        hipLaunchKernelGGL((k_ir_resid<D, SL>), dim3(nb), dim3(kBlock), 0, s, xa, e, xb, f, rlo, H->red,
                           H->lg, H->bc, 1.0 / (h * h), k > 0 ? 1 : 0);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->red + kRedBlocks, 1);
        NP_LAUNCH_CHECK();
        if (k > 0) std::swap(xa, xb);
        NP_TRY(read_scalars(H, 1, s));
        rr = H->hred[0] / nf;
        tr.push(rr);
        if (stop_rule(o, tol, rr, k, tr, prev, &st)) break;
        prev[0] = prev[1]; prev[1] = prev[2]; prev[2] = rr;
        // inner V-cycles on A e = r_lo from e = 0
        for (int c = 0; c < inner; ++c) {
            NP_TRY(O::vcycle(H, e, rlo, tt, c == 0, h, co, s));
            ++cycles;
        }
        ++k;
    }
    if (xa != x) NP_HIP_TRY(hipMemcpyAsync(x, xa, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    finish_stats(stats, tr, cycles, k, rr);
    return st;
}

}  // namespace np

using namespace np;

extern "C" void np_default_opts(np_mg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 2.0 / 3.0;
    o->max_cycles = 200;
    o->fixed_cycles = 0;
    o->smooth_prec = NP_FP64;
    o->inner_cycles = 0;
    o->warm_start = 0;
    o->stream = nullptr;
}

extern "C" const char *np_last_error(void) { return g_err.c_str(); }

extern "C" void np_release_all(void) {
    (void)hipDeviceSynchronize();
    release_mg_cache();
    release_ns_cache();
}

extern "C" void np_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_recs) {
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    g_prof = on != 0;
}

extern "C" np_status np_prof_read(int64_t *launches, double *total_ms, double *bytes) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double ms = 0.0, by = 0.0;
    for (auto &r : g_prof_recs) {
        NP_HIP_TRY(hipEventSynchronize(r.b));
        float t = 0.0f;
        NP_HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        by += r.bytes;
    }
    if (launches) *launches = int64_t(g_prof_recs.size());
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
    return NP_OK;
}

// Common validation of the solver's scalar arguments.
static np_status check_solve_args(const np_dims &dims, double h, int bc, const void *rhs, const void *x,
                                  double tol, const np_mg_opts &o, int *lg) {
    *lg = check_grid(dims);
    if (*lg < 0) return NP_EINVAL;
    if (!(h > 0.0) || !std::isfinite(h)) { set_error("h must be positive"); return NP_EINVAL; }
    if (bc != NP_BC_DIRICHLET0 && bc != NP_BC_PERIODIC) { set_error("unknown bc %d", bc); return NP_EINVAL; }
    if (!rhs || !x) { set_error("null array"); return NP_EINVAL; }
    if (o.fixed_cycles <= 0 && !(tol > 0.0)) { set_error("tol must be positive"); return NP_EINVAL; }
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 == 0 || o.nu1 > 16 || o.nu2 > 16) {
        set_error("nu1, nu2 must be in [0, 16] and not both zero");
        return NP_EINVAL;
    }
    if (!(o.omega > 0.0 && o.omega < 2.0)) { set_error("omega must be in (0, 2)"); return NP_EINVAL; }
    if (o.max_cycles < 0 || o.fixed_cycles < 0 || o.inner_cycles < 0 || o.inner_cycles > 64) {
        set_error("bad cycle counts");
        return NP_EINVAL;
    }
    if (o.smooth_prec != NP_FP64 && o.smooth_prec != NP_FP32 && o.smooth_prec != NP_BF16) {
        set_error("unknown smooth_prec");
        return NP_EINVAL;
    }
    if (o.warm_start != 0 && o.warm_start != 2) {
        set_error("warm_start must be 0 or 2 for this entry point");
        return NP_EINVAL;
    }
    return NP_OK;
}

namespace np {
// Solve used by mg_poisson_solve and ns_projection_step.
np_status poisson_solve(np_dims dims, double h, np_bc bc, const double *rhs, double *x, double tol,
                        const np_mg_opts *opts, np_mg_stats *stats) {
    np_mg_opts o;
    CycleOpts co;
    fill_opts(opts, co, o);
    int lg = -1;
    NP_TRY(check_solve_args(dims, h, bc, rhs, x, tol, o, &lg));
    if (stats) std::memset(stats, 0, sizeof *stats);
    const int d = dims.ndim;
    hipStream_t s = (hipStream_t)o.stream;
    Hier *Hp = nullptr;
    NP_TRY(get_hier(d, lg, bc, NP_FP64, &Hp));
    Hier *H = Hp;
    Hier *HL = nullptr;
    if (o.smooth_prec != NP_FP64) NP_TRY(get_hier(d, lg, bc, o.smooth_prec, &HL));
    std::lock_guard<std::mutex> lk(H->mu);
    std::unique_lock<std::mutex> lk2;
    if (HL) lk2 = std::unique_lock<std::mutex>(HL->mu);
    const int64_t m = cells(d, lg);
    NP_TRY(ensure_coarse(H, h, s));
    if (HL) NP_TRY(ensure_coarse(HL, h, s));
    const double *f = rhs;
    if (bc == NP_BC_PERIODIC) {
        if (!H->f64) NP_TRY(dmalloc((void **)&H->f64, sizeof(double) * m));
        NP_HIP_TRY(hipMemcpyAsync(H->f64, rhs, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        NP_TRY(remove_mean(H, H->f64, m, s));
        f = H->f64;
    }
    NP_TRY(dsum(H, f, m, 1, 0, s));
    NP_TRY(read_scalars(H, 1, s));
    const double nf = H->hred[0];
    if (!std::isfinite(nf)) {
        set_error("non-finite right-hand side");
        return NP_ENAN;
    }
    const bool warm = o.warm_start == 2;
    if (nf == 0.0 || !warm) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m);
        NP_LAUNCH_CHECK();
    }
    if (nf == 0.0) {
        if (stats) { stats->cycles = 0; stats->rel_res = 0.0; }
        NP_HIP_TRY(hipStreamSynchronize(s));
        return NP_OK;
    }
    np_status st;
    if (o.smooth_prec == NP_FP64) {
        st = d == 2 ? solve_fp64<2>(H, f, x, h, tol, o, co, s, !warm, nf, stats)
                    : solve_fp64<3>(H, f, x, h, tol, o, co, s, !warm, nf, stats);
    } else if (o.smooth_prec == NP_FP32) {
        st = d == 2 ? solve_mixed<2, float>(HL, f, x, h, tol, o, co, s, nf, stats)
                    : solve_mixed<3, float>(HL, f, x, h, tol, o, co, s, nf, stats);
    } else {
        st = d == 2 ? solve_mixed<2, bf16>(HL, f, x, h, tol, o, co, s, nf, stats)
                    : solve_mixed<3, bf16>(HL, f, x, h, tol, o, co, s, nf, stats);
    }
    if (st == NP_EHIP || st == NP_ENOMEM) return st;
    if (bc == NP_BC_PERIODIC) NP_TRY(remove_mean(H, x, m, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return st;
}
}  // namespace np

extern "C" np_status mg_poisson_solve(np_dims dims, double h, np_bc bc, const double *rhs, double *x,
                                      double tol, const np_mg_opts *opts, np_mg_stats *stats) {
    clear_error();
    return poisson_solve(dims, h, bc, rhs, x, tol, opts, stats);
}

// ------------------------------------------------------ single operators
static np_status op_prelude(const np_dims &dims, double h, int bc, int *lg, bool need_h = true) {
    clear_error();
    *lg = check_grid(dims);
    if (*lg < 0) return NP_EINVAL;
    if (need_h && !(h > 0.0)) { set_error("h must be positive"); return NP_EINVAL; }
    if (bc != NP_BC_DIRICHLET0 && bc != NP_BC_PERIODIC) { set_error("unknown bc"); return NP_EINVAL; }
    return NP_OK;
}

extern "C" np_status np_op_apply(np_dims dims, double h, np_bc bc, const double *x, double *y, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (!x || !y) { set_error("null array"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = cells(dims.ndim, lg);
    if (dims.ndim == 2)
        hipLaunchKernelGGL((k_apply<2>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, y, lg, (int)bc, 1.0 / (h * h));
    else
        hipLaunchKernelGGL((k_apply<3>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, y, lg, (int)bc, 1.0 / (h * h));
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_jacobi(np_dims dims, double h, np_bc bc, double omega, const double *f,
                                  const double *x_in, double *x_out, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (!f || !x_in || !x_out || x_in == x_out) { set_error("null or aliased array"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (dims.ndim == 2)
        NP_TRY((Ops<2, double>::jacobi(f, x_in, x_out, lg, bc, h, omega, false, s, false)));
    else
        NP_TRY((Ops<3, double>::jacobi(f, x_in, x_out, lg, bc, h, omega, false, s, false)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_resid_restrict(np_dims dims, double h, np_bc bc, const double *f, const double *x,
                                          double *fc, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (lg < 3) { set_error("need n >= 8 to restrict"); return NP_EINVAL; }
    if (!f || !x || !fc) { set_error("null array"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::resid_restrict(f, x, fc, lg, bc, h, s)));
    else NP_TRY((Ops<3, double>::resid_restrict(f, x, fc, lg, bc, h, s)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_prolong_add(np_dims dims, np_bc bc, const double *ec, double *x, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, 1.0, bc, &lg, false));
    if (lg < 3) { set_error("need n >= 8 to prolongate onto"); return NP_EINVAL; }
    if (!ec || !x) { set_error("null array"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::prolong_add(ec, x, lg - 1, bc, s)));
    else NP_TRY((Ops<3, double>::prolong_add(ec, x, lg - 1, bc, s)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_vcycle(np_dims dims, double h, np_bc bc, const double *f, double *x,
                                  const np_mg_opts *opts) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (!f || !x) { set_error("null array"); return NP_EINVAL; }
    np_mg_opts o;
    CycleOpts co;
    fill_opts(opts, co, o);
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 16 || o.nu2 > 16 || !(o.omega > 0.0 && o.omega < 2.0)) {
        set_error("bad smoothing settings");
        return NP_EINVAL;
    }
    hipStream_t s = (hipStream_t)o.stream;
    Hier *H = nullptr;
    NP_TRY(get_hier(dims.ndim, lg, bc, NP_FP64, &H));
    std::lock_guard<std::mutex> lk(H->mu);
    NP_TRY(ensure_coarse(H, h, s));
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::vcycle(H, x, f, (double *)H->t[0], false, h, co, s)));
    else NP_TRY((Ops<3, double>::vcycle(H, x, f, (double *)H->t[0], false, h, co, s)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_resid_norm(np_dims dims, double h, np_bc bc, const double *f, const double *x,
                                      double *out, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (!f || !x || !out) { set_error("null pointer"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    Hier *H = nullptr;
    NP_TRY(get_hier(dims.ndim, lg, bc, NP_FP64, &H));
    std::lock_guard<std::mutex> lk(H->mu);
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::resid_norm(f, x, lg, bc, h, H->red, 0, s)));
    else NP_TRY((Ops<3, double>::resid_norm(f, x, lg, bc, h, H->red, 0, s)));
    NP_TRY(read_scalars(H, 1, s));
    *out = H->hred[0];
    return NP_OK;
}
