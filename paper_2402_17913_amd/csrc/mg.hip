// Multigrid Poisson solver: level hierarchy, V-cycle driver, FP64 solve,
// mixed-precision iterative refinement and the single-operator entry points.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "mg_fused.h"
#include "mg_block2.h"
#include "mg_fused3.h"
#include "mg_zfused.h"
#include "mg_level.h"
#include "mg_kernels.h"
#include "ad_kernels.h"
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
int g_prof = 0;
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

int prof_on() { return g_prof; }

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

// ----------------------------------------------------------------- tuning
// Runtime knobs (np_set_tuning): kernel selection and launch shapes.  The
// autotuner sets them; defaults are the measured best on gfx950.
struct Tuning {
    int fused = 0;        // fused (temporally blocked) level kernels for V(2,2)
    int tail = 1;         // one-workgroup V-cycle below 16^3 / 64^2
    int graphs = 1;       // replay cycles from captured HIP graphs
    int fmin2 = 32;       // smallest 2D level handled by fused kernels
    int fmin3 = 16;       // smallest 3D level handled by fused kernels
    int fmax2 = 1 << 14;  // largest 2D level handled by fused kernels
    int fmax3 = 1 << 12;  // largest 3D level handled by fused kernels
    int bz2 = 0;          // rows per workgroup in 2D fused kernels (0 = automatic)
    int bz3 = 0;          // planes per workgroup in 3D fused kernels (0 = automatic)
    int inner_fp32 = 3;   // default inner cycles per refinement step
    int inner_bf16 = 2;
    int batch = 4;        // first batch of cycles enqueued before reading the controller
    int greps = 8;        // most cycles (outer steps) one graph holds: 1, 2, 4 or 8
    int tailck = 1;       // the cycle's convergence check run by the one-workgroup tail kernel
    int zbar = 1;         // barriers per plane step of the 3D zero-start down-leg pass (1 or 2)
    int d2cpt = 2;        // cells per thread of the 3D nonzero down-leg pass (1: k_down2z, 2: k_down2z2)
    int d2wg = 0;         // workgroups k_down2z2 aims for (256, 512 or 1024; 0: 256 in FP64, 512 otherwise)
    int sweep3 = 1;       // z-marching sweep, restriction, prolongation and refinement kernels (3D, n >= 128)
    int psweep = 1;       // prolongation + correction and the first post-sweep in one z-marching kernel
    int ir_cpt = 2;       // cells per thread of the 3D z-marching refinement kernel (1 or 2)
    int zero2 = 1;        // first two sweeps from a zero iterate in one pass
    int sweep2z = 1;      // two sweeps in one z-marching pass on 3D levels of n >= 128 (both legs)
    int down2z = 1;       // FP32/FP64 down-leg of a nonzero iterate with its restriction in that pass
    int fuseb = 1;        // temporally blocked down-leg (from zero) and up-leg block kernels on small 3D levels
    int fbmax = 6;        // largest such level (log2 cells per axis)
    int fbnt = 1024;      // threads per workgroup of those block kernels (512: one per cell, or 1024)
    int z2wg = 1;         // one-pass kernels that fit fewer than four workgroups per CU aim at 512 workgroups
    int blk2 = 1;         // 2D levels of 128^2 .. 1024^2: one block kernel per leg (64 x 16 cells per workgroup)
};
static Tuning g_tune;
int g_zc3 = 0;

// -------------------------------------------------------------- hierarchy
// Level l has n_l = n / 2^l cells per axis, l = 0..L with n_L = 4.  Level 0
// of the plain FP64 path uses the caller's x and rhs; t[0] is its ping-pong
// partner.  The mixed path keeps the correction e, the rounded residual and
// the ping-pong buffer of level 0 in x[0], f[0], t[0].
constexpr int kPartials = 65536;
constexpr unsigned kNormBlocks = 2048;  // workgroups of a sweep that also reduces the residual norm  // per-workgroup partial sums (fixed order)

struct GraphKey {
    int kind;  // 0: FP64 cycle; mixed: 1 first update, 2 inner cycles + update (a->b or b->a); 5 sawtooth;
               // advection-diffusion: 6 V-cycle, 7 sawtooth; mixed from a zero iterate x does not hold:
               // 8 first check, 9 first update
    int zero0, check;
    const void *x, *f;
    double h;
    int nu1, nu2, inner;
    double omega;
    double ad[5];  // advection-diffusion operator: dt, nu, a[3] (zero otherwise)
    int ad_scheme, ad_l1;
    int reps, par;  // run_graphs: the repetitions one graph holds, the parity of the first one
    bool operator==(const GraphKey &o) const {
        return kind == o.kind && zero0 == o.zero0 && check == o.check && x == o.x && f == o.f && h == o.h &&
               nu1 == o.nu1 && nu2 == o.nu2 && inner == o.inner && omega == o.omega &&
               std::memcmp(ad, o.ad, sizeof ad) == 0 && ad_scheme == o.ad_scheme && ad_l1 == o.ad_l1 &&
               reps == o.reps && par == o.par;
    }
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t used;
};

struct Hier {
    int dev = 0, d = 0, lg = 0, L = 0, bc = 0;
    np_prec prec = NP_FP64;
    size_t es = 8;
    bool levels = false;      // level buffers allocated
    std::vector<void *> x, f, t;
    double *Minv = nullptr;
    double Minv_h = -1.0;     // level-0 spacing Minv was built for
    double *red = nullptr;    // kPartials partials followed by 8 scalar slots
    double *hred = nullptr;   // pinned host mirror of the scalar slots
    double *f64 = nullptr;    // FP64 copy of the rhs (periodic mean removal)
    double *x64 = nullptr;    // second FP64 solution buffer (mixed path)
    double *saw = nullptr;    // level-0 correction and its partner (sawtooth cycle)
    double *ad_minv = nullptr;  // advection-diffusion: inverse of the coarsest operator
    double ad_key[6] = {-1.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // ad_minv built for: coarsest spacing, dt, nu, a[3]
    int ad_key_scheme = -1;
    double *xold = nullptr;   // advection-diffusion: iterate before the cycle (change gauge)
    double *ad_l1 = nullptr;  // advection-diffusion: per-cycle L1 change (256 slots)
    Ctl *ctl = nullptr;       // device controller
    Ctl *hctl = nullptr;      // pinned host mirror
    hipStream_t cap = nullptr;  // capture stream
    std::vector<GraphEntry> graphs;
    uint64_t tick = 0;
    bool direct = false;      // enqueue cycles directly, never capture or replay graphs
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

void drop_graphs(Hier *H) {
    for (auto &g : H->graphs) (void)hipGraphExecDestroy(g.exec);
    H->graphs.clear();
}

void free_hier(Hier *H) {
    drop_graphs(H);
    for (auto *p : H->x) if (p) (void)hipFree(p);
    for (auto *p : H->f) if (p) (void)hipFree(p);
    for (auto *p : H->t) if (p) (void)hipFree(p);
    if (H->Minv) (void)hipFree(H->Minv);
    if (H->red) (void)hipFree(H->red);
    if (H->hred) (void)hipHostFree(H->hred);
    if (H->f64) (void)hipFree(H->f64);
    if (H->x64) (void)hipFree(H->x64);
    if (H->saw) (void)hipFree(H->saw);
    if (H->ad_minv) (void)hipFree(H->ad_minv);
    if (H->xold) (void)hipFree(H->xold);
    if (H->ad_l1) (void)hipFree(H->ad_l1);
    if (H->ctl) (void)hipFree(H->ctl);
    if (H->hctl) (void)hipHostFree(H->hctl);
    if (H->cap) (void)hipStreamDestroy(H->cap);
    delete H;
}

np_status alloc_base(Hier *H) {
    NP_TRY(dmalloc((void **)&H->Minv, sizeof(double) * 64 * 64));
    NP_TRY(dmalloc((void **)&H->red, sizeof(double) * (kPartials + 8)));
    NP_TRY(dmalloc((void **)&H->ctl, sizeof(Ctl)));
    if (hipHostMalloc((void **)&H->hred, sizeof(double) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&H->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc failed");
        return NP_ENOMEM;
    }
    NP_HIP_TRY(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
    return NP_OK;
}
}  // namespace

// Allocates the level buffers on first use.
static np_status ensure_levels(Hier *H) {
    if (H->levels) return NP_OK;
    const int L = H->L;
    H->x.assign(L + 1, nullptr);
    H->f.assign(L + 1, nullptr);
    H->t.assign(L + 1, nullptr);
    const bool own0 = H->prec != NP_FP64;  // plain FP64 uses the caller's x and rhs on level 0
    for (int l = 0; l <= L; ++l) {
        const size_t bytes = size_t(cells(H->d, H->lg - l)) * H->es;
        if (l > 0 || own0) {
            NP_TRY(dmalloc(&H->x[l], bytes));
            NP_TRY(dmalloc(&H->f[l], bytes));
        }
        NP_TRY(dmalloc(&H->t[l], bytes));
    }
    if (H->prec != NP_FP64) NP_TRY(dmalloc((void **)&H->x64, sizeof(double) * cells(H->d, H->lg)));
    H->levels = true;
    return NP_OK;
}

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
    np_status st = alloc_base(H);
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

bool coarse_inverse_host(int d, int bc, double hc, std::vector<double> &inv) { return coarse_inverse(d, bc, hc, inv); }

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

// Fused tile shapes: 3D tiles are 64 (x) by 16 (y) columns including the halo;
// 2D tiles are 256 columns wide.
template <int D> struct Tile {
    static constexpr int TX = D == 3 ? 64 : 256;
    static constexpr int TY = D == 3 ? 16 : 1;
};

// Learned coarse-grid correction (np_mg_opts.cnn_cgc): on the way down, at
// `level` (after its right-hand side, the restricted residual, is written and
// before its first sweep), fn may set the level's iterate buffer to a starting
// correction and report whether it did; otherwise the level starts from zero.
struct CgcHook {
    int level = -1;
    std::function<np_status(const void *f, void *x, double h, hipStream_t s, bool *used)> fn;
};

// log2 size of the finest level of the cycle being enqueued (for profiling
// the finest-level launches only).
static thread_local int H_lg_top = -1;

template <int D, class S> struct Ops {
    typedef typename St<S>::C C;

    static np_status jacobi(const S *f, const S *xin, S *xout, int lg, int bc, double h, double omega,
                            bool zero, hipStream_t s, bool finest, const int *stop) {
        const int64_t m = cells(D, lg);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        void *tok = nullptr;
        const bool prof = finest && (prof_on() & kProfJacobi);
        if (prof) NP_TRY(prof_begin(s, &tok));
        if (zero)
            hipLaunchKernelGGL((k_jacobi<D, S, true>), dim3(blocks_for(m)), dim3(kBlock), 0, s, f, xin,
                               xout, lg, bc, inv_h2, wdiag, stop);
        else
            hipLaunchKernelGGL((k_jacobi<D, S, false>), dim3(blocks_for(m)), dim3(kBlock), 0, s, f, xin,
                               xout, lg, bc, inv_h2, wdiag, stop);
        NP_LAUNCH_CHECK();
        if (prof) NP_TRY(prof_end(s, tok, double(m) * sizeof(S) * (zero ? 2 : 3)));
        return NP_OK;
    }

    // Jacobi sweep used inside cycles; with partial != null it also reduces
    // ||f - A x_in||^2 into one partial per workgroup (count in *np).
    // zmode 0: one sweep of xin; 1: the sweep from a zero iterate (x = w f);
    // 2: the first two sweeps from a zero iterate in one pass (xin unused).
    static np_status sweep(const S *f, const S *xin, S *xout, int lg, int bc, double h, double omega, int zmode,
                           double *partial, int *np, hipStream_t s, bool finest, const int *stop) {
        const int64_t m = cells(D, lg);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        unsigned nb = unsigned((m + kSweepCells - 1) / kSweepCells);
        if (partial) nb = std::min<unsigned>(nb, kNormBlocks);  // few partials: a cheap check
        void *tok = nullptr;
        const bool prof = finest && (prof_on() & (zmode ? kProfSweepZero : kProfJacobi));
        if (prof) NP_TRY(prof_begin(s, &tok));
        if (D == 3 && zmode != 1 && lg >= 7 && g_tune.sweep3) {
            constexpr int CPT = ZCfg<S>::CPT;
            const int zc = sweep3_planes(lg, CPT, kPartials);
            nb = zblocks(lg, CPT, zc);
            if (zmode == 2)
                hipLaunchKernelGGL((k_sweep3<S, false, true>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, xout, partial,
                                   lg, bc, zc, inv_h2, wdiag, stop);
            else if (partial)
                hipLaunchKernelGGL((k_sweep3<S, true>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, xout, partial, lg,
                                   bc, zc, inv_h2, wdiag, stop);
            else
                hipLaunchKernelGGL((k_sweep3<S, false>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, xout, partial, lg,
                                   bc, zc, inv_h2, wdiag, stop);
        } else if (zmode == 1)
            hipLaunchKernelGGL((k_sweep<D, S, true, false>), dim3(nb), dim3(kBlock), 0, s, f, xin, xout, partial, lg,
                               bc, inv_h2, wdiag, stop);
        else if (zmode == 2)
            hipLaunchKernelGGL((k_sweep<D, S, false, false, true>), dim3(nb), dim3(kBlock), 0, s, f, xin, xout,
                               partial, lg, bc, inv_h2, wdiag, stop);
        else if (partial)
            hipLaunchKernelGGL((k_sweep<D, S, false, true>), dim3(nb), dim3(kBlock), 0, s, f, xin, xout, partial,
                               lg, bc, inv_h2, wdiag, stop);
        else
            hipLaunchKernelGGL((k_sweep<D, S, false, false>), dim3(nb), dim3(kBlock), 0, s, f, xin, xout, partial,
                               lg, bc, inv_h2, wdiag, stop);
        NP_LAUNCH_CHECK();
        if (prof) NP_TRY(prof_end(s, tok, double(m) * sizeof(S) * (zmode ? 2 : 3)));
        if (np) *np = int(nb);
        return NP_OK;
    }

    // Residual + restriction inside cycles (block kernel where the level is wide enough).
    static np_status restrict_(const S *f, const S *x, S *fc, int lg, int bc, double h, hipStream_t s,
                               const int *stop) {
        const int n = 1 << lg;
        if (n >= RBlk<D>::FX) {
            const int64_t nb = int64_t(n / RBlk<D>::FX) * (n / 2) * (D == 3 ? n / 2 : 1);
            void *tok = nullptr;
            const bool prof = lg == H_lg_top && (prof_on() & kProfRestrict);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (D == 3 && lg >= 7 && g_tune.sweep3) {
                constexpr int CPT = ZCfg<S>::CPT;
                const int zc = sweep3_planes(lg, CPT, kPartials);
                hipLaunchKernelGGL((k_restrict3<S>), dim3(zblocks(lg, CPT, zc)), dim3(kS3Threads), 0, s, f, x, fc, lg,
                                   bc, zc, C(1.0 / (h * h)), stop);
            } else {
                hipLaunchKernelGGL((k_restrict<D, S>), dim3(unsigned(nb)), dim3(kBlock), 0, s, f, x, fc, lg, bc,
                                   C(1.0 / (h * h)), stop);
            }
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * 2 * sizeof(S) + m / (1 << D) * sizeof(S)));
            }
            return NP_OK;
        }
        return resid_restrict(f, x, fc, lg, bc, h, s, stop);
    }

    // ctl: the tail first runs the convergence check on the np partials.
    static np_status tail(const S *f, S *x, const double *Minv, int lg, int bc, double h, const CycleOpts &o,
                          hipStream_t s, const int *stop, const double *partial = nullptr, int np = 0,
                          Ctl *ctl = nullptr) {
        hipLaunchKernelGGL((k_tail<D, S>), dim3(1), dim3(Tail<D>::NT), 0, s, f, x, Minv, lg, bc, h, o.omega, o.nu1,
                           o.nu2, stop, partial, np, ctl);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    static np_status resid_restrict(const S *f, const S *x, S *fc, int lg, int bc, double h, hipStream_t s,
                                    const int *stop) {
        const int64_t mc = cells(D, lg - 1);
        hipLaunchKernelGGL((k_resid_restrict<D, S>), dim3(blocks_for(mc)), dim3(kBlock), 0, s, f, x, fc,
                           lg, bc, C(1.0 / (h * h)), stop);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    static np_status prolong_add(const S *ec, S *x, int lgc, int bc, hipStream_t s, const int *stop) {
        const int64_t m = cells(D, lgc + 1);
        void *tok = nullptr;
        const bool prof = lgc + 1 == H_lg_top && (prof_on() & kProfProlong);
        if (prof) NP_TRY(prof_begin(s, &tok));
        if (D == 3 && lgc + 1 >= 5 && g_tune.sweep3) {
            // z-marching tiles from 32^3 up: the same arithmetic as the fused prolongation + sweep
            constexpr int CPT = ZCfg<S>::CPT;
            const int lg = lgc + 1, zc = sweep3_planes(lg, CPT, kPartials);
            by_tile_width(lg, [&](auto tx) {
                hipLaunchKernelGGL((k_prolong3<S, decltype(tx)::value>), dim3(zblocks(lg, CPT, zc)), dim3(kS3Threads),
                                   0, s, ec, x, lg, bc, zc, stop);
            });
        } else {
            hipLaunchKernelGGL((k_prolong_add<D, S>), dim3(blocks_for(m)), dim3(kBlock), 0, s, ec, x, lgc, bc,
                               stop);
        }
        NP_LAUNCH_CHECK();
        if (prof) NP_TRY(prof_end(s, tok, double(m) * 2 * sizeof(S) + double(m) / (1 << D) * sizeof(S)));
        return NP_OK;
    }

    // Whether a 3D level runs the block kernels (k_down0_b, k_up2_b): levels from 32^3 up to 2^fbmax.
    static bool fuseb_on(int lg) { return D == 3 && g_tune.fuseb && lg >= 5 && lg <= g_tune.fbmax; }

    // The block forms of down0 and up2 (8^3 cells per workgroup).
    static np_status down0b(const S *f, S *x, S *fc, int lg, int bc, double h, double omega, hipStream_t s,
                            bool finest, const int *stop) {
        if constexpr (D == 3) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            const unsigned nb = unsigned(int64_t(1) << (3 * (lg - 3)));
            void *tok = nullptr;
            const bool prof = finest && (prof_on() & kProfDownZero);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (g_tune.fbnt == 1024)
                hipLaunchKernelGGL((k_down0_b<S, 8, 1024>), dim3(nb), dim3(1024), 0, s, f, x, fc, lg, bc, inv_h2, wdiag,
                                   stop);
            else
                hipLaunchKernelGGL((k_down0_b<S, 8>), dim3(nb), dim3(BTile<8>::NT), 0, s, f, x, fc, lg, bc, inv_h2,
                                   wdiag, stop);
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * sizeof(S) * 2 + m / 8 * sizeof(S)));
            }
            return NP_OK;
        } else {
            (void)f; (void)x; (void)fc; (void)lg; (void)bc; (void)h; (void)omega; (void)s; (void)finest; (void)stop;
            return NP_EINVAL;
        }
    }
    static np_status up2b(const S *ec, const S *f, const S *x, S *xout, int lg, int bc, double h, double omega,
                          hipStream_t s, bool finest, const int *stop) {
        if constexpr (D == 3) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            const unsigned nb = unsigned(int64_t(1) << (3 * (lg - 3)));
            void *tok = nullptr;
            const bool prof = finest && (prof_on() & kProfUp);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (g_tune.fbnt == 1024)
                hipLaunchKernelGGL((k_up2_b<S, 8, 1024>), dim3(nb), dim3(1024), 0, s, ec, f, x, xout, lg, bc, inv_h2,
                                   wdiag, stop);
            else
                hipLaunchKernelGGL((k_up2_b<S, 8>), dim3(nb), dim3(BTile<8>::NT), 0, s, ec, f, x, xout, lg, bc,
                                   inv_h2, wdiag, stop);
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * sizeof(S) * 3 + m / 8 * sizeof(S)));
            }
            return NP_OK;
        } else {
            (void)ec; (void)f; (void)x; (void)xout; (void)lg; (void)bc; (void)h; (void)omega; (void)s; (void)finest;
            (void)stop;
            return NP_EINVAL;
        }
    }

    // Whether a 3D level of n >= 128 runs its two pre-sweeps, or its up-leg (prolongation + correction
    // and two post-sweeps), as one z-marching pass (k_sweep2z); 32-bit offsets bound it to n <= 1024.
    static bool z2_on(int lg) { return D == 3 && g_tune.sweep2z && g_tune.sweep3 && lg >= 7 && lg <= 10; }

    // xout = sweep(sweep(x')) on a 3D level of 128 <= n <= 1024 (k_sweep2z), x' = x + P ec when ec is
    // given, else x; with `partial`, also the per-workgroup partials of |f - A x|^2 (their count in *np).
    static np_status sweep2z(const S *ec, const S *f, const S *x, S *xout, double *partial, int *np, int lg,
                             int bc, double h, double omega, hipStream_t s, bool finest, const int *stop) {
        if constexpr (D == 3) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            constexpr int CPT = ZCfg<S>::CPT;
            // up-leg: 512 workgroups (two per CU), 256 in FP64 (one per CU at 129 VGPRs)
            const int zc = sweep2z_planes<S>(lg, ec && g_tune.z2wg ? (sizeof(S) == 8 ? 256 : 512) : 1024);
            const unsigned nb = zblocks(lg, CPT, zc);
            void *tok = nullptr;
            const bool prof = finest && (prof_on() & (ec ? kProfUp : kProfJacobi));
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (ec)
                hipLaunchKernelGGL((k_sweep2z<S, true, false>), dim3(nb), dim3(kS3Threads), 0, s, ec, f, x, xout,
                                   nullptr, lg, bc, zc, inv_h2, wdiag, stop);
            else if (partial)
                hipLaunchKernelGGL((k_sweep2z<S, false, true>), dim3(nb), dim3(kS3Threads), 0, s, nullptr, f, x,
                                   xout, partial, lg, bc, zc, inv_h2, wdiag, stop);
            else
                hipLaunchKernelGGL((k_sweep2z<S, false, false>), dim3(nb), dim3(kS3Threads), 0, s, nullptr, f, x,
                                   xout, nullptr, lg, bc, zc, inv_h2, wdiag, stop);
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * sizeof(S) * 3 + (ec ? m / 8 * sizeof(S) : 0.0)));
            }
            if (np) *np = int(nb);
            return NP_OK;
        } else {
            (void)ec; (void)f; (void)x; (void)xout; (void)partial; (void)np; (void)lg; (void)bc; (void)h;
            (void)omega; (void)s; (void)finest; (void)stop;
            return NP_EINVAL;
        }
    }

    // x = sweep(sweep(0)) and fc = R (f - A x) in one z-marching pass on a 3D level of
    // 128 <= n <= 1024 (k_down0z).
    static np_status down0z(const S *f, S *x, S *fc, int lg, int bc, double h, double omega, hipStream_t s,
                            bool finest, const int *stop) {
        if constexpr (D == 3) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            constexpr int CPT = ZCfg<S>::CPT;
            const int zc = sweep2z_planes<S>(lg, sizeof(S) == 8 && g_tune.z2wg ? 512 : 1024);
            void *tok = nullptr;
            const bool prof = finest && (prof_on() & kProfDownZero);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (g_tune.zbar == 1)
                hipLaunchKernelGGL((k_down0z1<S>), dim3(zblocks(lg, CPT, zc)), dim3(kS3Threads), 0, s, f, x, fc, lg,
                                   bc, zc, inv_h2, wdiag, stop);
            else
                hipLaunchKernelGGL((k_down0z<S>), dim3(zblocks(lg, CPT, zc)), dim3(kS3Threads), 0, s, f, x, fc, lg,
                                   bc, zc, inv_h2, wdiag, stop);
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * sizeof(S) * 2 + m / 8 * sizeof(S)));
            }
            return NP_OK;
        } else {
            (void)f; (void)x; (void)fc; (void)lg; (void)bc; (void)h; (void)omega; (void)s; (void)finest; (void)stop;
            return NP_EINVAL;
        }
    }

    // x = sweep(sweep(xin)) and fc = R (f - A x) in one z-marching pass on a 3D level of
    // 128 <= n <= 1024 in FP32 or FP64 storage (k_down2z); with `partial`, also the per-workgroup
    // partials of |f - A xin|^2 (their count in *np).
    // In the cycle: FP64 and FP32 from 256^3 (at 128^3 the one-cell form measured no faster, FP64
    // 28.2 against 26.6 us for the two passes).  On two cells per thread (k_down2z2, 512
    // workgroups) the 256^3 solves measured FP32-mixed 4.17 -> 4.01 ms and FP64 6.47 -> 6.18 ms
    // against the one-cell form in FP64 and the two passes in FP32; BF16 keeps the two passes
    // (4.455 against 4.48 ms).
    static bool down2_on(int lg) {
        return z2_on(lg) && lg >= 8 && (sizeof(S) == 8 || (sizeof(S) == 4 && g_tune.d2cpt == 2)) &&
               g_tune.down2z;
    }
    static np_status down2z(const S *f, const S *xin, S *x, S *fc, double *partial, int *np, int lg, int bc,
                            double h, double omega, hipStream_t s, bool finest, const int *stop) {
        if constexpr (D == 3) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            const bool two = g_tune.d2cpt == 2;  // two cells per thread (k_down2z2)
            // two cells per thread: one workgroup per CU in FP64 (148 VGPRs: the FP64 solve measured
            // 6.18 ms at 512 workgroups, 5.95 at 256), two in FP32 (85: 3.97 ms at 512, 4.13 at 256)
            const int wg2 = g_tune.d2wg ? g_tune.d2wg : (sizeof(S) == 8 ? 256 : 512);
            const int zc = two ? sweep2z_planes<S>(lg, wg2) : down2z_planes<S>(lg);
            const unsigned nb = zblocks(lg, two ? 2 : 1, zc);
            void *tok = nullptr;
            const bool prof = finest && (prof_on() & kProfDown);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (two && partial)
                hipLaunchKernelGGL((k_down2z2<S, true>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, x, fc, partial, lg,
                                   bc, zc, inv_h2, wdiag, stop);
            else if (two)
                hipLaunchKernelGGL((k_down2z2<S, false>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, x, fc, nullptr,
                                   lg, bc, zc, inv_h2, wdiag, stop);
            else if (partial)
                hipLaunchKernelGGL((k_down2z<S, true>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, x, fc, partial, lg,
                                   bc, zc, inv_h2, wdiag, stop);
            else
                hipLaunchKernelGGL((k_down2z<S, false>), dim3(nb), dim3(kS3Threads), 0, s, f, xin, x, fc, nullptr,
                                   lg, bc, zc, inv_h2, wdiag, stop);
            NP_LAUNCH_CHECK();
            if (prof) {
                const double m = double(cells(D, lg));
                NP_TRY(prof_end(s, tok, m * sizeof(S) * 3 + m / 8 * sizeof(S)));
            }
            if (np) *np = int(nb);
            return NP_OK;
        } else {
            (void)f; (void)xin; (void)x; (void)fc; (void)partial; (void)np; (void)lg; (void)bc; (void)h; (void)omega;
            (void)s; (void)finest; (void)stop;
            return NP_EINVAL;
        }
    }

    // 2D levels of 128^2 .. 1024^2 above the tail: one block kernel per leg (k_lvl2_b: MODE 0 the
    // down-leg from zero, 1 the down-leg of an iterate, 2 the up-leg), 64 x 16 cells per workgroup.
    static bool blk2_on(int lg) { return D == 2 && g_tune.blk2 && lg >= 7 && lg <= 10 && lg > Tail<2>::LG; }
    template <int MODE, bool NORM>
    static np_status lvl2b(const S *ec, const S *f, const S *xin, S *xout, S *fc, double *partial, int *np, int lg,
                           int bc, double h, double omega, hipStream_t s, const int *stop) {
        if constexpr (D == 2) {
            const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
            const int n = 1 << lg;
            const unsigned nb = unsigned((n / B2<S>::BX) * (n / B2<S>::BY));
            hipLaunchKernelGGL((k_lvl2_b<S, MODE, NORM>), dim3(nb), dim3(B2<S>::NT), 0, s, ec, f, xin, xout, fc,
                               partial, lg, bc, inv_h2, wdiag, stop);
            NP_LAUNCH_CHECK();
            if (np) *np = int(nb);
            return NP_OK;
        } else {
            (void)ec; (void)f; (void)xin; (void)xout; (void)fc; (void)partial; (void)np; (void)lg; (void)bc; (void)h;
            (void)omega; (void)s; (void)stop;
            return NP_EINVAL;
        }
    }

    // Whether prolongation + correction and the first post-sweep of a level run as one kernel
    // (2D: every level above the tail; 3D: levels of n >= 32 on the z-marching tiles).
    static bool psweep_on(int lg, int nu2) {
        if (!g_tune.psweep || nu2 < 1) return false;
        return D == 2 || (lg >= 5 && g_tune.sweep3);
    }

    // Calls fn(std::integral_constant<int, TX>) with the z-marching tile width of a
    // 3D level of 2^lg >= 32 cells per axis (128, or the level's width below that).
    template <class Fn>
    static void by_tile_width(int lg, Fn &&fn) {
        if (lg >= 7) fn(std::integral_constant<int, 128>());
        else if (lg == 6) fn(std::integral_constant<int, 64>());
        else fn(std::integral_constant<int, 32>());
    }

    // xout = sweep(x + P ec) on a level of 2^lg cells per axis (k_psweep3 in 3D, k_psweep in 2D;
    // psweep_on holds).
    static np_status psweep(const S *ec, const S *f, const S *x, S *xout, int lg, int bc, double h, double omega,
                            hipStream_t s, bool finest, const int *stop) {
        const int64_t m = cells(D, lg);
        const C inv_h2 = C(1.0 / (h * h)), wdiag = C(omega * h * h / (2.0 * D));
        void *tok = nullptr;
        const bool prof = finest && (prof_on() & kProfUp);
        if (prof) NP_TRY(prof_begin(s, &tok));
        if constexpr (D == 3) {
            constexpr int CPT = ZCfg<S>::CPT;
            const int zc = sweep3_planes(lg, CPT, kPartials);
            by_tile_width(lg, [&](auto tx) {
                hipLaunchKernelGGL((k_psweep3<S, decltype(tx)::value>), dim3(zblocks(lg, CPT, zc)),
                                   dim3(kS3Threads), 0, s, ec, f, x, xout, lg, bc, zc, inv_h2, wdiag, stop);
            });
        } else {
            hipLaunchKernelGGL((k_psweep<D, S>), dim3(blocks_for(m)), dim3(kBlock), 0, s, ec, f, x, xout, lg, bc,
                               inv_h2, wdiag, stop);
        }
        NP_LAUNCH_CHECK();
        if (prof) NP_TRY(prof_end(s, tok, double(m) * 3 * sizeof(S) + double(m) / (1 << D) * sizeof(S)));
        return NP_OK;
    }

    static np_status coarse(const S *f, S *x, const double *Minv, int bc, double hc, bool zero,
                            hipStream_t s, const int *stop) {
        hipLaunchKernelGGL((k_coarse<D, S>), dim3(1), dim3(64), 0, s, f, x, Minv, bc, 1.0 / (hc * hc),
                           zero ? 1 : 0, stop);
        NP_LAUNCH_CHECK();
        return NP_OK;
    }

    // Partials of ||f - A x||^2 (one per workgroup, <= kRedBlocks) into red.
    static np_status resid_sq(const S *f, const S *x, int lg, int bc, double h, double *red, hipStream_t s,
                              const int *stop, int *np) {
        const int64_t m = cells(D, lg);
        const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
        (void)stop;
        hipLaunchKernelGGL((k_resid_sq<D, S>), dim3(nb), dim3(kBlock), 0, s, f, x, red, lg, bc,
                           C(1.0 / (h * h)));
        NP_LAUNCH_CHECK();
        *np = int(nb);
        return NP_OK;
    }

    // Partials of x (f + r) (k_energy); *np receives their count.
    static np_status energy(const S *f, const S *x, int lg, int bc, double h, double *red, hipStream_t s, int *np) {
        const int64_t m = cells(D, lg);
        const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
        hipLaunchKernelGGL((k_energy<D, S>), dim3(nb), dim3(kBlock), 0, s, f, x, red, lg, bc, C(1.0 / (h * h)));
        NP_LAUNCH_CHECK();
        *np = int(nb);
        return NP_OK;
    }

    // One fused pass over a level (see mg_fused.h).  Returns the number of
    // workgroups (= partial sums written when NORM).
    template <int NJ, int PRE, bool RES, bool NORM>
    static np_status fused(const S *xin, const S *f, S *xout, const S *ec, S *fc, double *partial, int lg, int bc,
                           double h, double omega, hipStream_t s, const int *stop, bool finest, int *nblk) {
        constexpr int TX = Tile<D>::TX, TY = Tile<D>::TY;
        constexpr int H = NJ + (RES ? 1 : 0);
        constexpr int BX = TX - 2 * H, BY = D == 3 ? TY - 2 * H : 1;
        const int n = 1 << lg;
        FusedArgs<S> a;
        a.xin = xin; a.f = f; a.xout = xout; a.ec = ec; a.fc = fc; a.partial = partial; a.stop = stop;
        a.lg = lg; a.bc = bc;
        a.tiles_x = (n + BX - 1) / BX;
        a.tiles_y = D == 3 ? (n + BY - 1) / BY : 1;
        const int tiles = a.tiles_x * a.tiles_y;
        int bz = D == 3 ? g_tune.bz3 : g_tune.bz2;
        if (bz <= 0) {
            // enough workgroups to fill the chip, without making the marching halo dominant
            bz = n;
            while (bz > 8 && int64_t(tiles) * (n / bz) < 1024) bz >>= 1;
        }
        if (bz > n) bz = n;
        if (bz < 2) bz = 2;
        a.bz = bz;
        a.nblocks = tiles * (n / bz);
        if (NORM && a.nblocks > kPartials) {
            set_error("fused launch needs %d partials (max %d)", a.nblocks, kPartials);
            return NP_EINVAL;
        }
        a.inv_h2 = C(1.0 / (h * h));
        a.wdiag = C(omega * h * h / (2.0 * D));
        void *tok = nullptr;
        const int kind = PRE == PRE_PROLONG ? kProfUp : (PRE == PRE_ZERO ? kProfDownZero : kProfDown);
        const bool prof = finest && (prof_on() & kind);
        if (prof) NP_TRY(prof_begin(s, &tok));
        hipLaunchKernelGGL((k_fused<D, S, TX, TY, NJ, PRE, RES, NORM>), dim3(a.nblocks), dim3(256), 0, s, a);
        NP_LAUNCH_CHECK();
        if (prof) {
            // algorithmic bytes: stage-0 input (x unless zero guess, f), output x, coarse in/out
            const double m = double(cells(D, lg)), es = double(sizeof(S));
            double by = m * es;                                   // f
            if (PRE != PRE_ZERO) by += m * es;                    // x in
            if (NJ > 0) by += m * es;                             // x out
            if (PRE == PRE_PROLONG) by += m * es / (1 << D);      // coarse error
            if (RES) by += m * es / (1 << D);                     // restricted residual
            NP_TRY(prof_end(s, tok, by));
        }
        if (nblk) *nblk = a.nblocks;
        return NP_OK;
    }

    // Enqueues one V(nu1, nu2) cycle on the hierarchy.  Level 0 works on
    // (x0, f0) with t0 as partner; zero0: x0 is zero on entry (it is not
    // read); check: the residual norm of x0 is reduced and the controller's
    // stop rule runs before the rest of the cycle.  The level-0 result is in x0.
    static np_status cycle(Hier *H, S *x0, const S *f0, S *t0, bool zero0, bool check, double h,
                           const CycleOpts &o, hipStream_t s, const CgcHook *hook = nullptr) {
        const int L = H->L, bc = H->bc;
        const int *stop = &H->ctl->stop;
        H_lg_top = H->lg;
        const bool fz = g_tune.fused && o.nu1 == 2 && o.nu2 == 2;
        const int fmin = D == 3 ? g_tune.fmin3 : g_tune.fmin2;
        const int fmax = D == 3 ? g_tune.fmax3 : g_tune.fmax2;
        std::vector<S *> cur(L + 1), oth(L + 1), res(L + 1);
        std::vector<const S *> F(L + 1);
        std::vector<bool> fl(L + 1);
        for (int l = 0; l <= L; ++l) {
            cur[l] = l == 0 ? x0 : (S *)H->x[l];
            oth[l] = l == 0 ? t0 : (S *)H->t[l];
            F[l] = l == 0 ? f0 : (const S *)H->f[l];
            fl[l] = fz && l < L && (1 << (H->lg - l)) >= fmin && (1 << (H->lg - l)) <= fmax;
        }
        int tl = 0;  // level handed to the one-workgroup tail (0 = none)
        if (g_tune.tail && o.nu1 >= 1)
            for (int l = 1; l <= L; ++l)
                if (H->lg - l <= Tail<D>::LG && H->lg - l > 2 && !fl[l]) { tl = l; break; }
        // the check of level 0's partials: by the tail kernel where there is one and the level-0
        // down-leg writes only the partner buffer (safe): the tail then comes before every launch
        // that writes x0, and the levels between touch neither x0 nor the partials; else by a
        // launch of its own
        const bool defer = tl > 0 && !hook && g_tune.tailck;
        int pend = -1;
        auto check_now = [&](int nb, bool safe = true) -> np_status {
            if (defer && safe) {
                pend = nb;
                return NP_OK;
            }
            hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, nb, H->ctl);
            NP_LAUNCH_CHECK();
            return NP_OK;
        };
        double hl = h;
        // ------------------------------------------------------------ down
        for (int l = 0; l < L; ++l, hl *= 2.0) {
            const int lg = H->lg - l;
            bool zero = l > 0 || zero0;
            if (hook && l > 0 && l == hook->level && !fl[l]) {
                bool used = false;
                NP_TRY(hook->fn(F[l], cur[l], hl, s, &used));
                if (used) zero = false;
            }
            S *fc = (S *)H->f[l + 1];
            if (fl[l]) {
                int nb = 0;
                if (zero) {
                    NP_TRY((fused<1, PRE_ZERO, true, false>(nullptr, F[l], oth[l], nullptr, fc, nullptr, lg, bc, hl,
                                                            o.omega, s, stop, l == 0, &nb)));
                } else if (check && l == 0) {
                    NP_TRY((fused<2, PRE_NONE, true, true>(cur[l], F[l], oth[l], nullptr, fc, H->red, lg, bc, hl,
                                                           o.omega, s, stop, true, &nb)));
                    NP_TRY(check_now(nb));
                } else {
                    NP_TRY((fused<2, PRE_NONE, true, false>(cur[l], F[l], oth[l], nullptr, fc, nullptr, lg, bc, hl,
                                                            o.omega, s, stop, l == 0, &nb)));
                }
                std::swap(cur[l], oth[l]);  // the smoothed iterate is in the partner buffer
                continue;
            }
            if (o.nu1 == 2 && blk2_on(lg) && (!zero || g_tune.zero2)) {
                // 2D: both pre-sweeps, the residual and the restriction in one block kernel; from zero
                // on level 0 into the partner buffer, so that the one-pass up-leg ends in the caller's x
                if (zero) {
                    S *dst = l == 0 ? oth[0] : cur[l];
                    NP_TRY((lvl2b<0, false>(nullptr, F[l], nullptr, dst, fc, nullptr, nullptr, lg, bc, hl, o.omega, s,
                                            stop)));
                    if (l == 0) std::swap(cur[0], oth[0]);
                } else if (check && l == 0) {
                    int nb = 0;
                    NP_TRY((lvl2b<1, true>(nullptr, F[l], cur[l], oth[l], fc, H->red, &nb, lg, bc, hl, o.omega, s,
                                           stop)));
                    NP_TRY(check_now(nb));
                    std::swap(cur[l], oth[l]);
                } else {
                    NP_TRY((lvl2b<1, false>(nullptr, F[l], cur[l], oth[l], fc, nullptr, nullptr, lg, bc, hl, o.omega,
                                            s, stop)));
                    std::swap(cur[l], oth[l]);
                }
                if (l + 1 == tl) { hl *= 2.0; break; }
                continue;
            }
            if (zero && o.nu1 == 2 && g_tune.zero2 && (fuseb_on(lg) || z2_on(lg))) {
                // both pre-sweeps from zero, the residual and the restriction in one pass; on level 0
                // into the partner buffer, so that the one-pass up-leg ends in the caller's x
                S *dst = l == 0 ? oth[0] : cur[l];
                if (fuseb_on(lg)) NP_TRY(down0b(F[l], dst, fc, lg, bc, hl, o.omega, s, l == 0, stop));
                else NP_TRY(down0z(F[l], dst, fc, lg, bc, hl, o.omega, s, l == 0, stop));
                if (l == 0) std::swap(cur[0], oth[0]);
                if (l + 1 == tl) { hl *= 2.0; break; }
                continue;
            }
            bool zf = zero;
            if (zf && o.nu1 == 0) {
                hipLaunchKernelGGL((k_zero<S>), dim3(blocks_for(cells(D, lg))), dim3(kBlock), 0, s, cur[l],
                                   cells(D, lg), stop);
                NP_LAUNCH_CHECK();
                zf = false;
            }
            if (check && l == 0 && !zero && o.nu1 == 0) {
                int nb = 0;
                NP_TRY(resid_sq(F[0], cur[0], lg, bc, hl, H->red, s, stop, &nb));
                NP_TRY(check_now(nb));
            }
            if (!zf && o.nu1 == 2 && z2_on(lg)) {
                // both pre-sweeps in one pass (with the residual check of the input iterate on level 0),
                // in FP32 and FP64 with the residual and the restriction in the same pass
                const bool ck = check && l == 0 && !zero;
                int nb = 0;
                if (down2_on(lg)) {
                    NP_TRY(down2z(F[l], cur[l], oth[l], fc, ck ? H->red : nullptr, &nb, lg, bc, hl, o.omega, s, l == 0,
                                  stop));
                } else {
                    NP_TRY(sweep2z(nullptr, F[l], cur[l], oth[l], ck ? H->red : nullptr, &nb, lg, bc, hl, o.omega, s,
                                   l == 0, stop));
                }
                if (ck) NP_TRY(check_now(nb));
                std::swap(cur[l], oth[l]);
                if (!down2_on(lg)) NP_TRY(restrict_(F[l], cur[l], fc, lg, bc, hl, s, stop));
                if (l + 1 == tl) { hl *= 2.0; break; }
                continue;
            }
            for (int it = 0; it < o.nu1; ++it) {
                const bool ck = check && l == 0 && !zero && it == 0;  // residual of the input iterate
                // from a zero iterate: the first two sweeps in one pass where there are two
                const int zm = zf && it == 0 ? (o.nu1 >= 2 && g_tune.zero2 ? 2 : 1) : 0;
                int nb = 0;
                // a sweep from a zero iterate reads no iterate: it writes in place, which saves the
                // copy back into the caller's buffer at the end of the cycle -- on level 0 into the
                // partner buffer when the one-pass up-leg (which ends in the other buffer) follows
                const bool zpart = zm && l == 0 && o.nu2 == 2 && z2_on(lg) && psweep_on(lg, o.nu2);
                NP_TRY(sweep(F[l], zm ? nullptr : cur[l], zm && !zpart ? cur[l] : oth[l], lg, bc, hl, o.omega, zm,
                             ck ? H->red : nullptr, &nb, s, l == 0, stop));
                if (ck) NP_TRY(check_now(nb, o.nu1 == 1));  // a second sweep would write x0 back
                if (!zm || zpart) std::swap(cur[l], oth[l]);
                if (zm == 2) ++it;
            }
            NP_TRY(restrict_(F[l], cur[l], fc, lg, bc, hl, s, stop));
            if (l + 1 == tl) { hl *= 2.0; break; }
        }
        if (tl > 0) {
            // levels tl .. L in one workgroup; hl is the spacing of level tl
            hl = h * double(int64_t(1) << tl);
            if (pend >= 0)  // with the check of level 0's partials
                NP_TRY(tail(F[tl], cur[tl], H->Minv, H->lg - tl, bc, hl, o, s, stop, H->red, pend, H->ctl));
            else
                NP_TRY(tail(F[tl], cur[tl], H->Minv, H->lg - tl, bc, hl, o, s, stop));
            res[tl] = cur[tl];
        } else {
            // coarsest level: exact solve (zero guess unless the whole grid is 4^d)
            if (L == 0 && check && !zero0) {
                int nb = 0;
                NP_TRY(resid_sq(F[0], cur[0], H->lg, bc, hl, H->red, s, stop, &nb));
                hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, nb, H->ctl);
                NP_LAUNCH_CHECK();
            }
            NP_TRY(coarse(F[L], cur[L], H->Minv, bc, hl, L > 0 || zero0, s, stop));
            res[L] = cur[L];
        }
        // -------------------------------------------------------------- up
        for (int l = (tl > 0 ? tl : L) - 1; l >= 0; --l) {
            hl *= 0.5;
            const int lg = H->lg - l;
            if (fl[l]) {
                // pre-smoothed iterate in cur[l]; result into the other buffer
                NP_TRY((fused<2, PRE_PROLONG, false, false>(cur[l], F[l], oth[l], res[l + 1], nullptr, nullptr, lg,
                                                            bc, hl, o.omega, s, stop, l == 0, nullptr)));
                std::swap(cur[l], oth[l]);
                res[l] = cur[l];
                continue;
            }
            int it = 0;
            // prolongation + correction and both post-sweeps in one pass (on level 0 only when the
            // result lands in the caller's x)
            if (o.nu2 == 2 && fuseb_on(lg) && psweep_on(lg, o.nu2) && (l > 0 || cur[0] != x0)) {
                NP_TRY(up2b(res[l + 1], F[l], cur[l], oth[l], lg, bc, hl, o.omega, s, l == 0, stop));
                std::swap(cur[l], oth[l]);
                it = 2;
            } else if (o.nu2 == 2 && blk2_on(lg) && psweep_on(lg, o.nu2) && (l > 0 || cur[0] != x0)) {
                NP_TRY((lvl2b<2, false>(res[l + 1], F[l], cur[l], oth[l], nullptr, nullptr, nullptr, lg, bc, hl, o.omega,
                                        s, stop)));
                std::swap(cur[l], oth[l]);
                it = 2;
            } else if (o.nu2 == 2 && z2_on(lg) && psweep_on(lg, o.nu2) && (l > 0 || cur[0] != x0)) {
                NP_TRY(sweep2z(res[l + 1], F[l], cur[l], oth[l], nullptr, nullptr, lg, bc, hl, o.omega, s, l == 0,
                               stop));
                std::swap(cur[l], oth[l]);
                it = 2;
            } else if (psweep_on(lg, o.nu2)) {
                NP_TRY(psweep(res[l + 1], F[l], cur[l], oth[l], lg, bc, hl, o.omega, s, l == 0, stop));
                std::swap(cur[l], oth[l]);
                it = 1;
            } else {
                NP_TRY(prolong_add(res[l + 1], cur[l], lg - 1, bc, s, stop));
            }
            for (; it < o.nu2; ++it) {
                NP_TRY(sweep(F[l], cur[l], oth[l], lg, bc, hl, o.omega, 0, nullptr, nullptr, s, l == 0, stop));
                std::swap(cur[l], oth[l]);
            }
            res[l] = cur[l];
        }
        if (res[0] != x0) {
            hipLaunchKernelGGL((k_copy<S>), dim3(blocks_for(cells(D, H->lg))), dim3(kBlock), 0, s, res[0], x0,
                               cells(D, H->lg), stop);
            NP_LAUNCH_CHECK();
        }
        return NP_OK;
    }
};

// --------------------------------------------------------- graph replay
// Captures `enqueue` into a graph on the hierarchy's capture stream (cached by
// key) and launches it on s; without graphs, enqueues directly on s.
template <class F>
static np_status run_graph(Hier *H, const GraphKey &key, hipStream_t s, F enqueue) {
    // timed runs bracket individual launches with events: no graphs then
    if (!g_tune.graphs || prof_on() || H->direct) return enqueue(s);
    for (auto &g : H->graphs)
        if (g.key == key) {
            g.used = ++H->tick;
            NP_HIP_TRY(hipGraphLaunch(g.exec, s));
            return NP_OK;
        }
    NP_HIP_TRY(hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal));
    np_status st = enqueue(H->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(H->cap, &graph);
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
    if (H->graphs.size() >= 32) {  // evict the least recently used
        size_t v = 0;
        for (size_t i = 1; i < H->graphs.size(); ++i)
            if (H->graphs[i].used < H->graphs[v].used) v = i;
        // the evicted graph may have been launched earlier in this call: it is
        // destroyed only once the stream has finished every launch before it
        NP_HIP_TRY(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(H->graphs[v].exec);
        H->graphs.erase(H->graphs.begin() + v);
    }
    H->graphs.push_back(GraphEntry{key, exec, ++H->tick});
    NP_HIP_TRY(hipGraphLaunch(exec, s));
    return NP_OK;
}

// count repetitions of enqueue(q, j), j = j0, j0 + 1, ..., as graphs of 8, 4, 2 and 1 of them
// (key.reps tells them apart): the stream leaves a gap of several microseconds between
// consecutive graph launches, which a graph of several cycles pays once.  parity: what
// enqueue does depends on the parity of j, and key.par holds that of each graph's first j.
template <class F>
static np_status run_graphs(Hier *H, GraphKey key, hipStream_t s, int count, int j0, bool parity, F enqueue) {
    while (count > 0) {
        const int g = g_tune.greps;
        const int r = count >= 8 && g >= 8 ? 8 : count >= 4 && g >= 4 ? 4 : count >= 2 && g >= 2 ? 2 : 1;
        key.reps = r;
        key.par = parity ? (j0 & 1) : 0;
        NP_TRY(run_graph(H, key, s, [&](hipStream_t q) -> np_status {
            for (int i = 0; i < r; ++i) NP_TRY(enqueue(q, j0 + i));
            return NP_OK;
        }));
        count -= r;
        j0 += r;
    }
    return NP_OK;
}

// --------------------------------------------------------- solve helpers
static np_status read_scalars(Hier *H, int count, hipStream_t s) {
    NP_HIP_TRY(hipMemcpyAsync(H->hred, H->red + kPartials, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

static np_status read_ctl(Hier *H, hipStream_t s) {
    NP_HIP_TRY(hipMemcpyAsync(H->hctl, H->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// Sum (square = 0) or squared norm (square = 1) of an FP64 field into red slot.
static np_status dsum(Hier *H, const double *v, int64_t m, int square, int slot, hipStream_t s) {
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
    hipLaunchKernelGGL((k_sum<double>), dim3(nb), dim3(kBlock), 0, s, v, m, square, H->red);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->red + kPartials + slot,
                       square);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

static np_status remove_mean(Hier *H, double *v, int64_t m, hipStream_t s) {
    NP_TRY(dsum(H, v, m, 0, 7, s));
    hipLaunchKernelGGL(k_sub_scaled, dim3(blocks_for(m)), dim3(kBlock), 0, s, v, m, H->red + kPartials + 7,
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

// Initialises the device controller (k done, history entry 0 if known) with a
// kernel on the stream: its arguments carry the values, so no host buffer has
// to outlive the call and the host does not wait.
static np_status init_ctl(Hier *H, const np_mg_opts &o, double nf, double tol, int k0, double h0, hipStream_t s) {
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(kBlock), 0, s, H->ctl, k0, o.fixed_cycles, o.max_cycles, nf, tol,
                       h0);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// Host-side stop rule for the iterate known before any cycle (rr = 1 for a zero
// guess); returns true when no cycle may run.
static bool stop_before_first(const np_mg_opts &o, double tol, np_status *st) {
    *st = NP_OK;
    if (o.fixed_cycles > 0) return false;
    if (1.0 <= tol) return true;
    if (o.max_cycles <= 0) {
        set_error("tolerance %.3g not reached in 0 cycles", tol);
        *st = NP_ENOCONV;
        return true;
    }
    return false;
}

static np_status status_of(const Ctl &c, double tol) {
    switch (c.stop) {
    case kConverged:
    case kFixedDone: return NP_OK;
    case kNonFinite: set_error("non-finite residual norm after %d cycles", c.k); return NP_ENAN;
    case kDiverged: set_error("residual grew in three consecutive cycles (cycle %d)", c.k); return NP_ENOCONV;
    default:
        set_error("tolerance %.3g not reached in %d cycles (rel_res %.3g)", tol, c.k,
                  c.nhist > 0 ? c.hist[c.nhist - 1] : -1.0);
        return NP_ENOCONV;
    }
}

static void fill_stats(np_mg_stats *st, const Ctl &c, int cycles, int outer) {
    if (!st) return;
    st->cycles = cycles;
    st->outer_iters = outer;
    const int n = c.nhist;
    for (int i = 0; i < n && i < 256; ++i) st->hist[i] = c.hist[i];
    st->rel_res = n > 0 ? c.hist[n - 1] : 0.0;
    st->rho_est = (n > 1 && c.hist[0] > 0.0 && c.hist[n - 1] > 0.0)
                      ? std::pow(c.hist[n - 1] / c.hist[0], 1.0 / (n - 1)) : 0.0;
}

// How many more cycles (or refinement steps) to enqueue before reading the
// controller again: the steps the last contraction factor predicts down to
// tol, plus `tail` when the check of the last one runs only at the start of
// the next (check_last = false).  An under-estimate costs one host round
// trip; an over-estimate enqueues steps that run as no-ops.
static int next_batch(const Ctl &c, const np_mg_opts &o, bool check_last) {
    const int tail = check_last ? 0 : 1;
    if (o.fixed_cycles > 0) return std::max(1, o.fixed_cycles - c.k + tail);
    const int n = c.nhist;
    if (n < 2 || !(c.hist[n - 1] > 0.0) || !(c.hist[n - 2] > 0.0)) return g_tune.batch;
    double rho = c.hist[n - 1] / c.hist[n - 2];
    rho = std::min(0.95, std::max(0.02, rho));
    const double need = std::log(c.tol / c.hist[n - 1]) / std::log(rho);
    int b = int(std::ceil(need)) + tail;
    return std::max(1, std::min(b, 32));
}

template <int D>
static np_status solve_fp64(Hier *H, const double *f, double *x, double h, double tol, const np_mg_opts &o,
                            const CycleOpts &co, hipStream_t s, bool x_zero, double nf, np_mg_stats *stats) {
    typedef Ops<D, double> O;
    NP_TRY(ensure_levels(H));
    double *t0 = (double *)H->t[0];
    np_status st0;
    if (x_zero && stop_before_first(o, tol, &st0)) {
        Ctl c{};
        c.nhist = 1;
        c.hist[0] = 1.0;
        fill_stats(stats, c, 0, 0);
        return st0;
    }
    NP_TRY(init_ctl(H, o, nf, tol, x_zero ? 1 : 0, 1.0, s));
    // learned coarse-grid correction in the first o.cnn_cgc cycles: the coarse
    // problem on the attached network's grid starts from the network's
    // prediction, kept only if it lowers that level's energy-norm error
    // (2 e'r - e'A e > 0); these cycles are enqueued directly (the network
    // reads norms on the host)
    CgcHook hook;
    int cgc = 0, accepted = 0;
    if constexpr (D == 3) {
        const int lnet = H->lg - cnn_attached_lg();
        if (o.cnn_cgc > 0 && cnn_attached_lg() >= 0 && lnet >= 1 && lnet < H->L) {
            cgc = o.cnn_cgc;
            hook.level = lnet;
            hook.fn = [&](const void *fl, void *xl, double hl, hipStream_t q, bool *used) -> np_status {
                const int lgl = H->lg - lnet;
                NP_TRY(cnn_coarse_guess(lgl, (const double *)fl, (double *)xl, q, used));
                if (!*used) return NP_OK;
                int nb = 0;
                NP_TRY(O::energy((const double *)fl, (const double *)xl, lgl, H->bc, hl, H->red, q, &nb));
                hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, q, H->red, nb, H->red + kPartials, 0);
                NP_LAUNCH_CHECK();
                NP_TRY(read_scalars(H, 1, q));
                if (!(H->hred[0] > 0.0)) {
                    *used = false;
                    return NP_OK;
                }
                ++accepted;
                return NP_OK;
            };
        }
    }
    if (x_zero) {
        if (cgc > 0) {
            NP_TRY(O::cycle(H, x, f, t0, true, false, h, co, s, &hook));
            --cgc;
        } else {
            GraphKey k0{0, 1, 0, x, f, h, co.nu1, co.nu2, 0, co.omega};
            NP_TRY(run_graph(H, k0, s, [&](hipStream_t q) { return O::cycle(H, x, f, t0, true, false, h, co, q); }));
        }
    }
    for (; cgc > 0; --cgc) {
        NP_TRY(O::cycle(H, x, f, t0, false, true, h, co, s, &hook));
        NP_TRY(read_ctl(H, s));
        if (H->hctl->stop) break;
    }
    GraphKey key{0, 0, 1, x, f, h, co.nu1, co.nu2, 0, co.omega};
    int batch = o.fixed_cycles > 0 ? o.fixed_cycles + 1 : g_tune.batch;
    for (;;) {
        NP_TRY(run_graphs(H, key, s, batch, 0, false,
                          [&](hipStream_t q, int) { return O::cycle(H, x, f, t0, false, true, h, co, q); }));
        NP_TRY(read_ctl(H, s));
        if (H->hctl->stop) break;
        batch = next_batch(*H->hctl, o, false);
    }
    const Ctl c = *H->hctl;
    fill_stats(stats, c, c.k, c.k);
    if (stats) stats->cgc_accepted = accepted;
    return status_of(c, tol);
}

// One sawtooth cycle (Section 2.2; Appendix B), FP64, every launch gated by the
// controller: the finest residual (its norm is the convergence check), the
// residual restricted level by level to the coarsest grid, then on each level
// from the coarsest up e = r / A_00 + P e_coarse followed by nu2 relaxed-Jacobi
// steps (alpha = omega) on that level's residual equation, and x += e_0.
// Buffers: r_0 in t[0], r_l in f[l]; e_0 and its partner in `saw`, e_l and
// its partner in x[l], t[l].
template <int D>
static np_status saw_cycle(Hier *H, const double *f, double *x, double h, const np_mg_opts &o, hipStream_t s) {
    const int L = H->L, bc = H->bc, lg0 = H->lg;
    const int *stop = &H->ctl->stop;
    const int64_t m0 = cells(D, lg0);
    std::vector<double *> r(L + 1), e(L + 1), t(L + 1);
    for (int l = 0; l <= L; ++l) {
        r[l] = l == 0 ? (double *)H->t[0] : (double *)H->f[l];
        e[l] = l == 0 ? H->saw : (double *)H->x[l];
        t[l] = l == 0 ? H->saw + m0 : (double *)H->t[l];
    }
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m0));
    hipLaunchKernelGGL((k_saw_resid<D>), dim3(nb), dim3(kBlock), 0, s, f, x, r[0], H->red, lg0, bc, 1.0 / (h * h),
                       stop);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->ctl);
    NP_LAUNCH_CHECK();
    for (int l = 0; l < L; ++l) {
        const int lgc = lg0 - l - 1;
        hipLaunchKernelGGL((k_restrict_field<D>), dim3(blocks_for(cells(D, lgc))), dim3(kBlock), 0, s, r[l],
                           r[l + 1], lgc, stop);
        NP_LAUNCH_CHECK();
    }
    std::vector<double *> done(L + 2, nullptr);  // final correction of each level
    for (int l = L; l >= 0; --l) {
        const int lg = lg0 - l;
        const int64_t ml = cells(D, lg);
        const double hl = h * double(int64_t(1) << l);
        hipLaunchKernelGGL((k_saw_up<D>), dim3(blocks_for(ml)), dim3(kBlock), 0, s, r[l], done[l + 1], e[l], lg,
                           bc, hl * hl / (2.0 * D), o.prolong, stop);
        NP_LAUNCH_CHECK();
        double *cur = e[l], *oth = t[l];
        for (int it = 0; it < o.nu2; ++it) {
            hipLaunchKernelGGL((k_jacobi<D, double, false>), dim3(blocks_for(ml)), dim3(kBlock), 0, s, r[l], cur,
                               oth, lg, bc, 1.0 / (hl * hl), o.omega * hl * hl / (2.0 * D), stop);
            NP_LAUNCH_CHECK();
            std::swap(cur, oth);
        }
        done[l] = cur;
    }
    hipLaunchKernelGGL(k_add_to, dim3(blocks_for(m0)), dim3(kBlock), 0, s, x, done[0], m0, stop);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// Tolerance driver of the sawtooth cycle (the check opens every cycle).
template <int D>
static np_status solve_saw(Hier *H, const double *f, double *x, double h, double tol, const np_mg_opts &o,
                           hipStream_t s, double nf, np_mg_stats *stats) {
    NP_TRY(ensure_levels(H));
    if (!H->saw) NP_TRY(dmalloc((void **)&H->saw, sizeof(double) * 2 * cells(D, H->lg)));
    NP_TRY(init_ctl(H, o, nf, tol, 0, 0.0, s));
    GraphKey key{5, o.prolong, 1, x, f, h, 0, o.nu2, 0, o.omega};
    int batch = o.fixed_cycles > 0 ? o.fixed_cycles + 1 : g_tune.batch;
    for (;;) {
        NP_TRY(run_graphs(H, key, s, batch, 0, false,
                          [&](hipStream_t q, int) { return saw_cycle<D>(H, f, x, h, o, q); }));
        NP_TRY(read_ctl(H, s));
        if (H->hctl->stop) break;
        batch = next_batch(*H->hctl, o, false);
    }
    const Ctl c = *H->hctl;
    fill_stats(stats, c, c.k, c.k);
    return status_of(c, tol);
}

template <int D, class SL>
// part0 (np0 partials of |f|^2, with f already rounded into the low-precision
// right-hand side): the solve starts from a zero iterate that x does not hold --
// the first check reads those partials, and the first update reads no iterate.
static np_status solve_mixed(Hier *H, const double *f, double *x, double h, double tol, const np_mg_opts &o,
                             const CycleOpts &co, hipStream_t s, double nf, bool warm, np_mg_stats *stats,
                             const double *part0 = nullptr, int np0 = 0) {
    typedef Ops<D, SL> O;
    NP_TRY(ensure_levels(H));
    const int64_t m = cells(D, H->lg);
    const int inner = o.inner_cycles > 0 ? o.inner_cycles
                                         : (H->prec == NP_BF16 ? g_tune.inner_bf16 : g_tune.inner_fp32);
    SL *e = (SL *)H->x[0], *rlo = (SL *)H->f[0], *tt = (SL *)H->t[0];
    double *xa = x, *xb = H->x64;
    const bool zm = D == 3 && H->lg >= 7 && g_tune.sweep3;  // z-marching refinement kernel
    const int icpt = g_tune.ir_cpt;                           // its cells per thread (1 or 2)
    const bool cold = part0 && zm && icpt == 2;               // zero iterate, not held in x
    if (part0 && !cold) {  // the kernels below read the zero iterate from x
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
        NP_LAUNCH_CHECK();
    }
    np_status st0;
    if (!warm && stop_before_first(o, tol, &st0)) {
        if (cold) {  // the result is the zero iterate
            hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
            NP_LAUNCH_CHECK();
        }
        Ctl c{};
        c.nhist = 1;
        c.hist[0] = 1.0;
        fill_stats(stats, c, 0, 0);
        return st0;
    }
    NP_TRY(init_ctl(H, o, nf, tol, 0, 0.0, s));
    const int zc = zm ? sweep3_planes(H->lg, icpt, kPartials) : 0;
    const unsigned nb = zm ? zblocks(H->lg, icpt, zc)
                           : unsigned(std::min<int64_t>((m + kIrCells - 1) / kIrCells, kPartials));
    const int *stop = &H->ctl->stop;
    // one refinement step: x_out = x_in + e (step > 0), r = f - A x_out, check, inner cycles;
    // xz: x_in is zero and not read
    auto step = [&](hipStream_t q, const double *xin, double *xout, int has_e, bool xz = false) -> np_status {
        void *tok = nullptr;
        const bool prof = prof_on() & kProfRefine;
        if (prof) NP_TRY(prof_begin(q, &tok));
        if (xz)
            hipLaunchKernelGGL((k_ir_resid3<SL, true, 2, true>), dim3(nb), dim3(kS3Threads), 0, q, nullptr, e, xout,
                               f, rlo, H->red, H->lg, H->bc, zc, 1.0 / (h * h), stop);
        else if (zm && has_e && icpt == 2)
            hipLaunchKernelGGL((k_ir_resid3<SL, true, 2>), dim3(nb), dim3(kS3Threads), 0, q, xin, e, xout, f, rlo,
                               H->red, H->lg, H->bc, zc, 1.0 / (h * h), stop);
        else if (zm && icpt == 2)
            hipLaunchKernelGGL((k_ir_resid3<SL, false, 2>), dim3(nb), dim3(kS3Threads), 0, q, xin, e, xout, f,
                               rlo, H->red, H->lg, H->bc, zc, 1.0 / (h * h), stop);
        else if (zm && has_e)
            hipLaunchKernelGGL((k_ir_resid3<SL, true>), dim3(nb), dim3(kS3Threads), 0, q, xin, e, xout, f, rlo,
                               H->red, H->lg, H->bc, zc, 1.0 / (h * h), stop);
        else if (zm)
            hipLaunchKernelGGL((k_ir_resid3<SL, false>), dim3(nb), dim3(kS3Threads), 0, q, xin, e, xout, f, rlo,
                               H->red, H->lg, H->bc, zc, 1.0 / (h * h), stop);
        else
            hipLaunchKernelGGL((k_ir_resid<D, SL>), dim3(nb), dim3(kBlock), 0, q, xin, e, xout, f, rlo, H->red,
                               H->lg, H->bc, 1.0 / (h * h), has_e, stop);
        NP_LAUNCH_CHECK();
        if (prof)
            NP_TRY(prof_end(q, tok, double(m) * (has_e ? (xz ? 0 : 8) + sizeof(SL) + 8 + 8 + sizeof(SL)
                                                        : 8 + 8 + sizeof(SL))));
        hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, q, H->red, int(nb), H->ctl);
        NP_LAUNCH_CHECK();
        return NP_OK;
    };
    // the inner cycles of one step: e from the rounded residual
    auto cycles = [&](hipStream_t q) -> np_status {
        for (int c = 0; c < inner; ++c) NP_TRY(O::cycle(H, e, rlo, tt, c == 0, false, h, co, q));
        return NP_OK;
    };
    // graphs: the first update (x = x0); outer steps j = 1, 2, ...: the inner cycles, then
    // the update a -> b (j odd) or b -> a (j even), several steps to a graph; every batch
    // ends with an update and its check, so that a converged solve enqueues no further cycles
    GraphKey k1{cold ? 8 : 1, 0, 0, xa, f, h, co.nu1, co.nu2, inner, co.omega};
    GraphKey ks{2, 0, 0, xa, f, h, co.nu1, co.nu2, inner, co.omega};
    GraphKey k0a{9, 0, 0, xa, f, h, co.nu1, co.nu2, inner, co.omega};
    auto outer = [&](hipStream_t q, int j) -> np_status {
        NP_TRY(cycles(q));
        if (j == 1 && cold) return step(q, nullptr, xb, 1, true);
        return (j & 1) ? step(q, xa, xb, 1) : step(q, xb, xa, 1);
    };
    if (cold) {
        // r = f is already rounded into r_lo; its check reads the norm's partials
        NP_TRY(run_graph(H, k1, s, [&](hipStream_t q) -> np_status {
            hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, q, part0, np0, H->ctl);
            NP_LAUNCH_CHECK();
            return NP_OK;
        }));
    } else {
        NP_TRY(run_graph(H, k1, s, [&](hipStream_t q) { return step(q, xa, nullptr, 0); }));
    }
    int launched = 1;
    int batch = o.fixed_cycles > 0 ? o.fixed_cycles : std::max(1, g_tune.batch / 2);
    for (;;) {
        int b = batch;
        if (launched == 1 && cold) {  // the first update, from a zero x, in a graph of its own
            NP_TRY(run_graphs(H, k0a, s, 1, 1, false, outer));
            --b;
            ++launched;
        }
        NP_TRY(run_graphs(H, ks, s, b, launched, true, outer));
        launched += b;
        NP_TRY(read_ctl(H, s));
        if (H->hctl->stop) break;
        batch = next_batch(*H->hctl, o, true);
    }
    const Ctl c = *H->hctl;
    // stopped at the first check: x never received an update, and the iterate is zero
    if (cold && c.k == 0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
        NP_LAUNCH_CHECK();
    }
    // the iterate whose residual was checked last: x_a after an even number of updates
    if (c.k & 1) NP_HIP_TRY(hipMemcpyAsync(x, xb, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    fill_stats(stats, c, c.k * inner, c.k);
    return status_of(c, tol);
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
    o->cycle = 0;
    o->prolong = 0;
}

extern "C" const char *np_last_error(void) { return g_err.c_str(); }

extern "C" void np_release_all(void) {
    (void)hipDeviceSynchronize();
    release_mg_cache();
    release_ns_cache();
    release_batched_cache();
}

extern "C" void np_prof_enable(int mask) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_recs) {
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    g_prof = mask;
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

extern "C" np_status np_set_tuning(const char *key, int value) {
    clear_error();
    if (!key) { set_error("null key"); return NP_EINVAL; }
    struct { const char *k; int *v; int lo, hi; } tab[] = {
        {"fused", &g_tune.fused, 0, 1},         {"graphs", &g_tune.graphs, 0, 1},
        {"tail", &g_tune.tail, 0, 1},
        {"fmin2", &g_tune.fmin2, 4, 1 << 14},   {"fmin3", &g_tune.fmin3, 4, 1 << 12},
        {"fmax2", &g_tune.fmax2, 4, 1 << 14},   {"fmax3", &g_tune.fmax3, 4, 1 << 12},
        {"bz2", &g_tune.bz2, 0, 1 << 14},       {"bz3", &g_tune.bz3, 0, 1 << 12},
        {"inner_fp32", &g_tune.inner_fp32, 1, 64}, {"inner_bf16", &g_tune.inner_bf16, 1, 64},
        {"batch", &g_tune.batch, 1, 64},        {"sweep3", &g_tune.sweep3, 0, 1},
        {"zero2", &g_tune.zero2, 0, 1},         {"psweep", &g_tune.psweep, 0, 1},
        {"ir_cpt", &g_tune.ir_cpt, 1, 2},      {"fuseb", &g_tune.fuseb, 0, 1}, {"fbnt", &g_tune.fbnt, 512, 1024},  {"sweep2z", &g_tune.sweep2z, 0, 1}, {"down2z", &g_tune.down2z, 0, 1}, {"blk2", &g_tune.blk2, 0, 1}, {"z2wg", &g_tune.z2wg, 0, 1}, {"greps", &g_tune.greps, 1, 8}, {"tailck", &g_tune.tailck, 0, 1}, {"zbar", &g_tune.zbar, 1, 2}, {"d2cpt", &g_tune.d2cpt, 1, 2}, {"d2wg", &g_tune.d2wg, 0, 1024},
        {"fbmax", &g_tune.fbmax, 5, 10},
        {"batched_graphs", &g_batched_graphs, 0, 1}, {"batched_autotune", &g_batched_autotune, 0, 1},
        {"batched_rm", &g_batched_rm, 0, 1},    {"batched_wg", &g_batched_wg, 64, 1 << 20},
        {"zmarch_explicit", &g_zmarch_explicit, 0, 1}, {"mom_rows", &g_mom_rows, 4, 8}, {"mom_ring", &g_mom_ring, 2, 3}, {"zc3", &g_zc3, 0, 64}, {"conv3z", &g_conv3z, 0, 64},
        {"wgrad_mfma", &g_wgrad_mfma, 0, 1},
    };
    for (auto &e : tab)
        if (std::strcmp(e.k, key) == 0) {
            if (value < e.lo || value > e.hi || ((e.v == &g_tune.bz2 || e.v == &g_tune.bz3) && (value & 1)) ||
                (e.v == &g_zc3 && value != 0 && (value < 2 || (value & (value - 1)))) ||
                (e.v == &g_mom_rows && value != 4 && value != 8) ||
                (e.v == &g_tune.fbnt && value != 512 && value != 1024) ||
                (e.v == &g_tune.d2wg && value != 0 && value != 256 && value != 512 && value != 1024) ||
                (e.v == &g_tune.greps && (value & (value - 1))) ||
                (e.v == &g_conv3z && value > 1 && (value & (value - 1)))) {
                set_error("value %d out of range for %s", value, key);
                return NP_EINVAL;
            }
            *e.v = value;
            // cached graphs bake launch shapes in: drop them
            std::lock_guard<std::mutex> lk(g_cache_mu);
            for (auto &kv : g_cache) {
                std::lock_guard<std::mutex> l2(kv.second->mu);
                drop_graphs(kv.second);
            }
            return NP_OK;
        }
    set_error("unknown tuning key '%s'", key);
    return NP_EINVAL;
}

extern "C" int np_get_tuning(const char *key) {
    if (!key) return -1;
    if (!std::strcmp(key, "fused")) return g_tune.fused;
    if (!std::strcmp(key, "graphs")) return g_tune.graphs;
    if (!std::strcmp(key, "tail")) return g_tune.tail;
    if (!std::strcmp(key, "fmin2")) return g_tune.fmin2;
    if (!std::strcmp(key, "fmin3")) return g_tune.fmin3;
    if (!std::strcmp(key, "fmax2")) return g_tune.fmax2;
    if (!std::strcmp(key, "fmax3")) return g_tune.fmax3;
    if (!std::strcmp(key, "bz2")) return g_tune.bz2;
    if (!std::strcmp(key, "bz3")) return g_tune.bz3;
    if (!std::strcmp(key, "inner_fp32")) return g_tune.inner_fp32;
    if (!std::strcmp(key, "inner_bf16")) return g_tune.inner_bf16;
    if (!std::strcmp(key, "batch")) return g_tune.batch;
    if (!std::strcmp(key, "sweep3")) return g_tune.sweep3;
    if (!std::strcmp(key, "zero2")) return g_tune.zero2;
    if (!std::strcmp(key, "psweep")) return g_tune.psweep;
    if (!std::strcmp(key, "ir_cpt")) return g_tune.ir_cpt;
    if (!std::strcmp(key, "fuseb")) return g_tune.fuseb;
    if (!std::strcmp(key, "fbnt")) return g_tune.fbnt;
    if (!std::strcmp(key, "sweep2z")) return g_tune.sweep2z;
    if (!std::strcmp(key, "down2z")) return g_tune.down2z;
    if (!std::strcmp(key, "blk2")) return g_tune.blk2;
    if (!std::strcmp(key, "z2wg")) return g_tune.z2wg;
    if (!std::strcmp(key, "greps")) return g_tune.greps;
    if (!std::strcmp(key, "tailck")) return g_tune.tailck;
    if (!std::strcmp(key, "zbar")) return g_tune.zbar;
    if (!std::strcmp(key, "d2cpt")) return g_tune.d2cpt;
    if (!std::strcmp(key, "d2wg")) return g_tune.d2wg;
    if (!std::strcmp(key, "fbmax")) return g_tune.fbmax;
    if (!std::strcmp(key, "batched_graphs")) return g_batched_graphs;
    if (!std::strcmp(key, "batched_autotune")) return g_batched_autotune;
    if (!std::strcmp(key, "batched_rm")) return g_batched_rm;
    if (!std::strcmp(key, "batched_wg")) return g_batched_wg;
    if (!std::strcmp(key, "zmarch_explicit")) return g_zmarch_explicit;
    if (!std::strcmp(key, "mom_rows")) return g_mom_rows;
    if (!std::strcmp(key, "mom_ring")) return g_mom_ring;
    if (!std::strcmp(key, "zc3")) return g_zc3;
    if (!std::strcmp(key, "conv3z")) return g_conv3z;
    if (!std::strcmp(key, "wgrad_mfma")) return g_wgrad_mfma;
    return -1;
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
    if (o.max_cycles < 0 || o.fixed_cycles < 0 || o.inner_cycles < 0 || o.inner_cycles > 64 ||
        o.fixed_cycles > 100000 || o.max_cycles > 100000) {
        set_error("bad cycle counts");
        return NP_EINVAL;
    }
    if (o.smooth_prec != NP_FP64 && o.smooth_prec != NP_FP32 && o.smooth_prec != NP_BF16) {
        set_error("unknown smooth_prec");
        return NP_EINVAL;
    }
    if (o.warm_start != 0 && o.warm_start != 1 && o.warm_start != 2) {
        set_error("warm_start must be 0 (zero), 1 (learned) or 2 (caller x)");
        return NP_EINVAL;
    }
    if (o.cycle != 0 && o.cycle != 1) { set_error("cycle must be 0 (V) or 1 (sawtooth)"); return NP_EINVAL; }
    if (o.prolong != 0 && o.prolong != 1) { set_error("prolong must be 0 (linear) or 1 (copy)"); return NP_EINVAL; }
    if (o.cycle == 0 && o.prolong != 0) {
        set_error("the copying prolongation is available with the sawtooth cycle only");
        return NP_EINVAL;
    }
    if (o.cnn_cgc < 0 || o.cnn_cgc > 256 || (o.cnn_cgc > 0 && (o.smooth_prec != NP_FP64 || o.cycle != 0))) {
        set_error("cnn_cgc must be in [0, 256], with FP64 V-cycles");
        return NP_EINVAL;
    }
    if (o.cycle == 1 && (o.nu1 != 0 || o.smooth_prec != NP_FP64 || o.warm_start == 1)) {
        set_error("the sawtooth cycle runs in FP64 with nu1 = 0 and no learned warm start");
        return NP_EINVAL;
    }
    return NP_OK;
}

namespace np {
np_status cnn_warm_start(int d, int lg, int bc, const double *f, double *x0, const std::vector<void *> &fl,
                         const std::vector<void *> &xl, double *unused, hipStream_t s, bool *used);

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
    Hier *H = nullptr;
    NP_TRY(get_hier(d, lg, bc, NP_FP64, &H));
    Hier *HL = nullptr;
    if (o.smooth_prec != NP_FP64) NP_TRY(get_hier(d, lg, bc, o.smooth_prec, &HL));
    std::lock_guard<std::mutex> lk(H->mu);
    std::unique_lock<std::mutex> lk2;
    if (HL) lk2 = std::unique_lock<std::mutex>(HL->mu);
    const int64_t m = cells(d, lg);
    if (!HL) NP_TRY(ensure_coarse(H, h, s));
    else NP_TRY(ensure_coarse(HL, h, s));
    const double *f = rhs;
    if (bc == NP_BC_PERIODIC) {
        if (!H->f64) NP_TRY(dmalloc((void **)&H->f64, sizeof(double) * m));
        NP_HIP_TRY(hipMemcpyAsync(H->f64, rhs, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        NP_TRY(remove_mean(H, H->f64, m, s));
        f = H->f64;
    }
    // The 3D mixed solve from a zero iterate on z-marching levels (n >= 128): its first
    // residual is f itself, so the norm's pass also rounds f into the low-precision
    // right-hand side, the first check reads the norm's partials, and x is not
    // zeroed (the first update writes it).
    const bool cold = HL && o.warm_start == 0 && o.cycle == 0 && d == 3 && lg >= 7 && g_tune.sweep3 &&
                      g_tune.ir_cpt == 2;
    unsigned np0 = 0;
    if (cold) {
        NP_TRY(ensure_levels(HL));
        np0 = std::min<unsigned>(kRedBlocks, blocks_for(m));
        if (o.smooth_prec == NP_FP32)
            hipLaunchKernelGGL((k_sum_round<float>), dim3(np0), dim3(kBlock), 0, s, f, m, (float *)HL->f[0], H->red);
        else
            hipLaunchKernelGGL((k_sum_round<bf16>), dim3(np0), dim3(kBlock), 0, s, f, m, (bf16 *)HL->f[0], H->red);
        NP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, int(np0), H->red + kPartials, 1);
        NP_LAUNCH_CHECK();
    } else {
        NP_TRY(dsum(H, f, m, 1, 0, s));
    }
    NP_TRY(read_scalars(H, 1, s));
    const double nf = H->hred[0];
    if (!std::isfinite(nf)) {
        set_error("non-finite right-hand side");
        return NP_ENAN;
    }
    bool warm = o.warm_start == 2;
    if (nf == 0.0 || (!warm && !cold)) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
        NP_LAUNCH_CHECK();
    }
    if (nf == 0.0) {
        if (stats) { stats->cycles = 0; stats->rel_res = 0.0; }
        NP_HIP_TRY(hipStreamSynchronize(s));
        return NP_OK;
    }
    int fallback = 0;
    if (o.warm_start == 1) {
        // learned initial guess, accepted only if its energy-norm error is
        // below that of the zero iterate (the residual norm is a poor judge
        // here: the prolongated prediction's high-frequency interpolation
        // error is amplified by A and removed by the first smoothing sweeps)
        NP_TRY(ensure_levels(H));
        bool used = false;
        NP_TRY(cnn_warm_start(d, lg, bc, f, x, H->f, H->x, nullptr, s, &used));
        if (used) {
            if (bc == NP_BC_PERIODIC) NP_TRY(remove_mean(H, x, m, s));
            int nb = 0;
            if (d == 2) NP_TRY((Ops<2, double>::energy(f, x, lg, bc, h, H->red, s, &nb)));
            else NP_TRY((Ops<3, double>::energy(f, x, lg, bc, h, H->red, s, &nb)));
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, nb, H->red + kPartials, 0);
            NP_LAUNCH_CHECK();
            NP_TRY(read_scalars(H, 1, s));
            const double gain = H->hred[0];  // ||x*||_A^2 - ||x - x*||_A^2
            if (!(gain > 0.0)) {
                used = false;
                hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
                NP_LAUNCH_CHECK();
            }
        }
        warm = used;
        fallback = used ? 0 : 1;
    }
    np_status st;
    if (o.cycle == 1) {
        st = d == 2 ? solve_saw<2>(H, f, x, h, tol, o, s, nf, stats)
                    : solve_saw<3>(H, f, x, h, tol, o, s, nf, stats);
    } else if (o.smooth_prec == NP_FP64) {
        st = d == 2 ? solve_fp64<2>(H, f, x, h, tol, o, co, s, !warm, nf, stats)
                    : solve_fp64<3>(H, f, x, h, tol, o, co, s, !warm, nf, stats);
    } else if (o.smooth_prec == NP_FP32) {
        st = d == 2 ? solve_mixed<2, float>(HL, f, x, h, tol, o, co, s, nf, warm, stats)
                    : solve_mixed<3, float>(HL, f, x, h, tol, o, co, s, nf, warm, stats, cold ? H->red : nullptr,
                                            int(np0));
    } else {
        st = d == 2 ? solve_mixed<2, bf16>(HL, f, x, h, tol, o, co, s, nf, warm, stats)
                    : solve_mixed<3, bf16>(HL, f, x, h, tol, o, co, s, nf, warm, stats, cold ? H->red : nullptr,
                                           int(np0));
    }
    if (st == NP_EHIP || st == NP_ENOMEM || st == NP_EINVAL) return st;
    if (stats) stats->used_fallback = fallback;
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

// ------------------------------------------- solve in a static workspace
// mg_poisson_solve_noalloc keeps every buffer of the FP64 solve (controller,
// norm partials, coarsest inverse, level-0 partner and periodic rhs copy, the
// coarse levels) in one statically sized device array, `scratch`, so that a
// call allocates no device memory.  In host code `scratch` names a host-side
// stand-in: its device address is taken with hipGetSymbolAddress once per
// device (with that device current) and only that address is used.
constexpr size_t kScratchBytes = size_t(48) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch;  // device -> its copy of `scratch`

np_status scratch_on(int dev, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
            return NP_EHIP;
        }
        it = g_scratch.emplace(dev, (unsigned char *)p).first;
    }
    *out = it->second;
    return NP_OK;
}

// Carves 256-byte aligned pieces off the workspace (base == nullptr: counts only).
struct Carver {
    unsigned char *base;
    size_t used = 0;
    void *take(size_t bytes) {
        void *p = base ? base + used : nullptr;
        used += (bytes + 255) & ~size_t(255);
        return p;
    }
};

// Lays the FP64 solve's buffers for an n^d grid (n = 2^lg) into the workspace
// at base (nullptr: only the size); returns the bytes needed.
size_t layout_noalloc(Hier &H, unsigned char *base, int d, int lg, int bc) {
    Carver c{base};
    const int L = lg - 2;
    H.ctl = (Ctl *)c.take(sizeof(Ctl));
    H.red = (double *)c.take(sizeof(double) * (kPartials + 8));
    H.Minv = (double *)c.take(sizeof(double) * 64 * 64);
    H.x.assign(L + 1, nullptr);
    H.f.assign(L + 1, nullptr);
    H.t.assign(L + 1, nullptr);
    H.t[0] = c.take(sizeof(double) * size_t(cells(d, lg)));
    H.f64 = bc == NP_BC_PERIODIC ? (double *)c.take(sizeof(double) * size_t(cells(d, lg))) : nullptr;
    for (int l = 1; l <= L; ++l) {
        const size_t bytes = sizeof(double) * size_t(cells(d, lg - l));
        H.x[l] = c.take(bytes);
        H.f[l] = c.take(bytes);
        H.t[l] = c.take(bytes);
    }
    return c.used;
}
}  // namespace

extern "C" np_status mg_poisson_solve_noalloc(np_dims dims, double h, np_bc bc, const double *rhs, double *x,
                                              double tol, const np_mg_opts *opts, np_mg_stats *stats) {
    clear_error();
    np_mg_opts o;
    CycleOpts co;
    fill_opts(opts, co, o);
    int lg = -1;
    NP_TRY(check_solve_args(dims, h, bc, rhs, x, tol, o, &lg));
    if (o.smooth_prec != NP_FP64 || o.cycle != 0 || o.warm_start == 1 || o.cnn_cgc != 0) {
        set_error("the static-workspace solve runs FP64 V-cycles from a zero or caller guess");
        return NP_EINVAL;
    }
    const int d = dims.ndim;
    Hier H;
    const size_t need = layout_noalloc(H, nullptr, d, lg, bc);
    if (need > kScratchBytes) {
        set_error("grid needs %zu bytes of workspace, more than the static %zu", need, kScratchBytes);
        return NP_EINVAL;
    }
    if (stats) std::memset(stats, 0, sizeof *stats);
    int dev = 0;
    NP_HIP_TRY(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    NP_TRY(scratch_on(dev, &base));
    Ctl hctl;
    double hred[8];
    H.dev = dev;
    H.d = d;
    H.lg = lg;
    H.L = lg - 2;
    H.bc = bc;
    H.prec = NP_FP64;
    H.es = sizeof(double);
    H.levels = true;
    H.direct = true;
    H.hctl = &hctl;
    H.hred = hred;
    layout_noalloc(H, base, d, lg, bc);
    hipStream_t s = (hipStream_t)o.stream;
    const int64_t m = cells(d, lg);
    NP_TRY(ensure_coarse(&H, h, s));
    const double *f = rhs;
    if (bc == NP_BC_PERIODIC) {
        NP_HIP_TRY(hipMemcpyAsync(H.f64, rhs, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        NP_TRY(remove_mean(&H, H.f64, m, s));
        f = H.f64;
    }
    NP_TRY(dsum(&H, f, m, 1, 0, s));
    NP_TRY(read_scalars(&H, 1, s));
    const double nf = hred[0];
    if (!std::isfinite(nf)) {
        set_error("non-finite right-hand side");
        return NP_ENAN;
    }
    const bool warm = o.warm_start == 2 && nf != 0.0;
    if (!warm) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
        NP_LAUNCH_CHECK();
    }
    if (nf == 0.0) {
        NP_HIP_TRY(hipStreamSynchronize(s));
        return NP_OK;
    }
    np_status st = d == 2 ? solve_fp64<2>(&H, f, x, h, tol, o, co, s, !warm, nf, stats)
                          : solve_fp64<3>(&H, f, x, h, tol, o, co, s, !warm, nf, stats);
    if (st == NP_EHIP || st == NP_ENOMEM || st == NP_EINVAL) return st;
    if (bc == NP_BC_PERIODIC) NP_TRY(remove_mean(&H, x, m, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return st;
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
        NP_TRY((Ops<2, double>::jacobi(f, x_in, x_out, lg, bc, h, omega, false, s, false, nullptr)));
    else
        NP_TRY((Ops<3, double>::jacobi(f, x_in, x_out, lg, bc, h, omega, false, s, false, nullptr)));
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
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::resid_restrict(f, x, fc, lg, bc, h, s, nullptr)));
    else NP_TRY((Ops<3, double>::resid_restrict(f, x, fc, lg, bc, h, s, nullptr)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

extern "C" np_status np_op_prolong_add(np_dims dims, np_bc bc, const double *ec, double *x, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, 1.0, bc, &lg, false));
    if (lg < 3) { set_error("need n >= 8 to prolongate onto"); return NP_EINVAL; }
    if (!ec || !x) { set_error("null array"); return NP_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::prolong_add(ec, x, lg - 1, bc, s, nullptr)));
    else NP_TRY((Ops<3, double>::prolong_add(ec, x, lg - 1, bc, s, nullptr)));
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
    NP_TRY(ensure_levels(H));
    NP_TRY(ensure_coarse(H, h, s));
    const int zero = 0;
    NP_HIP_TRY(hipMemcpyAsync(&H->ctl->stop, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    if (dims.ndim == 2)
        NP_TRY((Ops<2, double>::cycle(H, x, f, (double *)H->t[0], false, false, h, co, s)));
    else
        NP_TRY((Ops<3, double>::cycle(H, x, f, (double *)H->t[0], false, false, h, co, s)));
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// Back-to-back launches of a level kernel the solver uses on this grid (same
// kernel and launch shape) between two events on the stream.  kind 0: the
// sweep y = sweep(x); 1: the residual restriction y = R (f - A x), y coarse;
// 2: the prolongation x += P y, y coarse.
template <int D, class S>
static np_status time_level(int kind, const void *f, void *x, void *y, int lg, int bc, double h, int reps,
                            hipStream_t s, double *avg_ms) {
    hipEvent_t a = nullptr, b = nullptr;
    NP_HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return NP_EHIP;
    }
    auto run = [&]() -> np_status {
        if (kind == 0)
            return Ops<D, S>::sweep((const S *)f, (const S *)x, (S *)y, lg, bc, h, 2.0 / 3.0, 0, nullptr, nullptr,
                                    s, false, nullptr);
        if (kind == 1) return Ops<D, S>::restrict_((const S *)f, (const S *)x, (S *)y, lg, bc, h, s, nullptr);
        return Ops<D, S>::prolong_add((const S *)y, (S *)x, lg - 1, bc, s, nullptr);
    };
    np_status st = run();  // warm-up
    if (st == NP_OK && hipEventRecord(a, s) != hipSuccess) st = NP_EHIP;
    for (int r = 0; r < reps && st == NP_OK; ++r) st = run();
    float ms = 0.f;
    if (st == NP_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&ms, a, b) != hipSuccess))
        st = NP_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st == NP_EHIP) set_error("event timing failed");
    if (st == NP_OK) *avg_ms = double(ms) / reps;
    return st;
}

extern "C" np_status np_prof_level(np_dims dims, double h, np_bc bc, np_prec prec, int kind, const void *f,
                                   void *x, void *y, int reps, void *stream, double *avg_ms) {
    clear_error();
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (!x || !y || !avg_ms || reps < 1 || x == y || kind < 0 || kind > 2 || (kind < 2 && !f) || lg < 3) {
        set_error("bad argument");
        return NP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool d3 = dims.ndim == 3;
    switch (prec) {
    case NP_FP64: return d3 ? time_level<3, double>(kind, f, x, y, lg, bc, h, reps, s, avg_ms)
                            : time_level<2, double>(kind, f, x, y, lg, bc, h, reps, s, avg_ms);
    case NP_FP32: return d3 ? time_level<3, float>(kind, f, x, y, lg, bc, h, reps, s, avg_ms)
                            : time_level<2, float>(kind, f, x, y, lg, bc, h, reps, s, avg_ms);
    case NP_BF16: return d3 ? time_level<3, bf16>(kind, f, x, y, lg, bc, h, reps, s, avg_ms)
                            : time_level<2, bf16>(kind, f, x, y, lg, bc, h, reps, s, avg_ms);
    }
    set_error("unknown precision");
    return NP_EINVAL;
}

// One step of a 3D level on caller buffers in storage precision S (the
// kernels the cycle runs on that level), for the checks of the temporally
// blocked kernels against the per-kernel path.
template <class S>
static np_status op_level(int kind, const void *f, void *x, void *xout, void *c, int lg, int bc, double h,
                          hipStream_t s) {
    typedef Ops<3, S> O;
    const double w = 2.0 / 3.0;
    switch (kind) {
    case 0: return O::sweep((const S *)f, nullptr, (S *)x, lg, bc, h, w, 2, nullptr, nullptr, s, false, nullptr);
    case 1: return O::restrict_((const S *)f, (const S *)x, (S *)c, lg, bc, h, s, nullptr);
    case 2: return O::down0b((const S *)f, (S *)x, (S *)c, lg, bc, h, w, s, false, nullptr);
    case 3:
        NP_TRY(O::psweep((const S *)c, (const S *)f, (const S *)x, (S *)xout, lg, bc, h, w, s, false, nullptr));
        return O::sweep((const S *)f, (const S *)xout, (S *)x, lg, bc, h, w, 0, nullptr, nullptr, s, false, nullptr);
    case 4: return O::up2b((const S *)c, (const S *)f, (const S *)x, (S *)xout, lg, bc, h, w, s, false, nullptr);
    case 5:
    case 6:
    case 7:
    case 8:
        if (lg < 7 || lg > 10) { set_error("kinds 5 to 8 need 128 <= n <= 1024"); return NP_EINVAL; }
        if (kind == 7) return O::down0z((const S *)f, (S *)x, (S *)c, lg, bc, h, w, s, false, nullptr);
        if (kind == 8) {
            return O::down2z((const S *)f, (const S *)x, (S *)xout, (S *)c, nullptr, nullptr, lg, bc, h, w, s, false,
                             nullptr);
        }
        return O::sweep2z(kind == 5 ? (const S *)c : nullptr, (const S *)f, (const S *)x, (S *)xout, nullptr,
                          nullptr, lg, bc, h, w, s, false, nullptr);
    }
    return NP_EINVAL;
}

extern "C" np_status np_op_level(np_dims dims, double h, np_bc bc, np_prec prec, int kind, const void *f, void *x,
                                 void *xout, void *c, void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    if (dims.ndim != 3 || lg < 5 || kind < 0 || kind > 8 || !f || !x || ((kind >= 3 && kind != 7) && (!xout || xout == x)) ||
        (kind != 0 && kind != 6 && !c)) {
        set_error("np_op_level: 3D grids of n >= 32, kind 0..8, distinct non-null buffers");
        return NP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    np_status st = NP_EINVAL;
    switch (prec) {
    case NP_FP64: st = op_level<double>(kind, f, x, xout, c, lg, bc, h, s); break;
    case NP_FP32: st = op_level<float>(kind, f, x, xout, c, lg, bc, h, s); break;
    case NP_BF16: st = op_level<bf16>(kind, f, x, xout, c, lg, bc, h, s); break;
    default: set_error("unknown precision"); return NP_EINVAL;
    }
    NP_TRY(st);
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
    int nb = 0;
    if (dims.ndim == 2) NP_TRY((Ops<2, double>::resid_sq(f, x, lg, bc, h, H->red, s, nullptr, &nb)));
    else NP_TRY((Ops<3, double>::resid_sq(f, x, lg, bc, h, H->red, s, nullptr, &nb)));
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, H->red, nb, H->red + kPartials, 1);
    NP_LAUNCH_CHECK();
    NP_TRY(read_scalars(H, 1, s));
    *out = H->hred[0];
    return NP_OK;
}

// ------------------------------------- implicit advection-diffusion multigrid
// The backward-Euler step of Section 2.2 with constant velocity a and
// diffusivity nu, A T^{n+1} = T^n, solved as in Section 3.2 by multigrid:
// V(nu1, nu2) cycles with relaxed Jacobi (dividing by the filter centre),
// residual restriction by 2^d averaging, linear prolongation and the exact
// solve on the 4^d grid, or the paper's sawtooth cycle.  Every level uses the
// operator re-discretised at its own spacing (dt and a fixed).  FP64.

// Weights of the operator at spacing h: identity, nu dt (-Lap_h), and dt a_e
// times the upwind (scheme 0: backward difference for a_e >= 0, forward for
// a_e < 0) or central (scheme 1) first difference along each axis.
static AdW ad_weights(const np_ad_op &op, int d, double h) {
    AdW W{};
    const double dif = op.nu * op.dt / (h * h);
    W.c0 = 1.0 + 2.0 * d * dif;
    for (int e = 0; e < d; ++e) {
        const double c = op.a[e] * op.dt / h;
        W.cm[e] = -dif;
        W.cp[e] = -dif;
        if (op.scheme == 0) {
            if (op.a[e] >= 0.0) {
                W.c0 += c;
                W.cm[e] -= c;
            } else {
                W.c0 -= c;
                W.cp[e] += c;
            }
        } else {
            W.cm[e] -= 0.5 * c;
            W.cp[e] += 0.5 * c;
        }
    }
    return W;
}

// Inverse of the operator on the 4^d coarsest grid at spacing hc (dense
// assembly from the stencil and its ghost rule, Gauss-Jordan elimination
// with partial pivoting: A is not symmetric), cached on the hierarchy.
static np_status ad_coarse(Hier *H, const np_ad_op &op, double hc, hipStream_t s) {
    const double key[6] = {hc, op.dt, op.nu, op.a[0], op.a[1], op.a[2]};
    if (H->ad_minv && std::memcmp(key, H->ad_key, sizeof key) == 0 && H->ad_key_scheme == op.scheme) return NP_OK;
    const int d = H->d, m = d == 3 ? 64 : 16;
    const AdW W = ad_weights(op, d, hc);
    std::vector<double> A(size_t(m) * m, 0.0), I(size_t(m) * m, 0.0);
    for (int c = 0; c < m; ++c) {
        const int ix[3] = {c & 3, (c >> 2) & 3, c >> 4};
        A[size_t(c) * m + c] += W.c0;
        for (int e = 0; e < d; ++e)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double w = sgn < 0 ? W.cm[e] : W.cp[e];
                int nb[3] = {ix[0], ix[1], ix[2]};
                nb[e] += sgn;
                if (nb[e] < 0 || nb[e] > 3) {
                    if (H->bc == NP_BC_DIRICHLET0) {  // ghost = -(own value)
                        A[size_t(c) * m + c] -= w;
                        continue;
                    }
                    nb[e] &= 3;
                }
                A[size_t(c) * m + (nb[0] | nb[1] << 2 | nb[2] << 4)] += w;
            }
        I[size_t(c) * m + c] = 1.0;
    }
    for (int p = 0; p < m; ++p) {
        int piv = p;
        for (int r = p + 1; r < m; ++r)
            if (std::fabs(A[size_t(r) * m + p]) > std::fabs(A[size_t(piv) * m + p])) piv = r;
        if (!(std::fabs(A[size_t(piv) * m + p]) > 0.0)) {
            set_error("singular coarsest advection-diffusion operator");
            return NP_EINVAL;
        }
        if (piv != p)
            for (int q = 0; q < m; ++q) {
                std::swap(A[size_t(p) * m + q], A[size_t(piv) * m + q]);
                std::swap(I[size_t(p) * m + q], I[size_t(piv) * m + q]);
            }
        const double inv = 1.0 / A[size_t(p) * m + p];
        for (int q = 0; q < m; ++q) {
            A[size_t(p) * m + q] *= inv;
            I[size_t(p) * m + q] *= inv;
        }
        for (int r = 0; r < m; ++r) {
            if (r == p) continue;
            const double l = A[size_t(r) * m + p];
            if (l == 0.0) continue;
            for (int q = 0; q < m; ++q) {
                A[size_t(r) * m + q] -= l * A[size_t(p) * m + q];
                I[size_t(r) * m + q] -= l * I[size_t(p) * m + q];
            }
        }
    }
    if (!H->ad_minv) NP_TRY(dmalloc((void **)&H->ad_minv, sizeof(double) * 64 * 64));
    NP_HIP_TRY(hipMemcpyAsync(H->ad_minv, I.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    NP_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(H->ad_key, key, sizeof key);
    H->ad_key_scheme = op.scheme;
    return NP_OK;
}

// Partials of ||x - xold||_1 (or ||x||_1 without xold) and their sum into the
// per-cycle gauge, both gated by the controller.
template <int D>
static np_status ad_l1_gauge(Hier *H, const double *x, const double *xold, hipStream_t s) {
    const int64_t m0 = cells(D, H->lg);
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m0));
    hipLaunchKernelGGL(k_l1_diff, dim3(nb), dim3(kBlock), 0, s, x, xold, m0, H->red, &H->ctl->stop);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_l1_store, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->ctl, H->ad_l1);
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// Level launchers.  3D levels of at least 128^3 run on the z-marching tiles,
// 2D levels of at least 1024^2 on row-marching strips, smaller levels one
// cell per thread.
template <int D> static bool ad_zm3(int lg) { return D == 3 && lg >= 7 && g_tune.sweep3; }
template <int D> static bool ad_rm2(int lg) { return D == 2 && lg >= 10 && g_tune.sweep3; }

// One relaxed-Jacobi sweep xo = xi + wd (f - A xi).  partial != null: also
// the per-workgroup partials of ||f - A xi||^2, their count into *np.
template <int D>
static np_status ad_launch_sweep(const double *f, const double *xi, double *xo, double *partial, unsigned *np, int lg,
                                 int bc, const AdW &W, double wd, hipStream_t s, const int *stop) {
    const int64_t m = cells(D, lg);
    unsigned nb;
    if (ad_zm3<D>(lg)) {
        const int zc = sweep3_planes(lg, 1, kPartials);
        nb = zblocks(lg, 1, zc);
        if (partial)
            hipLaunchKernelGGL((k_ad_sweep3<true>), dim3(nb), dim3(kS3Threads), 0, s, f, xi, xo, partial, lg, bc, zc,
                               W, wd, stop);
        else
            hipLaunchKernelGGL((k_ad_sweep3<false>), dim3(nb), dim3(kS3Threads), 0, s, f, xi, xo, nullptr, lg, bc, zc,
                               W, wd, stop);
    } else if (ad_rm2<D>(lg)) {
        const int ry = r2_rows(lg);
        nb = unsigned(m / (kR2 * ry));
        if (partial)
            hipLaunchKernelGGL((k_ad_sweep2<true>), dim3(nb), dim3(kR2), 0, s, f, xi, xo, partial, lg, bc, ry, W, wd,
                               stop);
        else
            hipLaunchKernelGGL((k_ad_sweep2<false>), dim3(nb), dim3(kR2), 0, s, f, xi, xo, nullptr, lg, bc, ry, W, wd,
                               stop);
    } else if (partial) {
        nb = std::min<unsigned>(kNormBlocks, blocks_for(m));
        hipLaunchKernelGGL((k_ad_sweep<D, false, true>), dim3(nb), dim3(kBlock), 0, s, f, xi, xo, partial, lg, bc, W,
                           wd, stop);
    } else {
        nb = blocks_for(m);
        hipLaunchKernelGGL((k_ad_sweep<D, false, false>), dim3(nb), dim3(kBlock), 0, s, f, xi, xo, nullptr, lg, bc, W,
                           wd, stop);
    }
    NP_LAUNCH_CHECK();
    if (np) *np = nb;
    return NP_OK;
}

// fc = R (f - A x) onto the next coarser level.
template <int D>
static np_status ad_launch_restrict(const double *f, const double *x, double *fc, int lg, int bc, const AdW &W,
                                    hipStream_t s, const int *stop) {
    if (ad_zm3<D>(lg)) {
        const int zc = sweep3_planes(lg, 1, kPartials);
        hipLaunchKernelGGL(k_ad_restrict3, dim3(zblocks(lg, 1, zc)), dim3(kS3Threads), 0, s, f, x, fc, lg, bc, zc, W,
                           stop);
    } else if (ad_rm2<D>(lg)) {
        const int ry = r2_rows(lg);
        hipLaunchKernelGGL(k_ad_restrict2, dim3(unsigned(cells(2, lg) / (kR2 * ry))), dim3(kR2), 0, s, f, x, fc, lg,
                           bc, ry, W, stop);
    } else {
        hipLaunchKernelGGL((k_ad_resid_restrict<D>), dim3(blocks_for(cells(D, lg - 1))), dim3(kBlock), 0, s, f, x, fc,
                           lg, bc, W, stop);
    }
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// x += P ec from the next coarser level (lg: the fine level).
template <int D>
static np_status ad_launch_prolong(const double *ec, double *x, int lg, int bc, hipStream_t s, const int *stop) {
    if (ad_zm3<D>(lg)) {
        // the solver's prolongation kernel: its tiles take ZCfg's cells per thread (the
        // advection-diffusion sweep and restriction above take one)
        constexpr int CPT = ZCfg<double>::CPT;
        const int zc = sweep3_planes(lg, CPT, kPartials);
        hipLaunchKernelGGL((k_prolong3<double>), dim3(zblocks(lg, CPT, zc)), dim3(kS3Threads), 0, s, ec, x, lg, bc,
                           zc, stop);
    } else {
        hipLaunchKernelGGL((k_prolong_add<D, double>), dim3(blocks_for(cells(D, lg))), dim3(kBlock), 0, s, ec, x,
                           lg - 1, bc, stop);
    }
    NP_LAUNCH_CHECK();
    return NP_OK;
}

// One V(nu1, nu2) cycle of the operator on x (level 0 uses x, f and t[0]),
// opened by the convergence check of the input iterate; every launch is
// gated by the controller.  l1: record the change of x over the cycle.
template <int D>
static np_status ad_vcycle(Hier *H, const np_ad_op &op, const double *f, double *x, double h, const CycleOpts &co,
                           bool l1, hipStream_t s) {
    const int L = H->L, bc = H->bc, lg0 = H->lg;
    const int *stop = &H->ctl->stop;
    const int64_t m0 = cells(D, lg0);
    if (l1) {
        hipLaunchKernelGGL((k_copy<double>), dim3(blocks_for(m0)), dim3(kBlock), 0, s, x, H->xold, m0, stop);
        NP_LAUNCH_CHECK();
    }
    std::vector<double *> cur(L + 1), oth(L + 1);
    std::vector<const double *> F(L + 1);
    for (int l = 0; l <= L; ++l) {
        cur[l] = l == 0 ? x : (double *)H->x[l];
        oth[l] = (double *)H->t[l];
        F[l] = l == 0 ? f : (const double *)H->f[l];
    }
    // level handed to the one-workgroup tail (0 = none): the first coarse level
    // that fits it, unless it is the coarsest grid itself
    int tl = 0;
    if (g_tune.tail && co.nu1 >= 1)
        for (int l = 1; l <= L; ++l)
            if (lg0 - l <= Tail<D>::LG && lg0 - l > 2) { tl = l; break; }
    double hl = h;
    for (int l = 0; l <= L; ++l, hl *= 2.0) {
        const int lg = lg0 - l;
        const int64_t m = cells(D, lg);
        const AdW W = ad_weights(op, D, hl);
        const double wd = co.omega / W.c0;
        const bool zero = l > 0;
        if (l > 0 && l == tl) {  // levels tl .. L in one workgroup
            AdLevels Wl{};
            for (int q = 0; q <= L - l; ++q) Wl.w[q] = ad_weights(op, D, hl * double(int64_t(1) << q));
            hipLaunchKernelGGL((k_ad_tail<D>), dim3(1), dim3(Tail<D>::NT_AD), 0, s, F[l], cur[l], H->ad_minv, lg, bc,
                               Wl, co.omega, co.nu1, co.nu2, stop);
            NP_LAUNCH_CHECK();
            break;
        }
        if (l == 0 && (co.nu1 == 0 || L == 0)) {  // the check on its own: no sweep opens this level
            const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m));
            hipLaunchKernelGGL((k_ad_resid<D>), dim3(nb), dim3(kBlock), 0, s, F[0], cur[0], nullptr, H->red, lg, bc,
                               W, stop);
            NP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->ctl);
            NP_LAUNCH_CHECK();
        }
        if (l == L) {  // exact solve on the coarsest grid
            hipLaunchKernelGGL((k_ad_coarse<D>), dim3(1), dim3(64), 0, s, F[L], cur[L], H->ad_minv, bc, W,
                               zero ? 1 : 0, stop);
            NP_LAUNCH_CHECK();
            break;
        }
        if (zero && co.nu1 == 0) {
            hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, cur[l], m, stop);
            NP_LAUNCH_CHECK();
        }
        for (int it = 0; it < co.nu1; ++it) {
            void *tok = nullptr;
            const bool prof = l == 0 && it > 0 && (prof_on() & kProfJacobi);
            if (prof) NP_TRY(prof_begin(s, &tok));
            if (zero && it == 0) {
                hipLaunchKernelGGL((k_ad_sweep<D, true, false>), dim3(blocks_for(m)), dim3(kBlock), 0, s, F[l],
                                   nullptr, oth[l], nullptr, lg, bc, W, wd, stop);
                NP_LAUNCH_CHECK();
            } else if (l == 0 && it == 0) {  // residual norm of the input iterate, then the stop rule
                unsigned nb = 0;
                NP_TRY(ad_launch_sweep<D>(F[l], cur[l], oth[l], H->red, &nb, lg, bc, W, wd, s, stop));
                hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->ctl);
                NP_LAUNCH_CHECK();
            } else {
                NP_TRY(ad_launch_sweep<D>(F[l], cur[l], oth[l], nullptr, nullptr, lg, bc, W, wd, s, stop));
            }
            if (prof) NP_TRY(prof_end(s, tok, double(m) * 3 * sizeof(double)));
            std::swap(cur[l], oth[l]);
        }
        void *tok = nullptr;
        const bool prof = l == 0 && (prof_on() & kProfRestrict);
        if (prof) NP_TRY(prof_begin(s, &tok));
        NP_TRY(ad_launch_restrict<D>(F[l], cur[l], (double *)H->f[l + 1], lg, bc, W, s, stop));
        if (prof) NP_TRY(prof_end(s, tok, double(m) * (2 + 1.0 / (1 << D)) * sizeof(double)));
    }
    for (int l = (tl > 0 ? tl : L) - 1; l >= 0; --l) {
        const int lg = lg0 - l;
        const int64_t m = cells(D, lg);
        const AdW W = ad_weights(op, D, h * double(int64_t(1) << l));
        const double wd = co.omega / W.c0;
        void *tok = nullptr;
        const bool prof = l == 0 && (prof_on() & kProfProlong);
        if (prof) NP_TRY(prof_begin(s, &tok));
        NP_TRY(ad_launch_prolong<D>(cur[l + 1], cur[l], lg, bc, s, stop));
        if (prof) NP_TRY(prof_end(s, tok, double(m) * (2 + 1.0 / (1 << D)) * sizeof(double)));
        for (int it = 0; it < co.nu2; ++it) {
            void *tk = nullptr;
            const bool pj = l == 0 && (prof_on() & kProfJacobi);
            if (pj) NP_TRY(prof_begin(s, &tk));
            NP_TRY(ad_launch_sweep<D>(F[l], cur[l], oth[l], nullptr, nullptr, lg, bc, W, wd, s, stop));
            if (pj) NP_TRY(prof_end(s, tk, double(m) * 3 * sizeof(double)));
            std::swap(cur[l], oth[l]);
        }
    }
    if (cur[0] != x) {
        hipLaunchKernelGGL((k_copy<double>), dim3(blocks_for(m0)), dim3(kBlock), 0, s, cur[0], x, m0, stop);
        NP_LAUNCH_CHECK();
    }
    if (l1) NP_TRY(ad_l1_gauge<D>(H, x, H->xold, s));
    return NP_OK;
}

// One sawtooth cycle of the operator (Section 2.2; Appendix B): the finest
// residual (its norm is the convergence check), restricted level by level to
// the coarsest grid; then from the coarsest up e = r / A_00 + P e_coarse
// (copy or linear prolongation) and nu2 relaxed-Jacobi steps (alpha = omega)
// on the level's residual equation; x += e_0.  Buffers as saw_cycle.
template <int D>
static np_status ad_saw_cycle(Hier *H, const np_ad_op &op, const double *f, double *x, double h,
                              const np_mg_opts &o, bool l1, hipStream_t s) {
    const int L = H->L, bc = H->bc, lg0 = H->lg;
    const int *stop = &H->ctl->stop;
    const int64_t m0 = cells(D, lg0);
    std::vector<double *> r(L + 1), e(L + 1), t(L + 1);
    for (int l = 0; l <= L; ++l) {
        r[l] = l == 0 ? (double *)H->t[0] : (double *)H->f[l];
        e[l] = l == 0 ? H->saw : (double *)H->x[l];
        t[l] = l == 0 ? H->saw + m0 : (double *)H->t[l];
    }
    const unsigned nb = std::min<unsigned>(kRedBlocks, blocks_for(m0));
    hipLaunchKernelGGL((k_ad_resid<D>), dim3(nb), dim3(kBlock), 0, s, f, x, r[0], H->red, lg0, bc,
                       ad_weights(op, D, h), stop);
    NP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, H->red, int(nb), H->ctl);
    NP_LAUNCH_CHECK();
    for (int l = 0; l < L; ++l) {
        const int lgc = lg0 - l - 1;
        hipLaunchKernelGGL((k_restrict_field<D>), dim3(blocks_for(cells(D, lgc))), dim3(kBlock), 0, s, r[l],
                           r[l + 1], lgc, stop);
        NP_LAUNCH_CHECK();
    }
    std::vector<double *> done(L + 2, nullptr);
    for (int l = L; l >= 0; --l) {
        const int lg = lg0 - l;
        const int64_t ml = cells(D, lg);
        const AdW W = ad_weights(op, D, h * double(int64_t(1) << l));
        hipLaunchKernelGGL((k_saw_up<D>), dim3(blocks_for(ml)), dim3(kBlock), 0, s, r[l], done[l + 1], e[l], lg, bc,
                           1.0 / W.c0, o.prolong, stop);
        NP_LAUNCH_CHECK();
        double *cur = e[l], *oth = t[l];
        for (int it = 0; it < o.nu2; ++it) {
            hipLaunchKernelGGL((k_ad_sweep<D, false, false>), dim3(blocks_for(ml)), dim3(kBlock), 0, s, r[l], cur,
                               oth, nullptr, lg, bc, W, o.omega / W.c0, stop);
            NP_LAUNCH_CHECK();
            std::swap(cur, oth);
        }
        done[l] = cur;
    }
    hipLaunchKernelGGL(k_add_to, dim3(blocks_for(m0)), dim3(kBlock), 0, s, x, done[0], m0, stop);
    NP_LAUNCH_CHECK();
    if (l1) NP_TRY(ad_l1_gauge<D>(H, done[0], nullptr, s));
    return NP_OK;
}

template <int D>
static np_status solve_ad(Hier *H, const np_ad_op &op, const double *f, double *x, double h, double tol,
                          const np_mg_opts &o, const CycleOpts &co, hipStream_t s, double nf, double *l1_out,
                          np_mg_stats *stats) {
    NP_TRY(ensure_levels(H));
    const int64_t m0 = cells(D, H->lg);
    const bool l1 = l1_out != nullptr;
    if (o.cycle == 1 && !H->saw) NP_TRY(dmalloc((void **)&H->saw, sizeof(double) * 2 * m0));
    if (l1 && o.cycle == 0 && !H->xold) NP_TRY(dmalloc((void **)&H->xold, sizeof(double) * m0));
    if (l1 && !H->ad_l1) NP_TRY(dmalloc((void **)&H->ad_l1, sizeof(double) * 256));
    if (o.cycle == 0) NP_TRY(ad_coarse(H, op, h * double(int64_t(1) << H->L), s));
    NP_TRY(init_ctl(H, o, nf, tol, 0, 0.0, s));
    GraphKey key{o.cycle == 1 ? 7 : 6, o.prolong, 1, x, f, h, co.nu1, co.nu2, 0, co.omega,
                 {op.dt, op.nu, op.a[0], op.a[1], op.a[2]}, op.scheme, l1 ? 1 : 0};
    int batch = o.fixed_cycles > 0 ? o.fixed_cycles + 1 : g_tune.batch;
    for (;;) {
        NP_TRY(run_graphs(H, key, s, batch, 0, false, [&](hipStream_t q, int) {
            return o.cycle == 1 ? ad_saw_cycle<D>(H, op, f, x, h, o, l1, q) : ad_vcycle<D>(H, op, f, x, h, co, l1, q);
        }));
        NP_TRY(read_ctl(H, s));
        if (H->hctl->stop) break;
        batch = next_batch(*H->hctl, o, false);
    }
    const Ctl c = *H->hctl;
    fill_stats(stats, c, c.k, c.k);
    if (l1) {
        const int n = std::min(c.k, 256);
        for (int i = n; i < 256; ++i) l1_out[i] = 0.0;
        if (n > 0) {
            NP_HIP_TRY(hipMemcpyAsync(l1_out, H->ad_l1, sizeof(double) * n, hipMemcpyDeviceToHost, s));
            NP_HIP_TRY(hipStreamSynchronize(s));
        }
    }
    return status_of(c, tol);
}

static np_status check_ad_op(const np_ad_op *op, int d) {
    if (!op) { set_error("null operator"); return NP_EINVAL; }
    if (!(op->dt > 0.0) || !std::isfinite(op->dt)) { set_error("dt must be positive"); return NP_EINVAL; }
    if (!(op->nu >= 0.0) || !std::isfinite(op->nu)) { set_error("nu must be non-negative"); return NP_EINVAL; }
    for (int e = 0; e < d; ++e)
        if (!std::isfinite(op->a[e])) { set_error("non-finite velocity"); return NP_EINVAL; }
    if (op->scheme != 0 && op->scheme != 1) { set_error("scheme must be 0 (upwind) or 1 (central)"); return NP_EINVAL; }
    return NP_OK;
}

extern "C" np_status np_ad_implicit_solve(np_dims dims, double h, np_bc bc, const np_ad_op *op, const double *rhs,
                                          double *x, double tol, const np_mg_opts *opts, np_mg_stats *stats,
                                          double *l1_change) {
    clear_error();
    np_mg_opts o;
    CycleOpts co;
    fill_opts(opts, co, o);
    int lg = -1;
    NP_TRY(check_solve_args(dims, h, bc, rhs, x, tol, o, &lg));
    NP_TRY(check_ad_op(op, dims.ndim));
    if (o.smooth_prec != NP_FP64 || o.warm_start == 1) {
        set_error("the advection-diffusion solve runs in FP64 from a zero or caller guess");
        return NP_EINVAL;
    }
    np_ad_op op2 = *op;
    for (int e = dims.ndim; e < 3; ++e) op2.a[e] = 0.0;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (l1_change) std::memset(l1_change, 0, sizeof(double) * 256);
    const int d = dims.ndim;
    hipStream_t s = (hipStream_t)o.stream;
    Hier *H = nullptr;
    NP_TRY(get_hier(d, lg, bc, NP_FP64, &H));
    std::lock_guard<std::mutex> lk(H->mu);
    const int64_t m = cells(d, lg);
    NP_TRY(dsum(H, rhs, m, 1, 0, s));
    NP_TRY(read_scalars(H, 1, s));
    const double nf = H->hred[0];
    if (!std::isfinite(nf)) {
        set_error("non-finite right-hand side");
        return NP_ENAN;
    }
    if (nf == 0.0 || o.warm_start == 0) {
        hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, m, nullptr);
        NP_LAUNCH_CHECK();
    }
    if (nf == 0.0) {
        NP_HIP_TRY(hipStreamSynchronize(s));
        return NP_OK;
    }
    np_status st = d == 2 ? solve_ad<2>(H, op2, rhs, x, h, tol, o, co, s, nf, l1_change, stats)
                          : solve_ad<3>(H, op2, rhs, x, h, tol, o, co, s, nf, l1_change, stats);
    if (st == NP_EHIP || st == NP_ENOMEM || st == NP_EINVAL) return st;
    NP_HIP_TRY(hipStreamSynchronize(s));
    return st;
}

extern "C" np_status np_ad_apply(np_dims dims, double h, np_bc bc, const np_ad_op *op, const double *x, double *y,
                                 void *stream) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    NP_TRY(check_ad_op(op, dims.ndim));
    if (!x || !y) { set_error("null array"); return NP_EINVAL; }
    np_ad_op op2 = *op;
    for (int e = dims.ndim; e < 3; ++e) op2.a[e] = 0.0;
    const int64_t m = cells(dims.ndim, lg);
    hipStream_t s = (hipStream_t)stream;
    const AdW W = ad_weights(op2, dims.ndim, h);
    if (dims.ndim == 2) hipLaunchKernelGGL((k_ad_apply<2>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, y, lg, bc, W);
    else hipLaunchKernelGGL((k_ad_apply<3>), dim3(blocks_for(m)), dim3(kBlock), 0, s, x, y, lg, bc, W);
    NP_LAUNCH_CHECK();
    NP_HIP_TRY(hipStreamSynchronize(s));
    return NP_OK;
}

// Back-to-back launches of an advection-diffusion level kernel the solver
// uses on this grid (same kernel and launch shape) between two events on the
// stream: kind 0 the sweep y = sweep(x); 1 the residual restriction y =
// R (f - A x); 2 the prolongation x += P y.
template <int D>
static np_status time_ad_level(int kind, const np_ad_op &op, const double *f, double *x, double *y, int lg, int bc,
                               double h, int reps, hipStream_t s, double *avg_ms) {
    hipEvent_t a = nullptr, b = nullptr;
    NP_HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return NP_EHIP;
    }
    const AdW W = ad_weights(op, D, h);
    auto run = [&]() -> np_status {
        if (kind == 0)
            return ad_launch_sweep<D>(f, x, y, nullptr, nullptr, lg, bc, W, (2.0 / 3.0) / W.c0, s, nullptr);
        if (kind == 1) return ad_launch_restrict<D>(f, x, y, lg, bc, W, s, nullptr);
        return ad_launch_prolong<D>(y, x, lg, bc, s, nullptr);
    };
    np_status st = run();  // warm-up
    if (st == NP_OK && hipEventRecord(a, s) != hipSuccess) st = NP_EHIP;
    for (int r = 0; r < reps && st == NP_OK; ++r) st = run();
    float ms = 0.f;
    if (st == NP_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&ms, a, b) != hipSuccess))
        st = NP_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st == NP_EHIP) set_error("event timing failed");
    if (st == NP_OK) *avg_ms = double(ms) / reps;
    return st;
}

extern "C" np_status np_ad_prof_level(np_dims dims, double h, np_bc bc, const np_ad_op *op, int kind, const double *f,
                                      double *x, double *y, int reps, void *stream, double *avg_ms) {
    int lg;
    NP_TRY(op_prelude(dims, h, bc, &lg));
    NP_TRY(check_ad_op(op, dims.ndim));
    if (!x || !y || !avg_ms || reps < 1 || x == y || kind < 0 || kind > 2 || (kind < 2 && !f) || lg < 3) {
        set_error("bad argument");
        return NP_EINVAL;
    }
    np_ad_op op2 = *op;
    for (int e = dims.ndim; e < 3; ++e) op2.a[e] = 0.0;
    hipStream_t s = (hipStream_t)stream;
    return dims.ndim == 3 ? time_ad_level<3>(kind, op2, f, x, y, lg, bc, h, reps, s, avg_ms)
                          : time_ad_level<2>(kind, op2, f, x, y, lg, bc, h, reps, s, avg_ms);
}
