// Host core and C ABI: geometry and PML tables (Sec. 2.1-2.2), the strip factorisation
// (Algorithm 1), the double sweep P (eqs. solve_upward / solve_downward), its reduced form
// (Algorithms 2-4) and right-preconditioned GMRES (Algorithm 5, Sec. 2.3).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

#include "helm_internal.hpp"

using helm::BLK;
using helm::NSLOT;
using helm::WP;

namespace helm {
// concurrent sweeps with Robin transmission (kernels_robin.hip)
hipError_t launch_robin_rhs(const double2* f, const double2* L, const double2* R, const double2* rho_l,
                            const double2* rho_r, double2* out, int nrhs, int Nrow, int Nx, int lo, int W,
                            int c0, int c1, double ih2, hipStream_t st);
hipError_t launch_parity_pick(const double2* E, const double2* O, const int* par, double2* out, int nrhs,
                              long Nrow, int Nx, hipStream_t st);
}  // namespace helm
using cd = std::complex<double>;

struct Work {
    int nrhs = 0;
    void* Yw = nullptr;
    double2 *V = nullptr, *G = nullptr, *PF = nullptr, *Psi = nullptr, *Wf = nullptr,
            *Hf = nullptr, *Ut = nullptr, *R = nullptr, *Tup = nullptr, *Tdn = nullptr;
    // interface-window fields of the reduced operator (v, g = psi - A v, w; concurrent sweep:
    // v, z, w')
    double2 *Vw = nullptr, *Gw = nullptr, *Ww = nullptr;
    // concurrent sweep: strip-solver workspaces of the downward chain and of the z solves, and
    // the input field of its reduced operator (zero off the reduced columns)
    void *Yw2 = nullptr, *Yw3 = nullptr;
    double2* PsiC = nullptr;
    // Robin transmission: [2][nrhs][Nrow], a zero half and the data (V_o - rho V_i) / h^2 of
    // the strip being solved (the transmission source is coef * (second half - first half))
    double2* Rob = nullptr;
    // concurrent Robin sweeps: the right-hand sides of a step's two subdomains, [2][nrhs][Nrow][WP]
    double2* RobR = nullptr;
    // GMRES.  gnrhs is the right-hand-side capacity of every buffer below and of R, Ut:
    // they are laid out for the nrhs of each call ([k][nrhs][n]) and reallocated when a
    // call brings more right-hand sides than they were sized for
    int mcap = 0, gnrhs = 0;
    long n = 0;
    double2* basis = nullptr;
    double2* w = nullptr;
    double2* h1 = nullptr;
    double2* h2 = nullptr;
    double* nrm = nullptr;
    double2* partial = nullptr;
    double* npartial = nullptr;
    double2* y = nullptr;
    double2* red = nullptr;
    double2* apin = nullptr;    // fixed input of the captured reduced operator
    double2* basis_old = nullptr;   // the previous cycle's basis, kept through a restart
    int mcap_old = 0;
};

// Event-pair timing of kernel launches (helm_set_kernel_timing).
struct EventTimer : helm::KTimer {
    static constexpr int kMax = 65536;
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;        // class of pair k (events 2k, 2k+1)
    int used = 0;
    long counts[helm::K_NCLASS] = {0};
    double ms[helm::K_NCLASS] = {0};
    int pending_cls = -1;
    unsigned mask = 0xFFu;       // classes whose launches are timed (all are counted)
    hipEvent_t get(int idx) {
        while ((int)pool.size() <= idx) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[idx];
    }
    void begin(int c, hipStream_t st) override {
        counts[c] += 1;
        if (used >= kMax || !(mask & (1u << c))) { pending_cls = -1; return; }
        hipEvent_t e = get(2 * used);
        if (!e || !get(2 * used + 1)) { pending_cls = -1; return; }
        (void)hipEventRecord(e, st);
        pending_cls = c;
    }
    void end(int c, hipStream_t st) override {
        if (pending_cls != c) return;
        (void)hipEventRecord(pool[2 * used + 1], st);
        cls.push_back(c);
        ++used;
        pending_cls = -1;
    }
    void collect() {
        for (int k = 0; k < used; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) ms[cls[k]] += t;
        }
        used = 0;
        cls.clear();
    }
    void reset() {
        used = 0; cls.clear(); pending_cls = -1;
        for (int c = 0; c < helm::K_NCLASS; ++c) { counts[c] = 0; ms[c] = 0; }
    }
    ~EventTimer() override { for (hipEvent_t e : pool) (void)hipEventDestroy(e); }
};

// slab groups (one stream each) of the 3-D complex64 factorisation
#ifndef FAC3_GROUPS
#define FAC3_GROUPS 2
#endif
#ifndef FAC3_BATCH
#define FAC3_BATCH 0      // slabs per group; 0: the slabs split evenly over the streams
#endif

struct Fuser;

struct helm_problem {
    helm::Geom g;
    helm::Chunks ch;
    helm::DevTables t;
    hipStream_t st = nullptr;
    int prec = HELM_C128, mode = HELM_FULL, max_iter = 200;
    std::string err;
    void* F = nullptr;          // factors: double2 (C128) or float2 (MIXED)
    void* Fc = nullptr;         // compact spike rows at the target columns, same precision
    void* Fs = nullptr;         // separator propagators of the two-level separator solve
    void* Fa = nullptr;         // complex64 2-D: operand-order copies of the factors
    void* Fw = nullptr;         //   (helm::launch_swizzle_factors)
    double2* F64 = nullptr;     // FP64 factor (the complex64 path's factorisation workspace)
    double2* Fs64 = nullptr;    // FP64 propagators (idem)
    int fac_m = 0;              // rows per chunk the factor buffers were laid out for
    int factor_path = 0;        // 3-D: 1 = complex64 blocked Gauss-Jordan, 0 = FP64 inverses
    // strips with identical operators share one factorisation: fidx[s] is the factor slot
    // of strip s; the factor kernels run on the slots' representative strips (tf, gf: the
    // per-strip tables and the geometry restricted to the representatives)
    std::vector<int> fidx;
    int nfac = 0;
    helm::DevTables tf;
    helm::Geom gf;
    bool factored = false;
    int* d_err = nullptr;
    Work wk;
    int stat_ap = 0, stat_restarts = 0;
    // right-hand sides that went through the GMRES operator, and as many without dropping
    // the converged ones from its panel
    long long stat_panel = 0, stat_panel_full = 0;
    // strip-solve rounds of the last helm_solve_batch this handle took part in: launched as
    // one multi-problem launch per phase, or problem by problem
    long long stat_fused = 0, stat_unfused = 0;
    int dev = 0;                // HIP device of the handle
    int use_graph = 1;          // replay Algorithm 3 from a captured HIP graph (REDUCED)
    // captured reduced operators, one per right-hand-side count (the GMRES panel shrinks to
    // the multiple of 16 that holds its unconverged right-hand sides): least recently used
    // entry replaced
    struct ApGraph {
        hipGraphExec_t exec = nullptr;
        int nrhs = 0;
        const void* out = nullptr;
        long epoch = -1;
        unsigned long used = 0;
    };
    static constexpr int NGRAPH = 4;
    ApGraph apg[NGRAPH];
    unsigned long ap_tick = 0;
    int sweep = 0;              // 0: the double sweep P; 1: the concurrent double sweep P_c
    int trans = 0;              // 0: PML transmission; 1: Robin transmission (Sec. 4.4)
    int* colpar = nullptr;      // concurrent Robin sweeps: parity of the strip whose core holds each column
    int restart = 0;            // GMRES cycle length (0: by mode)
    int batch_fuse = 0;         // join fused strip-solve launches in helm_solve_batch
    hipStream_t st_c[2] = {};   // concurrent sweep: streams of the downward chain and the z solves
    hipEvent_t ev_c[3] = {};    // fork / join events of the concurrent sweep
    hipStream_t st_fac[FAC3_GROUPS - 1] = {};   // group streams of the 3-D complex64 factorisation
    hipStream_t cap_st = nullptr;  // private stream the graph is captured on (capture is not
                                   // allowed on the legacy default stream); replays go to st
    long ws_epoch = 0;          // workspace generation (graphs captured before it are stale)
    double stat_ms = 0.0;
    std::vector<void*> owned;   // table allocations
    EventTimer* timer = nullptr; // non-null while kernel timing is enabled
    Fuser* fuser = nullptr;     // set during helm_solve_batch: strip solves join fused launches
    hipEvent_t fuse_ev = nullptr; // marks this handle's work before a fused strip solve
    helm::KTimer* kt() { return timer; }
};

// Strip solves of several problems' host threads in one launch per phase (helm_solve_batch).
// Every participating thread deposits each strip solve and waits; when every thread that
// has not finished its solve has deposited one, the last to arrive launches the round on
// the fuser's stream and releases the others.  The round's jobs are grouped by the form of
// their phase C (target columns or all); a group of two or more jobs that qualify is one
// multi-problem launch per phase, the rest launch one by one.  Waiting for every unfinished
// thread keeps the problems in lockstep, one strip of each per round (a thread between two
// operator applications holds the round until it deposits again).  Each problem keeps its
// own stream: the fuser's stream waits for an event recorded on the depositor's stream,
// and the depositor's stream waits for an event recorded after the launch, so each
// problem's work stays in its program order and its synchronisations wait for its own work.
struct Fuser {
    struct Pending {
        helm::StripJob job;
        hipStream_t st;
        hipEvent_t ready;
        hipError_t* result;
    };
    std::mutex mu;
    std::condition_variable cv;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    int active = 0;                  // participants that have not finished their solve
    long round = 0;
    std::vector<Pending> pend;
    long fused_launches = 0, single_launches = 0;

    void join() {
        std::lock_guard<std::mutex> lk(mu);
        ++active;
    }
    void leave() {
        std::unique_lock<std::mutex> lk(mu);
        --active;
        if (!pend.empty() && (int)pend.size() >= active) launch_round();
    }
    hipError_t submit(const helm::StripJob& j, hipStream_t own, hipEvent_t ready) {
        hipError_t e = hipEventRecord(ready, own);
        if (e != hipSuccess) return e;
        std::unique_lock<std::mutex> lk(mu);
        pend.push_back(Pending{j, own, ready, &e});
        const long my = round;
        if ((int)pend.size() >= active) launch_round();
        else cv.wait(lk, [&] { return round != my; });
        return e;
    }
    // with mu held
    void launch_round() {
        const int n = (int)pend.size();
        hipError_t e = hipSuccess;
        for (const Pending& p : pend)
            if (e == hipSuccess) e = hipStreamWaitEvent(st, p.ready, 0);
        // groups: jobs that qualify alone for a multi-problem launch, by phase-C form
        std::vector<helm::StripJob> grp[2], rest;
        for (const Pending& p : pend) {
            const helm::StripJob& j = p.job;
            const int cls = (j.io.targets_only && j.Fc) ? 1 : 0;
            helm::StripJob pair[2] = {j, j};
            if (helm::strip_jobs_fusable(pair, 2)) grp[cls].push_back(j);
            else rest.push_back(j);
        }
        auto single = [&](const helm::StripJob& j) {
            ++single_launches;
            return helm::launch_strip_solve<float>(
                *j.t, *j.g, *j.ch, j.s, j.fs, static_cast<const float2*>(j.F),
                static_cast<const float2*>(j.Fc), static_cast<const float2*>(j.Fs),
                static_cast<const float2*>(j.Fa), static_cast<const float2*>(j.Fw),
                static_cast<float2*>(j.Yw), j.nrhs, j.io, st, nullptr);
        };
        for (auto& gj : grp)
            for (size_t k0 = 0; k0 < gj.size() && e == hipSuccess; k0 += helm::MULTI_MAX) {
                const int m = (int)std::min<size_t>(helm::MULTI_MAX, gj.size() - k0);
                if (m >= 2) {
                    e = helm::launch_strip_solve_multi(gj.data() + k0, m, st, nullptr);
                    ++fused_launches;
                } else {
                    e = single(gj[k0]);
                }
            }
        for (size_t k = 0; k < rest.size() && e == hipSuccess; ++k) e = single(rest[k]);
        (void)n;
        if (e == hipSuccess) e = hipEventRecord(done, st);
        for (const Pending& p : pend) {
            hipError_t w = e == hipSuccess ? hipStreamWaitEvent(p.st, done, 0) : e;
            *p.result = w;
        }
        pend.clear();
        ++round;
        cv.notify_all();
    }
};

namespace {

// roctx range over a scope (host side; visible to rocprofv3 --marker-trace, free otherwise)
struct Range {
    explicit Range(const char* m) { roctxRangePushA(m); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

thread_local std::string g_setup_err;   // message of the last failed helm_setup

// y-partition of the strip solver: m rows per chunk, the last row of every chunk but the
// last a separator; separator groups of q ~ sqrt(#separators) for the two-level solve
void set_chunks(helm_t H, int m) {
    const int Ny = H->g.Ny;
    m = std::max(2, m);
    H->ch.m = m;
    H->ch.P = (Ny + m - 1) / m;
    if (H->ch.P > 1 && (H->ch.P - 1) * m >= Ny) H->ch.P -= 1;
    const int ns = H->ch.P - 1;
    H->ch.q = std::max(2, (int)std::ceil(std::sqrt((double)std::max(ns, 1))));
    H->ch.G = ns >= 4 ? (ns + H->ch.q - 1) / H->ch.q : 1;
}

// HELM_TRACE=1 in the environment prints the residual history of every GMRES cycle to stderr
bool trace_on() {
    static const bool on = [] { const char* e = std::getenv("HELM_TRACE"); return e && e[0] == '1'; }();
    return on;
}

helm_status fail(helm_t H, helm_status code, const std::string& msg) {
    if (H) H->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(H, e_ == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EHIP,            \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

#define CHK(expr)                                 \
    do {                                          \
        helm_status s_ = (expr);                  \
        if (s_ != HELM_OK) return s_;             \
    } while (0)

template <typename P>
helm_status dmalloc(helm_t H, P** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess)
        return fail(H, HELM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                        hipGetErrorString(e));
    return HELM_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

// ---------------------------------------------------------------- PML profile
// sigma(xi) = sigma_max (xi / (w h))^power for depth xi = depth_cells * h inside a layer
// of w cells; alpha = 1 / (1 + i sigma / omega)  (Sec. 2.1).
double sigma_of(double depth_cells, int width, double smax, double power) {
    if (depth_cells <= 0.0 || width <= 0) return 0.0;
    return smax * std::pow(depth_cells / width, power);
}
cd alpha_of(double sigma, double omega) { return 1.0 / cd(1.0, sigma / omega); }

double outer_depth(const helm::Geom& g, double pos, int N) {
    const double lo = g.wout - 0.5, hi = N - g.wout - 0.5;
    return std::max(std::max(lo - pos, pos - hi), 0.0);
}
double smax_of(const helm::Geom& g, int width, double s0) {
    return width > 0 ? s0 * g.cref / (width * g.h) : 0.0;
}
cd alpha_outer(const helm::Geom& g, double pos, int N) {
    return alpha_of(sigma_of(outer_depth(g, pos, N), g.wout, smax_of(g, g.wout, g.s0), g.power), g.omega);
}
// alpha_x of the padded strip operator at global position pos (points integer, half-points
// x.5): pad profile left of the left pad edge / right of the right pad edge, else global.
// The pads take their own strength s0i: they enter only the strip operators.
cd alpha_strip(const helm::Geom& g, const helm::Strip& s, double pos) {
    if (s.lpad && pos < s.core_lo - 0.5)
        return alpha_of(sigma_of(s.core_lo - 0.5 - pos, g.w, smax_of(g, g.w, g.s0i), g.power), g.omega);
    if (s.rpad && pos > s.dom_hi - 0.5)
        return alpha_of(sigma_of(pos - (s.dom_hi - 0.5), g.w, smax_of(g, g.w, g.s0i), g.power), g.omega);
    return alpha_outer(g, pos, g.Nx);
}

double2 d2(cd z) { return make_double2(z.real(), z.imag()); }

helm_status upload(helm_t H, void** dptr, const void* src, size_t bytes) {
    CHK(dmalloc(H, dptr, bytes));
    H->owned.push_back(*dptr);
    HIPCHK(hipMemcpy(*dptr, src, bytes, hipMemcpyHostToDevice));
    return HELM_OK;
}

// ---------------------------------------------------------------- workspaces
void free_work(Work& w) {
    void* ps[] = {w.Yw, w.V, w.G, w.PF, w.Psi, w.Wf, w.Hf, w.Vw, w.Gw, w.Ww, w.Ut, w.R, w.Tup, w.Tdn, w.basis,
                  w.w, w.h1, w.h2, w.nrm, w.partial, w.npartial, w.y, w.red, w.apin, w.basis_old,
                  w.Yw2, w.Yw3, w.PsiC, w.Rob, w.RobR};
    for (void* p : ps) dfree(p);
    w = Work();
}

size_t field_bytes(helm_t H, int nrhs) { return (size_t)nrhs * H->g.Nrow() * H->g.Nx * sizeof(double2); }

int rhs_pad16(int nrhs) { return (nrhs + 15) / 16 * 16; }

helm_status ensure_sweep_ws(helm_t H, int nrhs) {
    Work& w = H->wk;
    if (w.nrhs >= nrhs && w.V) return HELM_OK;
    free_work(w);
    H->ws_epoch += 1;
    const auto& g = H->g;
    const size_t fb = field_bytes(H, nrhs);
    const size_t yw = g.dim == 3 ? (size_t)(g.Ny + 2) * g.Bp * rhs_pad16(nrhs) * sizeof(double2)
                                 : (size_t)nrhs * g.Ny * WP * sizeof(double2);
    CHK(dmalloc(H, &w.Yw, yw));
    if (H->sweep == 1) {
        CHK(dmalloc(H, &w.Yw2, yw));
        CHK(dmalloc(H, &w.Yw3, yw));
        CHK(dmalloc(H, &w.PsiC, fb));
        HIPCHK(hipMemsetAsync(w.PsiC, 0, fb, H->st));
    }
    if (H->trans == 1) {
        const size_t rb = (size_t)2 * nrhs * g.Nrow() * sizeof(double2);
        CHK(dmalloc(H, &w.Rob, rb));
        HIPCHK(hipMemsetAsync(w.Rob, 0, rb, H->st));
        if (H->sweep == 1) CHK(dmalloc(H, &w.RobR, (size_t)2 * nrhs * g.Nrow() * WP * sizeof(double2)));
    }
    double2** fields[] = {&w.V, &w.G, &w.PF, &w.Psi, &w.Wf, &w.Hf};
    for (double2** f : fields) {
        CHK(dmalloc(H, f, fb));
        HIPCHK(hipMemsetAsync(*f, 0, fb, H->st));
    }
    // window fields: entries no sweep writes (the windows' outer columns, the columns of
    // strips a reduced sweep skips) must stay zero
    const size_t wb = (size_t)nrhs * g.Nrow() * std::max(1, g.J - 1) * helm::IWIN * sizeof(double2);
    double2** wfields[] = {&w.Vw, &w.Gw, &w.Ww};
    for (double2** f : wfields) {
        CHK(dmalloc(H, f, wb));
        HIPCHK(hipMemsetAsync(*f, 0, wb, H->st));
    }
    const size_t tb = (size_t)std::max(1, g.J) * 2 * nrhs * g.Nrow() * sizeof(double2);
    CHK(dmalloc(H, &w.Tup, tb));
    CHK(dmalloc(H, &w.Tdn, tb));
    HIPCHK(hipMemsetAsync(w.Tup, 0, tb, H->st));
    HIPCHK(hipMemsetAsync(w.Tdn, 0, tb, H->st));
    w.nrhs = nrhs;
    return HELM_OK;
}

// class-timed launch: HIPCHK(TIMED(H, cls, launch_expr))
struct TimedScope {
    helm_t H; int c;
    TimedScope(helm_t h, int cc) : H(h), c(cc) { if (H->timer) H->timer->begin(c, H->st); }
    ~TimedScope() { if (H->timer) H->timer->end(c, H->st); }
};
#define TIMED(H, cls, expr) ([&]() { TimedScope ts_(H, cls); return (expr); }())

// ---------------------------------------------------------------- sweeps
// yw: the strip solver's workspace (null: the handle's own, H->wk.Yw); kt: kernel timer
template <typename T>
helm_status strip_solve3(helm_t H, int s, int nrhs, const helm::IOSpec& io, void* yw, helm::KTimer* kt) {
    const auto& g = H->g;
    helm::Solve3Args<T> a;
    a.F = static_cast<const helm::cplx<T>*>(H->F) + (size_t)H->fidx[s] * g.Ny * g.Bp * g.Bp;
    a.Yw = static_cast<helm::cplx<T>*>(yw ? yw : H->wk.Yw);
    a.cy = H->t.cy;
    a.by = H->t.by;
    a.io = io;
    if (!a.io.trA || !a.io.trB || a.io.q_t < 0) {
        a.io.trA = a.io.trB = a.io.src;
        a.io.q_t = -1;
        a.io.coef = 0.0;
    }
    a.Ny = g.Ny; a.Nz = g.Nz; a.W = g.strips[s].W; a.B = a.W * g.Nz; a.Bp = g.Bp;
    a.nrhs = nrhs; a.RP = rhs_pad16(nrhs); a.Nrow = g.Nrow();
    a.Tw = a.Yw + (size_t)g.Ny * g.Bp * a.RP;     // two planes after the Ny planes of Yw
    HIPCHK(helm::launch_strip_solve3<T>(a, H->st, kt));
    return HELM_OK;
}

template <typename T>
helm_status strip_solve(helm_t H, int s, int nrhs, const helm::IOSpec& io, void* yw, helm::KTimer* kt) {
    if (H->g.dim == 3) return strip_solve3<T>(H, s, nrhs, io, yw, kt);
    if (H->fuser && std::is_same<T, float>::value) {
        helm::StripJob j;
        j.t = &H->t; j.g = &H->g; j.ch = &H->ch; j.s = s; j.fs = H->fidx[s]; j.f32 = true;
        j.F = H->F; j.Fc = H->Fc; j.Fs = H->Fs; j.Fa = H->Fa; j.Fw = H->Fw; j.Yw = yw ? yw : H->wk.Yw;
        j.nrhs = nrhs; j.io = io;
        if (!H->fuse_ev) HIPCHK(hipEventCreateWithFlags(&H->fuse_ev, hipEventDisableTiming));
        HIPCHK(H->fuser->submit(j, H->st, H->fuse_ev));
        return HELM_OK;
    }
    const auto* F = static_cast<const helm::cplx<T>*>(H->F);
    const auto* Fc = static_cast<const helm::cplx<T>*>(H->Fc);
    const auto* Fs = static_cast<const helm::cplx<T>*>(H->Fs);
    const auto* Fa = static_cast<const helm::cplx<T>*>(H->Fa);
    const auto* Fw = static_cast<const helm::cplx<T>*>(H->Fw);
    auto* Yw = static_cast<helm::cplx<T>*>(yw ? yw : H->wk.Yw);
    HIPCHK(helm::launch_strip_solve<T>(H->t, H->g, H->ch, s, H->fidx[s], F, Fc, Fs, Fa, Fw, Yw, nrhs, io,
                                       H->st, kt));
    return HELM_OK;
}

helm_status strip_solve_any(helm_t H, int s, int nrhs, const helm::IOSpec& io, void* yw = nullptr,
                            bool timed = true) {
    helm::KTimer* kt = timed ? H->kt() : nullptr;
    return H->prec == HELM_C128 ? strip_solve<double>(H, s, nrhs, io, yw, kt)
                                : strip_solve<float>(H, s, nrhs, io, yw, kt);
}

// Bytes of strip-solver workspace a solve of nrhs right-hand sides needs (the Yw buffer of
// ensure_sweep_ws: 2-D [nrhs][Ny][WP]; 3-D Ny + 2 planes of [Bp][nrhs rounded up to 16])
size_t strip_ws_bytes(helm_t H, int nrhs) {
    const auto& g = H->g;
    const size_t esz = H->prec == HELM_C128 ? sizeof(double2) : sizeof(float2);
    return g.dim == 3 ? (size_t)(g.Ny + 2) * g.Bp * rhs_pad16(nrhs) * esz : (size_t)nrhs * g.Ny * WP * esz;
}

double2* trace(double2* base, int s, int k, int nrhs, long Nrow) {
    return base + ((size_t)s * 2 + k) * nrhs * Nrow;
}

helm::IOSpec field_io(helm_t H, int s) {
    helm::IOSpec io;
    const auto& g = H->g;
    io.src_rs = g.Nrow() * g.Nx; io.src_ls = g.Nx; io.src_off = g.strips[s].a;
    io.dst_rs = g.Nrow() * g.Nx; io.dst_ls = g.Nx; io.dst_off[0] = io.dst_off[1] = g.strips[s].a;
    return io;
}

// Offset that maps strip-local column q of strip s to its place in the window of interface j
// (window column x - (beta_j - 2) for x = a_s + q); false if [x0, x0 + n) leaves the window.
bool win_off(const helm::Geom& g, int s, int j, int x0, int n, int* off) {
    const int w0 = g.beta[j] - 2;
    *off = (j - 1) * helm::IWIN - w0 + g.strips[s].a;
    return x0 >= w0 && x0 + n <= w0 + helm::IWIN;
}

// Robin transmission source of a strip (Sec. 4.4): the ghost beyond its boundary column
// q_t carries the neighbour field's Robin data, which moves (V_o - rho_j V_i) / h^2 onto
// column q_t; rho_j of interface j (column beta_j), V_o / V_i the neighbour's traces at the
// columns outside / inside the strip.
helm_status robin_source(helm_t H, int nrhs, int j, const double2* vo, const double2* vi, int q_t,
                         helm::IOSpec& io) {
    const auto& g = H->g;
    Work& w = H->wk;
    const long plane = (long)nrhs * g.Nrow();
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_robin_data(vo, vi, H->t.rho + (size_t)(j - 1) * g.Nrow(),
                                                           w.Rob + plane, nrhs, g.Nrow(),
                                                           1.0 / (g.h * g.h), H->st)));
    io.trA = w.Rob;
    io.trB = w.Rob + plane;
    io.q_t = q_t;
    io.t_cols = 1;
    io.coef = 1.0;
    return HELM_OK;
}

// Upward sweep (eq. solve_upward) for strips s0..J-1.  full: keep v^(j) on its whole core;
// otherwise only the columns the interface residuals read.  src = input field.
helm_status sweep_up(helm_t H, int nrhs, const double2* src, int s0, bool full,
                     const double2* red_src) {
    const auto& g = H->g;
    Work& w = H->wk;
    const double ih2 = 1.0 / (g.h * g.h);
    for (int s = s0; s < g.J; ++s) {
        const auto& S = g.strips[s];
        helm::IOSpec io = field_io(H, s);
        if (red_src) {
            // reduced input: columns beta_s, beta_s+1 of interface s (s >= 1)
            const int nred = 2 * (g.J - 1);
            io.src = red_src; io.src_rs = g.Nrow() * nred; io.src_ls = nred;
            io.src_lo = g.beta[s] - S.a; io.src_hi = io.src_lo + 2;
            io.src_off = 2 * (s - 1) - io.src_lo;
        } else {
            io.src = src;
            io.src_lo = S.core_lo - S.a; io.src_hi = S.core_hi - S.a;
        }
        if (s > s0 && H->trans == 1) {
            // Robin data of v^(j-1) at its columns beta_s - 1 (outside) and beta_s (inside)
            CHK(robin_source(H, nrhs, s, trace(w.Tup, s - 1, 0, nrhs, g.Nrow()),
                             trace(w.Tup, s - 1, 1, nrhs, g.Nrow()), 0, io));
        } else if (s > s0) {
            io.trA = trace(w.Tup, s - 1, 0, nrhs, g.Nrow());
            io.trB = trace(w.Tup, s - 1, 1, nrhs, g.Nrow());
            io.q_t = g.beta[s] - 1 - S.a;
            io.coef = -ih2;                                   // -2 delta d_x v, delta = 1/(2h)
        }
        io.dst = full ? w.V : w.Vw;
        io.targets_only = full ? 0 : 1;
        if (full) {
            io.o_lo[0] = S.core_lo - S.a; io.o_hi[0] = S.core_hi - S.a;
        } else {
            // window fields: the first two core columns in the window of interface s, the
            // last two in that of interface s + 1
            const long wrow = (long)(g.J - 1) * helm::IWIN;
            io.dst_rs = g.Nrow() * wrow; io.dst_ls = (int)wrow;
            bool in = true;
            if (s > 0) {                       // strip 0 has no interface on its left
                io.o_lo[0] = S.core_lo - S.a; io.o_hi[0] = io.o_lo[0] + 2;
                in = win_off(g, s, s, S.core_lo, 2, &io.dst_off[0]);
            }
            if (s < g.J - 1) {
                io.o_lo[1] = S.core_hi - 2 - S.a; io.o_hi[1] = S.core_hi - S.a;
                in = in && win_off(g, s, s + 1, S.core_hi - 2, 2, &io.dst_off[1]);
            }
            if (!in) return fail(H, HELM_EINVAL, "core columns outside the interface window");
        }
        if (s < g.J - 1) {
            io.tro0 = trace(w.Tup, s, 0, nrhs, g.Nrow());
            io.tro1 = trace(w.Tup, s, 1, nrhs, g.Nrow());
            io.qo0 = g.beta[s + 1] - 1 - S.a;
            io.qo1 = g.beta[s + 1] - S.a;
        }
        CHK(strip_solve_any(H, s, nrhs, io));
    }
    return HELM_OK;
}

// Downward sweep (eq. solve_downward) for strips J-2..0 with right-hand side g = G on
// the residual columns beta_j - 1, beta_j.  full: accumulate w^(j) on D~^(j) into dst;
// otherwise write only the columns the interface residuals read into dst.
helm_status sweep_down(helm_t H, int nrhs, double2* dst, bool full) {
    const auto& g = H->g;
    Work& w = H->wk;
    const double ih2 = 1.0 / (g.h * g.h);
    for (int s = g.J - 2; s >= 0; --s) {
        const auto& S = g.strips[s];
        helm::IOSpec io = field_io(H, s);
        const long wrow = (long)(g.J - 1) * helm::IWIN;
        io.src = full ? w.G : w.Gw;
        io.src_lo = g.beta[s + 1] - 1 - S.a; io.src_hi = io.src_lo + 2;
        if (!full) {
            io.src_rs = g.Nrow() * wrow; io.src_ls = (int)wrow;
            if (!win_off(g, s, s + 1, g.beta[s + 1] - 1, 2, &io.src_off))
                return fail(H, HELM_EINVAL, "columns outside the interface window");
            io.dst_rs = g.Nrow() * wrow; io.dst_ls = (int)wrow;
        }
        if (s < g.J - 2 && H->trans == 1) {
            // Robin data of w^(j+1) at its columns beta_{s+1} + 1 (outside) and beta_{s+1}
            // (inside)
            CHK(robin_source(H, nrhs, s + 1, trace(w.Tdn, s + 1, 1, nrhs, g.Nrow()),
                             trace(w.Tdn, s + 1, 0, nrhs, g.Nrow()), S.W - 1, io));
        } else if (s < g.J - 2) {
            io.trA = trace(w.Tdn, s + 1, 0, nrhs, g.Nrow());
            io.trB = trace(w.Tdn, s + 1, 1, nrhs, g.Nrow());
            io.q_t = g.beta[s + 1] - S.a;
            io.coef = ih2;                                     // +2 delta d_x w
        }
        io.dst = dst;
        io.targets_only = full ? 0 : 1;
        if (full) {
            io.o_lo[0] = S.kdn_lo - S.a; io.o_hi[0] = S.kdn_hi - S.a;
            io.accumulate = 1;
        } else {
            io.o_lo[0] = g.beta[s + 1] - 1 - S.a; io.o_hi[0] = io.o_lo[0] + 2;
            io.dst_off[0] = io.src_off;
            if (s > 0) {
                io.o_lo[1] = g.beta[s] + 1 - S.a; io.o_hi[1] = io.o_lo[1] + 2;
                if (!win_off(g, s, s, g.beta[s] + 1, 2, &io.dst_off[1]))
                    return fail(H, HELM_EINVAL, "columns outside the interface window");
            }
        }
        if (s > 0) {
            io.tro0 = trace(w.Tdn, s, 0, nrhs, g.Nrow());
            io.tro1 = trace(w.Tdn, s, 1, nrhs, g.Nrow());
            io.qo0 = g.beta[s] - S.a;
            io.qo1 = g.beta[s] + 1 - S.a;
        }
        CHK(strip_solve_any(H, s, nrhs, io));
    }
    return HELM_OK;
}

// out = P f = v + w  (full form, Sec. 2.1)
helm_status apply_P_full(helm_t H, int nrhs, const double2* f, double2* out) {
    CHK(ensure_sweep_ws(H, nrhs));
    const auto& g = H->g;
    Work& w = H->wk;
    CHK(sweep_up(H, nrhs, f, 0, true, nullptr));
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A_pairs(H->t, g, nrhs, H->t.rcols, g.J - 1, w.V, f, w.G, H->st)));
    HIPCHK(hipMemcpyAsync(out, w.V, field_bytes(H, nrhs), hipMemcpyDeviceToDevice, H->st));
    CHK(sweep_down(H, nrhs, out, true));
    return HELM_OK;
}

// Algorithm 3: out = (A P psi) on the reduced columns for reduced psi.  v, g and w live on
// interface windows only: the reduced sweeps write just the window columns, the residual
// stencils read just them.
helm_status apply_AP_reduced(helm_t H, int nrhs, const double2* psi, double2* out) {
    CHK(ensure_sweep_ws(H, nrhs));
    const auto& g = H->g;
    Work& w = H->wk;
    if (g.J < 2) return HELM_OK;
    // v^(1) = 0 (Algorithm 3 starts at j = 2): strip 1 never writes its window columns
    CHK(sweep_up(H, nrhs, nullptr, 1, false, psi));
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_stencil_win(0, H->t, g, nrhs, w.Vw, psi, w.Gw, nullptr, H->st)));
    CHK(sweep_down(H, nrhs, w.Ww, false));
    // h = g - A w on the reduced columns; output psi - h
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_stencil_win(1, H->t, g, nrhs, w.Ww, psi, w.Gw, out, H->st)));
    return HELM_OK;
}

// A restart's reduced right-hand side b = (r - A P r) on the reduced columns for a full field
// r, with both sweeps of P in the target-only form of Algorithm 3: g = r - A v vanishes off
// the columns beta_j - 1, beta_j and r - A (v + w) = g - A w off beta_j, beta_j + 1 (Sec. 2.1,
// exact arithmetic), so the interface windows hold all that b needs.  P r itself is added
// with the cycle's final application of P, P (r + psi) = P r + P psi.
helm_status restart_rhs_reduced(helm_t H, int nrhs, const double2* r, double2* b) {
    CHK(ensure_sweep_ws(H, nrhs));
    const auto& g = H->g;
    Work& w = H->wk;
    if (g.J < 2) return HELM_OK;
    CHK(sweep_up(H, nrhs, r, 0, false, nullptr));
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_stencil_win(3, H->t, g, nrhs, w.Vw, r, w.Gw, nullptr, H->st)));
    // Algorithm 3's upward sweeps start at the second strip and rely on the first interface's
    // window of v holding zeros where the first strip would write
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_clear_win_cols(w.Vw, (long)nrhs * g.Nrow(),
                                                               (long)(g.J - 1) * helm::IWIN, 0, helm::IWIN, H->st)));
    CHK(sweep_down(H, nrhs, w.Ww, false));
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_stencil_win(4, H->t, g, nrhs, w.Ww, nullptr, w.Gw, b, H->st)));
    return HELM_OK;
}

// ---------------------------------------------------------------- concurrent double sweep
// P_c f = v + w' - z on every core D^(j): v the upward sweep on f (eq. solve_upward), w' a
// downward sweep on f (eq. solve_downward with f~^(j) in place of the residual), z^(j) the
// strip solve of f on D^(j) and D~^(j) (the sources both chains contain).  The upward chain
// runs on the handle's stream, the downward chain and the z solves on two streams of their
// own, each with its own strip-solver workspace; f - A P_c f lives on the columns
// beta_j - 1, beta_j, where the reduced form of this sweep keeps its unknowns.

// strip solve of strip s on stream q with workspace yw
helm_status solve_on(helm_t H, hipStream_t q, int s, int nrhs, const helm::IOSpec& io, void* yw) {
    const hipStream_t keep = H->st;
    H->st = q;
    helm_status r = strip_solve_any(H, s, nrhs, io, yw);
    H->st = keep;
    return r;
}

helm_status conc_streams(helm_t H) {
    for (hipStream_t& q : H->st_c)
        if (!q) HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    for (hipEvent_t& e : H->ev_c)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return HELM_OK;
}

// Window outputs of a strip: its first two core columns into the window of interface s
// (s >= 1), its last two into that of interface s + 1 (s <= J - 2).
helm_status conc_windows(helm_t H, int s, helm::IOSpec& io) {
    const auto& g = H->g;
    const auto& S = g.strips[s];
    const long wrow = (long)(g.J - 1) * helm::IWIN;
    io.dst_rs = g.Nrow() * wrow; io.dst_ls = (int)wrow;
    io.targets_only = 1;
    int k = 0;
    bool in = true;
    if (s >= 1) {
        io.o_lo[k] = S.core_lo - S.a; io.o_hi[k] = io.o_lo[k] + 2;
        in = in && win_off(g, s, s, S.core_lo, 2, &io.dst_off[k]);
        ++k;
    }
    if (s <= g.J - 2) {
        io.o_lo[k] = S.core_hi - 2 - S.a; io.o_hi[k] = S.core_hi - S.a;
        in = in && win_off(g, s, s + 1, S.core_hi - 2, 2, &io.dst_off[k]);
        ++k;
    }
    if (!in) return fail(H, HELM_EINVAL, "core columns outside the interface window");
    return HELM_OK;
}

// The three parts of P_c src.  full: v, w', z on whole cores into dv, dw, dz (full fields);
// otherwise (src zero off the reduced columns) on the interface windows Vw, Ww, Gw.
helm_status sweep_concurrent(helm_t H, int nrhs, const double2* src, bool full, double2* dv, double2* dw,
                             double2* dz) {
    const auto& g = H->g;
    Work& w = H->wk;
    const int J = g.J;
    const double ih2 = 1.0 / (g.h * g.h);
    CHK(conc_streams(H));
    const hipStream_t qa = H->st, qb = H->st_c[0], qc = H->st_c[1];
    HIPCHK(hipEventRecord(H->ev_c[0], qa));
    HIPCHK(hipStreamWaitEvent(qb, H->ev_c[0], 0));
    HIPCHK(hipStreamWaitEvent(qc, H->ev_c[0], 0));
    // reduced input: strip J - 1 has no source on D~^(J) (so w'^(J) = 0) nor on D and D~
    const int dn_first = full ? J - 1 : J - 2;
    const int z_last = full ? J - 1 : J - 2;
    for (int i = 0; i < J; ++i) {
        {   // upward, strip i
            const int s = i;
            const auto& S = g.strips[s];
            helm::IOSpec io = field_io(H, s);
            io.src = src; io.src_lo = S.core_lo - S.a; io.src_hi = S.core_hi - S.a;
            if (s > 0) {
                io.trA = trace(w.Tup, s - 1, 0, nrhs, g.Nrow());
                io.trB = trace(w.Tup, s - 1, 1, nrhs, g.Nrow());
                io.q_t = g.beta[s] - 1 - S.a;
                io.coef = -ih2;
            }
            if (s < J - 1) {
                io.tro0 = trace(w.Tup, s, 0, nrhs, g.Nrow());
                io.tro1 = trace(w.Tup, s, 1, nrhs, g.Nrow());
                io.qo0 = g.beta[s + 1] - 1 - S.a;
                io.qo1 = g.beta[s + 1] - S.a;
            }
            if (full) {
                io.dst = dv; io.o_lo[0] = S.core_lo - S.a; io.o_hi[0] = S.core_hi - S.a;
            } else {
                io.dst = w.Vw;
                CHK(conc_windows(H, s, io));
            }
            CHK(solve_on(H, qa, s, nrhs, io, w.Yw));
        }
        if (dn_first - i >= 0) {   // downward, strip dn_first - i
            const int s = dn_first - i;
            const auto& S = g.strips[s];
            helm::IOSpec io = field_io(H, s);
            io.src = src; io.src_lo = S.kdn_lo - S.a; io.src_hi = S.kdn_hi - S.a;
            if (s < dn_first) {
                io.trA = trace(w.Tdn, s + 1, 0, nrhs, g.Nrow());
                io.trB = trace(w.Tdn, s + 1, 1, nrhs, g.Nrow());
                io.q_t = g.beta[s + 1] - S.a;
                io.coef = ih2;
            }
            if (s > 0) {
                io.tro0 = trace(w.Tdn, s, 0, nrhs, g.Nrow());
                io.tro1 = trace(w.Tdn, s, 1, nrhs, g.Nrow());
                io.qo0 = g.beta[s] - S.a;
                io.qo1 = g.beta[s] + 1 - S.a;
            }
            if (full) {
                io.dst = dw; io.o_lo[0] = S.core_lo - S.a; io.o_hi[0] = S.core_hi - S.a;
            } else {
                io.dst = w.Ww;
                CHK(conc_windows(H, s, io));
            }
            CHK(solve_on(H, qb, s, nrhs, io, w.Yw2));
        }
        if (i <= z_last) {   // the strip's own sources, strip i
            const int s = i;
            const auto& S = g.strips[s];
            helm::IOSpec io = field_io(H, s);
            io.src = src;
            io.src_lo = std::max(S.core_lo, S.kdn_lo) - S.a;
            io.src_hi = std::min(S.core_hi, S.kdn_hi) - S.a;
            if (full) {
                io.dst = dz; io.o_lo[0] = S.core_lo - S.a; io.o_hi[0] = S.core_hi - S.a;
            } else {
                io.dst = w.Gw;
                CHK(conc_windows(H, s, io));
            }
            CHK(solve_on(H, qc, s, nrhs, io, w.Yw3));
        }
    }
    HIPCHK(hipEventRecord(H->ev_c[1], qb));
    HIPCHK(hipEventRecord(H->ev_c[2], qc));
    HIPCHK(hipStreamWaitEvent(qa, H->ev_c[1], 0));
    HIPCHK(hipStreamWaitEvent(qa, H->ev_c[2], 0));
    return HELM_OK;
}

// out = P_c f on the whole grid
helm_status apply_Pc_full(helm_t H, int nrhs, const double2* f, double2* out) {
    CHK(ensure_sweep_ws(H, nrhs));
    Work& w = H->wk;
    CHK(sweep_concurrent(H, nrhs, f, true, w.V, w.Wf, w.G));
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_sum_diff(w.V, w.Wf, w.G, out, (long)nrhs * H->g.Nrow() * H->g.Nx, H->st)));
    return HELM_OK;
}

// out = (A P_c psi) on the columns beta_j - 1, beta_j, for psi given there
helm_status apply_APc_reduced(helm_t H, int nrhs, const double2* psi, double2* out) {
    CHK(ensure_sweep_ws(H, nrhs));
    const auto& g = H->g;
    Work& w = H->wk;
    if (g.J < 2) return HELM_OK;
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_scatter_cols(psi, H->t.rcols, 2 * (g.J - 1), nrhs, g.Nrow(), g.Nx, w.PsiC, H->st)));
    CHK(sweep_concurrent(H, nrhs, w.PsiC, false, nullptr, nullptr, nullptr));
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_stencil_win(2, H->t, g, nrhs, w.Vw, w.Ww, w.Gw, out, H->st)));
    return HELM_OK;
}

// The starting point of the reduced form of P_c: u~ from independent strip solves of f on
// D^(j), kept on D^(j) (f - A u~ then lives on the columns beta_j - 1, beta_j); the solves
// go round the three streams
helm_status conc_setup(helm_t H, int nrhs, const double2* f, double2* ut) {
    const auto& g = H->g;
    Work& w = H->wk;
    CHK(conc_streams(H));
    const hipStream_t qs[3] = {H->st, H->st_c[0], H->st_c[1]};
    void* yws[3] = {w.Yw, w.Yw2, w.Yw3};
    HIPCHK(hipEventRecord(H->ev_c[0], H->st));
    HIPCHK(hipStreamWaitEvent(qs[1], H->ev_c[0], 0));
    HIPCHK(hipStreamWaitEvent(qs[2], H->ev_c[0], 0));
    for (int s = 0; s < g.J; ++s) {
        const auto& S = g.strips[s];
        helm::IOSpec io = field_io(H, s);
        io.src = f;
        io.src_lo = S.core_lo - S.a; io.src_hi = S.core_hi - S.a;
        io.dst = ut;
        io.o_lo[0] = io.src_lo; io.o_hi[0] = io.src_hi;
        CHK(solve_on(H, qs[s % 3], s, nrhs, io, yws[s % 3]));
    }
    HIPCHK(hipEventRecord(H->ev_c[1], qs[1]));
    HIPCHK(hipEventRecord(H->ev_c[2], qs[2]));
    HIPCHK(hipStreamWaitEvent(H->st, H->ev_c[1], 0));
    HIPCHK(hipStreamWaitEvent(H->st, H->ev_c[2], 0));
    return HELM_OK;
}

// the preconditioner of the handle's sweep on whole fields
// Concurrent sweeps with Robin transmission (Sec. 3.1; conditions of Sec. 4.4): step
// n = 1..J updates subdomains n and J + 1 - n, each from f on its core and the Robin data
// of both neighbours' solutions of earlier steps (none for a neighbour not yet solved);
// where the chains meet, both right-hand sides are formed before either subdomain is
// solved, so each takes the other's data from the step before.  The latest solutions of
// even and odd subdomains live in two fields (neighbours' extra columns overlap); v takes
// every core from its subdomain's field.  A step's two strip solves are one multi-problem
// launch in complex64.
helm_status apply_PcR_full(helm_t H, int nrhs, const double2* f, double2* out) {
    CHK(ensure_sweep_ws(H, nrhs));
    const auto& g = H->g;
    Work& w = H->wk;
    const int J = g.J;
    const double ih2 = 1.0 / (g.h * g.h);
    double2* fld[2] = {w.V, w.G};
    const size_t rstride = (size_t)nrhs * g.Nrow() * WP;
    std::vector<char> done(J, 0);
    for (int n = 1; n <= J; ++n) {
        int upd[2] = {n - 1, J - n};
        const int nu = upd[0] == upd[1] ? 1 : 2;
        helm::IOSpec io[2];
        for (int k = 0; k < nu; ++k) {
            const int s = upd[k];
            const auto& S = g.strips[s];
            const double2* L = s > 0 && done[s - 1] ? fld[(s - 1) & 1] : nullptr;
            const double2* R = s < J - 1 && done[s + 1] ? fld[(s + 1) & 1] : nullptr;
            const double2* rl = H->t.rho + (size_t)(s > 0 ? s - 1 : 0) * g.Nrow();
            const double2* rr = H->t.rho + (size_t)(s < J - 1 ? s : 0) * g.Nrow();
            double2* rhs = w.RobR + k * rstride;
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_robin_rhs(f, L, R, rl, rr, rhs, nrhs, (int)g.Nrow(), g.Nx, S.a,
                                                                  S.W, S.core_lo - S.a, S.core_hi - S.a, ih2, H->st)));
            io[k] = field_io(H, s);
            io[k].src = rhs; io[k].src_rs = g.Nrow() * S.W; io[k].src_ls = S.W; io[k].src_off = 0;
            io[k].src_lo = 0; io[k].src_hi = S.W;
            io[k].dst = fld[s & 1];
            io[k].o_lo[0] = 0; io[k].o_hi[0] = S.W;
        }
        bool fused = false;
        if (nu == 2 && H->prec == HELM_MIXED_C64 && !H->kt()) {
            helm::StripJob jb[2];
            for (int k = 0; k < 2; ++k) {
                const int s = upd[k];
                jb[k].t = &H->t; jb[k].g = &H->g; jb[k].ch = &H->ch; jb[k].s = s; jb[k].fs = H->fidx[s];
                jb[k].f32 = true; jb[k].F = H->F; jb[k].Fc = H->Fc; jb[k].Fs = H->Fs;
                jb[k].Fa = H->Fa; jb[k].Fw = H->Fw;
                jb[k].Yw = k == 0 ? w.Yw : w.Yw2; jb[k].nrhs = nrhs; jb[k].io = io[k];
            }
            if (helm::strip_jobs_fusable(jb, 2)) {
                HIPCHK(helm::launch_strip_solve_multi(jb, 2, H->st, nullptr));
                fused = true;
            }
        }
        if (!fused)
            for (int k = 0; k < nu; ++k) CHK(strip_solve_any(H, upd[k], nrhs, io[k]));
        for (int k = 0; k < nu; ++k) done[upd[k]] = 1;
    }
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_parity_pick(fld[0], fld[1], H->colpar, out, nrhs, g.Nrow(), g.Nx, H->st)));
    return HELM_OK;
}

helm_status apply_P_any(helm_t H, int nrhs, const double2* f, double2* out) {
    if (H->sweep == 1 && H->trans == 1) return apply_PcR_full(H, nrhs, f, out);
    return H->sweep == 1 ? apply_Pc_full(H, nrhs, f, out) : apply_P_full(H, nrhs, f, out);
}

// Algorithm 2: u~ on D~^(j) from independent strip solves with f on D~^(j).
helm_status reduced_setup(helm_t H, int nrhs, const double2* f, double2* ut) {
    const auto& g = H->g;
    for (int s = 0; s < g.J; ++s) {
        const auto& S = g.strips[s];
        helm::IOSpec io = field_io(H, s);
        io.src = f;
        io.src_lo = S.kdn_lo - S.a; io.src_hi = S.kdn_hi - S.a;
        io.dst = ut;
        io.o_lo[0] = io.src_lo; io.o_hi[0] = io.src_hi;
        CHK(strip_solve_any(H, s, nrhs, io));
    }
    return HELM_OK;
}

// ---------------------------------------------------------------- GMRES
struct Givens {
    int m = 0;
    std::vector<cd> R;      // m x m upper triangular, column-major
    std::vector<double> c;
    std::vector<cd> sn, gv;
    int k = 0;
    bool done = false;
    double res = 0.0;
    void init(int mm, double beta) {
        m = mm; R.assign((size_t)m * m, 0.0); c.assign(m, 0.0); sn.assign(m, 0.0);
        gv.assign(m + 1, 0.0); gv[0] = beta; k = 0; done = false; res = beta;
    }
    // add Hessenberg column k (entries 0..k from CGS, hk1 = ||w||)
    void push(const cd* h, double hk1) {
        std::vector<cd> col(k + 2);
        for (int i = 0; i <= k; ++i) col[i] = h[i];
        col[k + 1] = hk1;
        for (int i = 0; i < k; ++i) {
            const cd a = col[i], b = col[i + 1];
            col[i] = c[i] * a + sn[i] * b;
            col[i + 1] = -std::conj(sn[i]) * a + c[i] * b;
        }
        const cd a = col[k];
        const double b = std::abs(col[k + 1]);
        const double t = std::hypot(std::abs(a), b);
        double ck;
        cd sk;
        if (std::abs(a) == 0.0) { ck = 0.0; sk = 1.0; }
        else { ck = std::abs(a) / t; sk = (a / std::abs(a)) * std::conj(col[k + 1]) / t; }
        c[k] = ck; sn[k] = sk;
        col[k] = ck * a + sk * col[k + 1];
        for (int i = 0; i <= k; ++i) R[(size_t)k * m + i] = col[i];
        gv[k + 1] = -std::conj(sk) * gv[k];
        gv[k] = ck * gv[k];
        res = std::abs(gv[k + 1]);
        ++k;
    }
    std::vector<cd> solve(int kk) const {
        std::vector<cd> y(kk);
        for (int i = kk - 1; i >= 0; --i) {
            cd s = gv[i];
            for (int j = i + 1; j < kk; ++j) s -= R[(size_t)j * m + i] * y[j];
            const cd d = R[(size_t)i * m + i];
            y[i] = (std::abs(d) > 0.0) ? s / d : 0.0;
        }
        return y;
    }
};

helm_status ensure_gmres_ws(helm_t H, int nrhs, long n, int mwant) {
    Work& w = H->wk;
    if (w.basis && w.n == n && w.mcap >= mwant && w.gnrhs >= nrhs) return HELM_OK;
    dfree(w.basis); dfree(w.w); dfree(w.h1); dfree(w.h2); dfree(w.nrm); dfree(w.partial);
    dfree(w.npartial); dfree(w.y); dfree(w.red); dfree(w.apin); dfree(w.basis_old);
    dfree(w.R); dfree(w.Ut);
    w.basis = w.w = w.h1 = w.h2 = w.y = w.red = w.apin = w.partial = w.basis_old = nullptr;
    w.R = w.Ut = nullptr;
    w.mcap_old = 0;
    w.gnrhs = 0;
    w.nrm = w.npartial = nullptr;
    H->ws_epoch += 1;
    size_t freeb = 0, totb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totb));
    const size_t vb = (size_t)nrhs * n * sizeof(double2);
    size_t fit = vb ? (size_t)(0.8 * (double)freeb) / vb : (size_t)mwant + 3;
    int m = (int)std::min<size_t>((size_t)mwant, fit > 3 ? fit - 3 : 1);
    if (m < 1) return fail(H, HELM_ENOMEM, "not enough device memory for the GMRES basis");
    CHK(dmalloc(H, &w.basis, vb * (m + 1)));
    CHK(dmalloc(H, &w.w, vb));
    CHK(dmalloc(H, &w.red, vb));
    CHK(dmalloc(H, &w.apin, vb));
    CHK(dmalloc(H, &w.h1, (size_t)nrhs * (m + 1) * sizeof(double2)));
    CHK(dmalloc(H, &w.h2, (size_t)nrhs * (m + 1) * sizeof(double2)));
    CHK(dmalloc(H, &w.y, (size_t)nrhs * (m + 1) * sizeof(double2)));
    CHK(dmalloc(H, &w.nrm, (size_t)nrhs * sizeof(double)));
    const int nb = helm::dots_blocks(std::max(n, H->g.Nrow() * H->g.Nx));
    CHK(dmalloc(H, &w.partial, (size_t)nb * nrhs * (m + 1) * sizeof(double2)));
    CHK(dmalloc(H, &w.npartial, (size_t)nb * nrhs * sizeof(double)));
    CHK(dmalloc(H, &w.R, field_bytes(H, nrhs)));
    CHK(dmalloc(H, &w.Ut, field_bytes(H, nrhs)));
    w.mcap = m;
    w.n = n;
    w.gnrhs = nrhs;
    return HELM_OK;
}

// the reduced operator of the handle's sweep (Algorithm 3, or its concurrent counterpart)
helm_status apply_AP_red(helm_t H, int nrhs, const double2* x, double2* out) {
    return H->sweep == 1 ? apply_APc_reduced(H, nrhs, x, out) : apply_AP_reduced(H, nrhs, x, out);
}

// columns of the reduced unknowns: beta_j, beta_j + 1 (P), beta_j - 1, beta_j (P_c)
const int* red_cols(helm_t H) { return H->sweep == 1 ? H->t.rcols : H->t.redcols; }

// Destroys one captured reduced operator (every one: slot < 0) once its last replay has
// completed.
helm_status drop_graph(helm_t H, int slot = -1) {
    bool any = false;
    for (int i = 0; i < helm_problem::NGRAPH; ++i) any = any || ((slot < 0 || i == slot) && H->apg[i].exec);
    if (!any) return HELM_OK;
    HIPCHK(H->st ? hipStreamSynchronize(H->st) : hipDeviceSynchronize());
    for (int i = 0; i < helm_problem::NGRAPH; ++i) {
        if ((slot >= 0 && i != slot) || !H->apg[i].exec) continue;
        HIPCHK(hipGraphExecDestroy(H->apg[i].exec));
        H->apg[i] = helm_problem::ApGraph();
    }
    return HELM_OK;
}

// operator of the GMRES space: full = A P on the padded grid, reduced = Algorithm 3
helm_status apply_op(helm_t H, int nrhs, const double2* x, double2* out) {
    H->stat_ap += 1;
    if (H->mode == HELM_FULL) {
        CHK(apply_P_any(H, nrhs, x, H->wk.PF));
        HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A(H->t, H->g, nrhs, H->wk.PF, nullptr, out, H->st)));
        return HELM_OK;
    }
    // kernel timing brackets launches with events, which a graph replay cannot time here
    // (hipEventElapsedTime rejects events recorded by graph nodes): timed runs go eagerly
    if (!H->use_graph || H->timer || H->fuser) return apply_AP_red(H, nrhs, x, out);
    // graph replay: the captured launches read the fixed buffer apin and write `out`
    Work& w = H->wk;
    CHK(ensure_sweep_ws(H, nrhs));
    const size_t bytes = (size_t)nrhs * H->g.Nrow() * 2 * (H->g.J - 1) * sizeof(double2);
    if (x != w.apin) HIPCHK(hipMemcpyAsync(w.apin, x, bytes, hipMemcpyDeviceToDevice, H->st));
    int slot = -1, lru = 0;
    for (int i = 0; i < helm_problem::NGRAPH; ++i) {
        const auto& e = H->apg[i];
        if (e.exec && e.nrhs == nrhs && e.out == out && e.epoch == H->ws_epoch) slot = i;
        if (H->apg[i].used < H->apg[lru].used) lru = i;
    }
    if (slot < 0) {
        slot = lru;
        CHK(drop_graph(H, slot));
        if (!H->cap_st) HIPCHK(hipStreamCreateWithFlags(&H->cap_st, hipStreamNonBlocking));
        // the captured work only reads buffers written before the replay on st; nothing is
        // executed during the capture itself
        hipGraph_t graph = nullptr;
        const hipStream_t user_st = H->st;
        HIPCHK(hipStreamBeginCapture(H->cap_st, hipStreamCaptureModeRelaxed));
        H->st = H->cap_st;
        helm_status cs = apply_AP_red(H, nrhs, w.apin, out);
        H->st = user_st;
        hipError_t ce = hipStreamEndCapture(H->cap_st, &graph);
        if (cs != HELM_OK) { if (graph) (void)hipGraphDestroy(graph); return cs; }
        HIPCHK(ce);
        auto& e = H->apg[slot];
        hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ie);
        e.nrhs = nrhs; e.out = out; e.epoch = H->ws_epoch;
    }
    H->apg[slot].used = ++H->ap_tick;
    HIPCHK(hipGraphLaunch(H->apg[slot].exec, H->st));
    return HELM_OK;
}

helm_status norms(helm_t H, const double2* v, int nrhs, long n, std::vector<double>& out) {
    Work& w = H->wk;
    const int nb = helm::dots_blocks(n);
    HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_norms(v, nrhs, n, w.npartial, nb, w.nrm, H->st)));
    out.resize(nrhs);
    HIPCHK(hipMemcpyAsync(out.data(), w.nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    return HELM_OK;
}

// Recycled space of a restart (reduced mode): the previous cycle's basis V (nv vectors per
// right-hand side block; k_r + 1 of them used by right-hand side r) with M V_k = V_{k+1} Hr.
// With Hr = Qh R (Qh orthonormal columns), C = V_{k+1} Qh is orthonormal and M U = C for
// U = V_k R^{-1}.  The new cycle runs Arnoldi on (I - C C^H) M (B_j = C^H M v_j recorded per
// step) and its solution gains U (a - B y), a = C^H b of the starting residual: GMRES over
// span(U) + the new Krylov space (the GCRO form of augmented restarting).
struct Aug {
    const double2* V = nullptr;
    int nv = 0;
    std::vector<int> k;                   // per rhs: size of the recycled space
    std::vector<std::vector<cd>> Qh;      // per rhs (k + 1) x k, column-major
    std::vector<std::vector<cd>> R;       // per rhs k x k upper triangular, column-major
    std::vector<std::vector<cd>> a;       // per rhs C^H b
    std::vector<std::vector<cd>> B;       // per rhs, k entries per Arnoldi step
};

// One GMRES(m) cycle on op(y) = b.  b is copied into the basis.  Each right-hand side
// stops when its residual is <= target[r]; returns y (device, [nrhs][n]) and per-rhs
// iteration counts.  active[r] == false rhs take no part (y = 0).
// w.w = op(v) for the right-hand sides still iterating; rows of converged ones are zero.
// When their number fits fewer groups of 16 than nrhs, they are gathered into the fixed
// input panel apin (rounded up to a multiple of 16, the padding zero: the operator is linear
// and acts on every right-hand side alone, so each result is bitwise the one of the full
// panel), the operator runs on that smaller panel, and the results move back to their rows
// from the last one down (row i goes to act[i] >= i, never onto a row still to be read).
helm_status apply_op_active(helm_t H, int nrhs, long n, const std::vector<Givens>& gv, const double2* v) {
    Work& w = H->wk;
    std::vector<int> act;
    for (int r = 0; r < nrhs; ++r)
        if (!gv[r].done) act.push_back(r);
    const int nact = (int)act.size();
    const int npad = std::min(nrhs, (nact + 15) / 16 * 16);
    H->stat_panel_full += nrhs;
    H->stat_panel += npad < nrhs && nact > 0 ? npad : nrhs;
    if (npad >= nrhs || nact == 0) return apply_op(H, nrhs, v, w.w);
    const size_t row = (size_t)n * sizeof(double2);
    for (int i = 0; i < nact;) {                     // runs of consecutive right-hand sides
        int e = i + 1;
        while (e < nact && act[e] == act[e - 1] + 1) ++e;
        HIPCHK(hipMemcpyAsync(w.apin + (size_t)i * n, v + (size_t)act[i] * n, row * (e - i),
                              hipMemcpyDeviceToDevice, H->st));
        i = e;
    }
    if (npad > nact) HIPCHK(hipMemsetAsync(w.apin + (size_t)nact * n, 0, row * (npad - nact), H->st));
    CHK(apply_op(H, npad, w.apin, w.w));
    for (int i = nact - 1; i >= 0; --i)
        if (act[i] != i)
            HIPCHK(hipMemcpyAsync(w.w + (size_t)act[i] * n, w.w + (size_t)i * n, row, hipMemcpyDeviceToDevice,
                                  H->st));
    for (int r = 0, i = 0; r < nrhs; ++r) {
        if (i < nact && act[i] == r) { ++i; continue; }
        HIPCHK(hipMemsetAsync(w.w + (size_t)r * n, 0, row, H->st));
    }
    return HELM_OK;
}

helm_status gmres_cycle(helm_t H, int nrhs, long n, const double2* b, const std::vector<double>& bnorm,
                        const std::vector<double>& target, int maxit, double2* yout,
                        std::vector<int>& its, std::vector<double>& resid,
                        std::vector<std::vector<cd>>* hess = nullptr, Aug* aug = nullptr) {
    Work& w = H->wk;
    const int m = std::min(maxit, w.mcap);
    const size_t vs = (size_t)nrhs * n;
    std::vector<Givens> gv(nrhs);
    std::vector<double> scale(nrhs);
    its.assign(nrhs, 0);
    resid.assign(nrhs, 0.0);
    // Hessenberg columns of each right-hand side, column k with entries 0 .. k + 1
    if (hess) hess->assign(nrhs, std::vector<cd>());
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
        gv[r].init(m, bnorm[r]);
        gv[r].done = !(bnorm[r] > target[r]);
        resid[r] = bnorm[r];
        all = all && gv[r].done;
    }
    // V_0 = b / ||b||
    {
        HIPCHK(hipMemcpyAsync(w.nrm, bnorm.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, H->st));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_scale(b, w.nrm, w.basis, nrhs, n, H->st)));
        HIPCHK(hipStreamSynchronize(H->st));
    }
    int k = 0;
    std::vector<double2> hh1((size_t)nrhs * (m + 1)), hh2((size_t)nrhs * (m + 1));
    std::vector<double2> aug_d, aug_e;
    std::vector<double> nr(nrhs);
    const int nb = helm::dots_blocks(n);
    while (!all && k < m) {
        double2* vk = w.basis + (size_t)k * vs;
        CHK(apply_op_active(H, nrhs, n, gv, vk));
        if (aug) {
            // w <- (I - C C^H) w: B_j = C^H w = Qh^H (V^H w), w -= V (Qh B_j)
            const int anv = aug->nv;
            HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_dots(aug->V, anv, w.w, nrhs, n, w.partial, nb, w.h1, H->st)));
            // host buffers outlive the step (the upload below completes at the step's sync)
            std::vector<double2>& d = aug_d;
            std::vector<double2>& e = aug_e;
            d.assign((size_t)nrhs * anv, make_double2(0, 0));
            e.assign((size_t)nrhs * anv, make_double2(0, 0));
            HIPCHK(hipMemcpyAsync(d.data(), w.h1, d.size() * sizeof(double2), hipMemcpyDeviceToHost, H->st));
            HIPCHK(hipStreamSynchronize(H->st));
            for (int r = 0; r < nrhs; ++r) {
                const int kr = aug->k[r];
                if (gv[r].done || kr < 1) continue;
                const std::vector<cd>& Q = aug->Qh[r];
                for (int i = 0; i < kr; ++i) {
                    cd bj = 0.0;
                    for (int q = 0; q <= kr; ++q)
                        bj += std::conj(Q[(size_t)i * (kr + 1) + q]) * cd(d[(size_t)r * anv + q].x, d[(size_t)r * anv + q].y);
                    aug->B[r].push_back(bj);
                }
                const cd* bj = aug->B[r].data() + aug->B[r].size() - kr;
                for (int q = 0; q <= kr; ++q) {
                    cd acc = 0.0;
                    for (int i = 0; i < kr; ++i) acc += Q[(size_t)i * (kr + 1) + q] * bj[i];
                    e[(size_t)r * anv + q] = make_double2(acc.real(), acc.imag());
                }
            }
            HIPCHK(hipMemcpyAsync(w.h2, e.data(), e.size() * sizeof(double2), hipMemcpyHostToDevice, H->st));
            HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_update(aug->V, anv, w.h2, w.w, nrhs, n, H->st)));
        }
        const int nv = k + 1;
        // classical Gram-Schmidt, twice
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_dots(w.basis, nv, w.w, nrhs, n, w.partial, nb, w.h1, H->st)));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_update(w.basis, nv, w.h1, w.w, nrhs, n, H->st)));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_dots(w.basis, nv, w.w, nrhs, n, w.partial, nb, w.h2, H->st)));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_update(w.basis, nv, w.h2, w.w, nrhs, n, H->st)));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_norms(w.w, nrhs, n, w.npartial, nb, w.nrm, H->st)));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_scale(w.w, w.nrm, w.basis + (size_t)(k + 1) * vs, nrhs, n, H->st)));
        HIPCHK(hipMemcpyAsync(hh1.data(), w.h1, (size_t)nrhs * nv * sizeof(double2), hipMemcpyDeviceToHost, H->st));
        HIPCHK(hipMemcpyAsync(hh2.data(), w.h2, (size_t)nrhs * nv * sizeof(double2), hipMemcpyDeviceToHost, H->st));
        HIPCHK(hipMemcpyAsync(nr.data(), w.nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, H->st));
        HIPCHK(hipStreamSynchronize(H->st));
        all = true;
        for (int r = 0; r < nrhs; ++r) {
            Givens& G = gv[r];
            if (!G.done) {
                std::vector<cd> col(nv);
                for (int i = 0; i < nv; ++i) {
                    const double2 a = hh1[(size_t)r * nv + i], c2 = hh2[(size_t)r * nv + i];
                    col[i] = cd(a.x + c2.x, a.y + c2.y);
                }
                if (hess) {
                    for (int i = 0; i < nv; ++i) (*hess)[r].push_back(col[i]);
                    (*hess)[r].push_back(cd(nr[r], 0.0));
                }
                G.push(col.data(), nr[r]);
                its[r] = G.k;
                resid[r] = G.res;
                if (trace_on() && r == 0)
                    std::fprintf(stderr, "[helm] gmres k=%d rhs0 res=%.3e target=%.3e hnext=%.3e\n", G.k,
                                 G.res, target[r], nr[r]);
                if (G.res <= target[r] || !(nr[r] > 0.0)) G.done = true;
            }
            all = all && G.done;
        }
        ++k;
    }
    // y for each rhs from its own k, zero-padded to the k basis vectors built
    const int nvec = std::max(k, 1);
    std::vector<double2> yh((size_t)nrhs * nvec, make_double2(0, 0));
    for (int r = 0; r < nrhs; ++r) {
        std::vector<cd> y = gv[r].solve(gv[r].k);
        for (int i = 0; i < (int)y.size(); ++i) yh[(size_t)r * nvec + i] = make_double2(y[i].real(), y[i].imag());
    }
    HIPCHK(hipMemcpyAsync(w.y, yh.data(), yh.size() * sizeof(double2), hipMemcpyHostToDevice, H->st));
    HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_lincomb(w.basis, nvec, w.y, yout, nrhs, n, 0, H->st)));
    HIPCHK(hipStreamSynchronize(H->st));
    if (aug) {
        // + U (a - B y) = V_k R^{-1} (a - B y)
        const int anv = aug->nv;
        std::vector<double2> gco((size_t)nrhs * anv, make_double2(0, 0));
        for (int r = 0; r < nrhs; ++r) {
            const int kr = aug->k[r];
            if (kr < 1) continue;
            std::vector<cd> y = gv[r].solve(gv[r].k);
            std::vector<cd> t = aug->a[r];
            for (int j = 0; j < (int)y.size() && (size_t)(j + 1) * kr <= aug->B[r].size(); ++j)
                for (int i = 0; i < kr; ++i) t[i] -= aug->B[r][(size_t)j * kr + i] * y[j];
            const std::vector<cd>& R = aug->R[r];
            for (int i = kr - 1; i >= 0; --i) {
                cd acc = t[i];
                for (int j = i + 1; j < kr; ++j) acc -= R[(size_t)j * kr + i] * t[j];
                t[i] = acc / R[(size_t)i * kr + i];
            }
            for (int i = 0; i < kr; ++i) gco[(size_t)r * anv + i] = make_double2(t[i].real(), t[i].imag());
        }
        HIPCHK(hipMemcpyAsync(w.y, gco.data(), gco.size() * sizeof(double2), hipMemcpyHostToDevice, H->st));
        HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_lincomb(aug->V, anv, w.y, yout, nrhs, n, 1, H->st)));
        HIPCHK(hipStreamSynchronize(H->st));
    }
    return HELM_OK;
}

// Restart in reduced mode: from the previous cycle's basis V (in w.basis) and Hessenberg
// matrices, the recycled space of the coming cycle (see Aug): Hr = Qh R by modified
// Gram-Schmidt on the host (the space is cut where R loses rank), a = C^H b, and the new
// starting residual b <- b - C a.  The previous basis is then moved to w.basis_old so that
// the coming cycle builds its own in w.basis.  Returns with aug.nv = 0 (no recycling) when
// there is nothing to recycle or no memory for the second basis.
helm_status build_aug(helm_t H, int nrhs, long n, double2* b, const std::vector<std::vector<cd>>& hess,
                      const std::vector<int>& kprev, Aug& aug) {
    Work& w = H->wk;
    aug = Aug();
    int kmax = 0;
    for (int r = 0; r < nrhs; ++r) kmax = std::max(kmax, kprev[r]);
    // a short first cycle is cheap to rebuild: recycling pays for its extra dot products
    // against the old basis only after a long one (measured at 2000^2: first cycles of
    // about 10 steps gained 0.3 iterations on average but no lockstep step, and lost 5 to
    // 10 ms per solve; first cycles of 25 to 33 steps saved 6 to 7 steps)
    constexpr int RECYCLE_MIN_K = 16;
    if (kmax < RECYCLE_MIN_K || (int)hess.size() != nrhs) return HELM_OK;
    if (!w.basis_old || w.mcap_old < w.mcap) {
        dfree(w.basis_old);
        w.basis_old = nullptr;
        w.mcap_old = 0;
        // the same capacity as w.basis (the two buffers are swapped below)
        if (hipMalloc((void**)&w.basis_old, (size_t)w.gnrhs * n * sizeof(double2) * (w.mcap + 1)) != hipSuccess) {
            (void)hipGetLastError();
            w.basis_old = nullptr;
            return HELM_OK;                      // no room: a plain restart
        }
        w.mcap_old = w.mcap;
    }
    const int nv = kmax + 1;
    const int nb = helm::dots_blocks(n);
    std::vector<double2> c((size_t)nrhs * nv);
    HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_dots(w.basis, nv, b, nrhs, n, w.partial, nb, w.h1, H->st)));
    HIPCHK(hipMemcpyAsync(c.data(), w.h1, c.size() * sizeof(double2), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    aug.k.assign(nrhs, 0);
    aug.Qh.assign(nrhs, {});
    aug.R.assign(nrhs, {});
    aug.a.assign(nrhs, {});
    aug.B.assign(nrhs, {});
    std::vector<double2> e((size_t)nrhs * nv, make_double2(0, 0));
    for (int r = 0; r < nrhs; ++r) {
        int k = kprev[r];
        if (k < 1 || (int)hess[r].size() < k * (k + 3) / 2) continue;
        std::vector<cd> Hm((size_t)(k + 1) * k, 0.0);
        size_t pos = 0;
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= j + 1; ++i) Hm[(size_t)j * (k + 1) + i] = hess[r][pos++];
        // modified Gram-Schmidt: Hm = Q R
        double hnorm = 0.0;
        for (const cd& v : Hm) hnorm = std::max(hnorm, std::abs(v));
        std::vector<cd> Q = Hm, R((size_t)k * k, 0.0);
        int kk = 0;
        for (int j = 0; j < k; ++j) {
            cd* qj = Q.data() + (size_t)j * (k + 1);
            for (int i = 0; i < j; ++i) {
                const cd* qi = Q.data() + (size_t)i * (k + 1);
                cd dot = 0.0;
                for (int q = 0; q <= k; ++q) dot += std::conj(qi[q]) * qj[q];
                R[(size_t)j * k + i] = dot;
                for (int q = 0; q <= k; ++q) qj[q] -= dot * qi[q];
            }
            double nrm = 0.0;
            for (int q = 0; q <= k; ++q) nrm += std::norm(qj[q]);
            nrm = std::sqrt(nrm);
            if (!(nrm > 1e-12 * hnorm)) break;   // rank lost: recycle the leading j columns
            R[(size_t)j * k + j] = nrm;
            for (int q = 0; q <= k; ++q) qj[q] /= nrm;
            kk = j + 1;
        }
        if (kk < 1) continue;
        // keep the leading kk columns; V_{kk+1} spans them (Hessenberg structure)
        std::vector<cd> Qk((size_t)(kk + 1) * kk), Rk((size_t)kk * kk);
        for (int j = 0; j < kk; ++j) {
            for (int q = 0; q <= kk; ++q) Qk[(size_t)j * (kk + 1) + q] = Q[(size_t)j * (k + 1) + q];
            for (int i = 0; i <= j; ++i) Rk[(size_t)j * kk + i] = R[(size_t)j * k + i];
        }
        std::vector<cd> av(kk, 0.0);
        for (int i = 0; i < kk; ++i)
            for (int q = 0; q <= kk; ++q)
                av[i] += std::conj(Qk[(size_t)i * (kk + 1) + q]) * cd(c[(size_t)r * nv + q].x, c[(size_t)r * nv + q].y);
        for (int q = 0; q <= kk; ++q) {
            cd acc = 0.0;
            for (int i = 0; i < kk; ++i) acc += Qk[(size_t)i * (kk + 1) + q] * av[i];
            e[(size_t)r * nv + q] = make_double2(acc.real(), acc.imag());
        }
        aug.k[r] = kk;
        aug.Qh[r] = std::move(Qk);
        aug.R[r] = std::move(Rk);
        aug.a[r] = std::move(av);
    }
    HIPCHK(hipMemcpyAsync(w.h2, e.data(), e.size() * sizeof(double2), hipMemcpyHostToDevice, H->st));
    HIPCHK(TIMED(H, helm::K_GMRES, helm::launch_update(w.basis, nv, w.h2, b, nrhs, n, H->st)));
    HIPCHK(hipStreamSynchronize(H->st));
    std::swap(w.basis, w.basis_old);
    aug.V = w.basis_old;
    aug.nv = nv;
    return HELM_OK;
}

// first-cycle stop of the complex64 path, relative to the rounding noise Algorithm 2 leaves
// off the reduced columns.  The true residual after a first cycle run to tol stalls at 4 to
// 7 times that noise (2000^2 layers: noise 9.1e-6, stall 6.4e-5; 1000^2 lens: 6.0e-6 and
// 2.2e-5 of ||f||), so the cycle stops at 3 times it: iterating further gains nothing, the
// restart starts from the stall anyway
#ifndef FLOOR_PER_NOISE
#define FLOOR_PER_NOISE 3.0
#endif

helm_status solve_impl(helm_t H, int nrhs, const double2* f, double2* u, double tol,
                       int* iters, double* relres) {
    const auto& g = H->g;
    CHK(ensure_sweep_ws(H, nrhs));
    Work& w = H->wk;
    const long nfull = g.Nrow() * g.Nx;
    const int nred = 2 * (g.J - 1);
    const bool reduced = H->mode == HELM_REDUCED && nred > 0;
    // restarts of the double sweep with PML transmission take their right-hand side from the
    // target-only form of P and fold P r into the cycle's final application of P
    const bool merge = reduced && H->sweep == 0 && H->trans == 0;
    const long n = reduced ? g.Nrow() * nred : nfull;
    CHK(ensure_gmres_ws(H, nrhs, n, std::min(H->max_iter, H->restart > 0 ? H->restart : reduced ? 60 : 30)));
    std::vector<double> fn, rn;
    CHK(norms(H, f, nrhs, nfull, fn));
    // u is first written at the end of cycle 0 (u = correction), so it starts unset
    std::vector<int> total(nrhs, 0), its;
    std::vector<double> resid;
    int used = 0;
    H->stat_restarts = -1;
    bool ok = false;
    std::vector<std::vector<cd>> hess;   // Hessenberg columns of the last cycle (reduced)
    Aug aug;                       // recycled space of a restart (reduced)
    // an augmented cycle's Hessenberg matrix describes the projected operator
    // (I - C C^H) M, not M, so only a cycle that was not itself augmented is recycled
    bool prev_aug = false;
    for (int cycle = 0; used < H->max_iter; ++cycle) {
        // explicit FP64 residual of the current iterate (u = 0 in cycle 0: r = f)
        if (cycle == 0)
            HIPCHK(hipMemcpyAsync(w.R, f, field_bytes(H, nrhs), hipMemcpyDeviceToDevice, H->st));
        else
            HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A(H->t, g, nrhs, u, f, w.R, H->st)));
        CHK(norms(H, w.R, nrhs, nfull, rn));
        bool conv = true;
        for (int r = 0; r < nrhs; ++r) conv = conv && (rn[r] <= tol * fn[r] || fn[r] == 0.0);
        if (trace_on())
            std::fprintf(stderr, "[helm] cycle %d true relres rhs0 %.3e (used %d)\n", cycle,
                         fn[0] > 0 ? rn[0] / fn[0] : rn[0], used);
        if (cycle > 0 && conv) { ok = true; break; }
        H->stat_restarts += 1;
        Range range(cycle == 0 ? "GMRES cycle 0 (Algorithms 2, 3, 4)" : "GMRES restart cycle");
        std::vector<double> bn, target(nrhs);
        // right-hand sides that already meet tol take no part in this cycle: their
        // residual is cleared so the correction (P y + u~) added to them is zero
        if (cycle > 0)
            for (int r = 0; r < nrhs; ++r)
                if (rn[r] <= tol * fn[r])
                    HIPCHK(hipMemsetAsync(w.R + (size_t)r * nfull, 0, nfull * sizeof(double2), H->st));
        const double2* b = w.R;
        if (reduced) {
            // first cycle, Algorithm 2: u~ from independent strip solves of f on D~^(j)
            // (the strips' D~ ranges partition the columns, so u~ is written everywhere).
            // A restart starts from u~ = P r instead: r - A P r is again supported on the
            // reduced columns (Sec. 2.1, exact arithmetic), and the sweep removes the
            // complex64 rounding residual left off those columns (which the reduced GMRES
            // cannot see) together with its transmission across the interfaces, where
            // strip solves alone would leave it on the interface columns.
            if (cycle == 0) {
                if (H->sweep == 1) CHK(conc_setup(H, nrhs, w.R, w.Ut));
                else CHK(reduced_setup(H, nrhs, w.R, w.Ut));
            } else {
                // the restart's counterpart of Algorithm 2: an application of P, not a GMRES
                // iteration (it is counted in the operator applications of helm_get_stats
                // and against max_iter)
                H->stat_ap += 1;
                if (merge) CHK(restart_rhs_reduced(H, nrhs, w.R, w.red));
                else CHK(apply_P_any(H, nrhs, w.R, w.Ut));
                used += 1;
            }
            if (cycle == 0 || !merge) {
                HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A(H->t, g, nrhs, w.Ut, w.R, w.Hf, H->st)));
                HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_gather_cols(w.Hf, red_cols(H), nred, nrhs, g.Nrow(), g.Nx, w.red, H->st)));
            }
            b = w.red;
            if (cycle > 0 && !prev_aug) CHK(build_aug(H, nrhs, n, w.red, hess, its, aug));
        }
        CHK(norms(H, b, nrhs, n, bn));
        // complex64, first cycle: f - A u~ off the reduced columns vanishes in exact arithmetic
        // (Sec. 2.3), so what is there is the rounding noise of the complex64 strip solves:
        // the level below which the reduced GMRES cannot lower the true residual.  Measured
        // per right-hand side, so that even a handle's first solve stops its first cycle there
        std::vector<double> noise(nrhs, 0.0);
        if (reduced && cycle == 0 && H->prec != HELM_C128) {
            std::vector<double> hn;
            CHK(norms(H, w.Hf, nrhs, nfull, hn));
            for (int r = 0; r < nrhs; ++r) noise[r] = std::sqrt(std::max(hn[r] * hn[r] - bn[r] * bn[r], 0.0));
            if (trace_on())
                std::fprintf(stderr, "[helm] complex64 noise of Algorithm 2 rhs0 %.3e relative\n",
                             fn[0] > 0 ? noise[0] / fn[0] : 0.0);
        }
        if (trace_on())
            std::fprintf(stderr, "[helm] cycle %d |b| rhs0 %.3e |f| %.3e\n", cycle, bn[0], fn[0]);
        for (int r = 0; r < nrhs; ++r) {
            // the GMRES residual is the true residual of the updated iterate (reduced form:
            // Sec. 2.3).  First cycle: the paper's reduction by tol of the starting
            // residual, capped at tol ||f||; a restart only has to reach tol ||f||.
            target[r] = cycle == 0 ? tol * std::min(bn[r], fn[r]) : tol * fn[r];
            // complex64: iterating the first cycle below the rounding floor of the
            // preconditioner gains nothing (the restart starts from the floor anyway)
            if (cycle == 0 && noise[r] > 2.0 * tol * fn[r])
                target[r] = std::max(target[r], FLOOR_PER_NOISE * noise[r]);
        }
        // GMRES on op(y) = b; the solution increment is P y (+ u~)
        CHK(gmres_cycle(H, nrhs, n, b, bn, target, H->max_iter - used, w.w, its, resid,
                        reduced ? &hess : nullptr, aug.nv > 0 ? &aug : nullptr));
        prev_aug = aug.nv > 0;
        aug = Aug();
        int kmax = 0;
        for (int r = 0; r < nrhs; ++r) { total[r] += its[r]; kmax = std::max(kmax, its[r]); }
        used += std::max(kmax, 1);
        if (reduced && cycle > 0 && merge) {
            // Algorithm 4 with the restart's P r folded in: u += P (r + psi)
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_scatter_cols(w.w, red_cols(H), nred, nrhs, g.Nrow(), g.Nx, w.R, H->st, true)));
            CHK(apply_P_any(H, nrhs, w.R, w.Hf));
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_sum3(u, w.Hf, nullptr, u, nrhs * nfull, H->st)));
        } else if (reduced) {
            // Algorithm 4: u += P psi + u~   (psi scattered onto the reduced columns of Psi,
            // which is zero everywhere else: nothing but this scatter writes it)
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_scatter_cols(w.w, red_cols(H), nred, nrhs, g.Nrow(), g.Nx, w.Psi, H->st)));
            CHK(apply_P_any(H, nrhs, w.Psi, w.Hf));
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_sum3(cycle == 0 ? nullptr : u, w.Hf, w.Ut, u, nrhs * nfull, H->st)));
        } else {
            CHK(apply_P_any(H, nrhs, w.w, w.Hf));
            HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_sum3(cycle == 0 ? nullptr : u, w.Hf, nullptr, u, nrhs * nfull, H->st)));
        }
    }
    if (!ok) {
        HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A(H->t, g, nrhs, u, f, w.R, H->st)));
        CHK(norms(H, w.R, nrhs, nfull, rn));
    }
    bool conv = true;
    for (int r = 0; r < nrhs; ++r) {
        const double rr = fn[r] > 0 ? rn[r] / fn[r] : rn[r];
        if (relres) relres[r] = rr;
        if (iters) iters[r] = total[r];
        conv = conv && (rr <= tol);
    }
    if (!conv) return fail(H, HELM_ENOCONV, "GMRES did not reach the tolerance within max_iter");
    return HELM_OK;
}

}  // namespace

// ---------------------------------------------------------------- shared with other entry points
namespace helm {

size_t strip_workspace_bytes(helm_t H, int nrhs) { return strip_ws_bytes(H, nrhs); }

// x = A^(j)^{-1} r for strip `strip` ([rhs][row][strip-local column] layout of
// helm_strip_solve).  ws: the strip-solver workspace, at least strip_workspace_bytes(H, nrhs)
// bytes (null: the handle's own, which must already be sized for nrhs); a caller-supplied
// workspace solve is never event-timed.
helm_status strip_solve_into(helm_t H, int strip, int nrhs, const void* r, void* x, void* ws) {
    const auto& g = H->g;
    const int W = g.strips[strip].W;
    helm::IOSpec io;
    io.src = static_cast<const double2*>(r);
    io.src_rs = g.Nrow() * W; io.src_ls = W; io.src_off = 0;
    io.src_lo = 0; io.src_hi = W;
    io.dst = static_cast<double2*>(x);
    io.dst_rs = g.Nrow() * W; io.dst_ls = W; io.dst_off[0] = io.dst_off[1] = 0;
    io.o_lo[0] = 0; io.o_hi[0] = W;
    return strip_solve_any(H, strip, nrhs, io, ws, ws == nullptr);
}

hipStream_t handle_stream(helm_t H) { return H->st; }
int handle_device(helm_t H) { return H->dev; }
bool handle_factored(helm_t H) { return H->factored; }
int handle_strips(helm_t H) { return H->g.J; }
helm_status handle_fail(helm_t H, helm_status code, const std::string& msg) { return fail(H, code, msg); }

}  // namespace helm

// =====================================================================================
extern "C" {

void helm_default_opts(helm_opts* o, int n_x, int n_y) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dim = 2;
    o->n[0] = n_x; o->n[1] = n_y; o->n[2] = 1;
    o->pml_outer = 16; o->pml_iface = 8;
    o->pml_power = 2.0; o->pml_s0 = 10.0; o->pml_cref = 0.0;
    o->beta = nullptr; o->beta_rule = 0;
    o->prec = HELM_C128; o->mode = HELM_FULL; o->max_iter = 200; o->chunk = 0;
    o->stream = nullptr;
    o->graph = 1;
    o->pml_iface_s0 = -1.0;     // 2.5 per cell of the pad
    o->sweep = 0;
    o->transmission = 0;
    o->restart = 0;
    o->batch_fuse = 0;
}

helm_status helm_setup(const double* c, double omega, double h, const helm_opts* opts, int J,
                       helm_t* out) {
    if (!out) return HELM_EINVAL;
    *out = nullptr;
    g_setup_err.clear();
    if (!c || !opts) { g_setup_err = "null c or opts"; return HELM_EINVAL; }
    helm_t H = new helm_problem();
    auto bad = [&](const std::string& m) {
        g_setup_err = m;
        delete H;
        return HELM_EINVAL;
    };
    if (opts->dim != 2 && opts->dim != 3) return bad("dim must be 2 or 3");
    const int dim = opts->dim;
    const int nx = opts->n[0], ny = opts->n[1], nz = dim == 3 ? opts->n[2] : 1;
    if (nx < 2 || ny < 2 || nz < 1 || (dim == 3 && nz < 2))
        return bad("interior grid must be at least 2 points along every axis");
    if (!(omega > 0) || !std::isfinite(omega)) return bad("omega must be positive and finite");
    if (!(h > 0) || !std::isfinite(h)) return bad("h must be positive and finite");
    if (J < 1) return bad("J must be >= 1");
    if (opts->pml_outer < 1) return bad("pml_outer must be >= 1");
    if (opts->transmission != 0 && opts->transmission != 1)
        return bad("transmission must be 0 (PML) or 1 (Robin)");
    const bool robin = opts->transmission == 1;
    if (robin && (opts->dim != 2 || opts->mode == HELM_REDUCED))
        return bad("the Robin transmission is built for 2-D problems and the full form");
    if (J > 1 && !robin && opts->pml_iface < 1) return bad("pml_iface must be >= 1");
    double cmax = 0.0;
    for (size_t i = 0; i < (size_t)nx * ny * nz; ++i) {
        if (!(c[i] > 0.0) || !std::isfinite(c[i])) return bad("c must be positive and finite");
        cmax = std::max(cmax, c[i]);
    }
    helm::Geom& g = H->g;
    g.nx = nx; g.ny = ny; g.wout = opts->pml_outer; g.w = opts->pml_iface; g.J = J;
    g.Nx = nx + 2 * g.wout; g.Ny = ny + 2 * g.wout;
    g.dim = dim;
    g.nz = dim == 3 ? nz : 0;
    g.Nz = dim == 3 ? nz + 2 * g.wout : 1;
    g.h = h; g.omega = omega;
    g.power = opts->pml_power > 0 ? opts->pml_power : 2.0;
    g.s0 = opts->pml_s0 >= 0 ? opts->pml_s0 : 10.0;
    // interface pads: unless given, the same damping per cell for every width,
    // sigma_max h / c_ref = 2.5 (s0 = 2.5 w)
    g.s0i = opts->pml_iface_s0 >= 0 ? opts->pml_iface_s0 : 2.5 * g.w;
    g.cref = opts->pml_cref > 0 ? opts->pml_cref : cmax;
    // ---- partition (Sec. 2.2; eq. define_beta_j for rule 1)
    g.beta.assign(J + 1, 0);
    g.beta[J] = g.Nx;
    for (int s = 1; s < J; ++s) {
        if (opts->beta) g.beta[s] = opts->beta[s - 1];
        else if (opts->beta_rule == 1)
            g.beta[s] = (int)std::floor(g.w + s * (double)(g.Nx - 2 * g.w - 1) / J + 0.5);
        else
            g.beta[s] = g.wout + (int)std::floor(s * (double)nx / J + 0.5);
    }
    for (int s = 1; s <= J; ++s)
        if (g.beta[s] - g.beta[s - 1] < 2) return bad("every strip core needs at least two columns");
    for (int s = 1; s < J; ++s)
        if (g.beta[s] - 1 < g.wout || g.beta[s] + 1 > g.wout + nx - 1)
            return bad("interfaces must lie inside the interior, clear of the outer PML");
    g.strips.resize(J);
    for (int s = 0; s < J; ++s) {
        helm::Strip& S = g.strips[s];
        S.lpad = s > 0; S.rpad = s < J - 1;
        S.core_lo = g.beta[s]; S.core_hi = g.beta[s + 1];
        S.dom_lo = S.core_lo; S.dom_hi = S.core_hi + (S.rpad ? 1 : 0);
        // Robin subdomains are D^(j) and the extra column, with no pads
        const int pad = robin ? 0 : g.w;
        S.a = S.core_lo - (S.lpad ? pad : 0);
        S.W = S.dom_hi + (S.rpad ? pad : 0) - S.a;
        S.kdn_lo = S.core_lo + (S.lpad ? 1 : 0);
        S.kdn_hi = S.core_hi + (S.rpad ? 1 : 0);
        if (S.W > WP) return bad("padded strip " + std::to_string(s) + " is " + std::to_string(S.W) +
                                 " columns wide; at most 64 are supported (use more strips)");
    }
    if (dim == 3) {
        int Bmax = 0;
        for (const auto& S : g.strips) Bmax = std::max(Bmax, S.W * g.Nz);
        g.Bp = (Bmax + 63) / 64 * 64;
        if (g.Bp > helm::BP3_MAX)
            return bad("3-D slab blocks of " + std::to_string(Bmax) + " unknowns exceed " +
                       std::to_string(helm::BP3_MAX) + " (use thinner slabs or fewer z points)");
    }
    // ---- chunks along y (3-D slabs: one chunk, each plane step is a large product)
    set_chunks(H, dim == 3 ? g.Ny : (opts->chunk > 0 ? opts->chunk : 32));
    H->prec = opts->prec == HELM_MIXED_C64 ? HELM_MIXED_C64 : HELM_C128;
    H->mode = opts->mode == HELM_REDUCED ? HELM_REDUCED : HELM_FULL;
    H->max_iter = opts->max_iter > 0 ? opts->max_iter : 200;
    H->st = static_cast<hipStream_t>(opts->stream);
    H->use_graph = opts->graph ? 1 : 0;
    if (opts->sweep != 0 && opts->sweep != 1) return bad("sweep must be 0 (double sweep) or 1 (concurrent)");
    H->sweep = opts->sweep;
    H->trans = opts->transmission;
    if (opts->restart < 0) return bad("restart must be >= 0");
    H->restart = opts->restart;
    H->batch_fuse = opts->batch_fuse ? 1 : 0;
    if (hipGetDevice(&H->dev) != hipSuccess) H->dev = 0;

    // ---- tables (FP64 complex), Sec. 2.1-2.2
    const int Nx = g.Nx, Ny = g.Ny, Nz = g.Nz;
    std::vector<double> k2((size_t)Nx * Ny * Nz);
    for (int z = 0; z < Nz; ++z) {
        const int zi = dim == 3 ? std::min(std::max(z - g.wout, 0), nz - 1) : 0;
        for (int l = 0; l < Ny; ++l) {
            const int li = std::min(std::max(l - g.wout, 0), ny - 1);
            for (int i = 0; i < Nx; ++i) {
                const int ii = std::min(std::max(i - g.wout, 0), nx - 1);
                const double cc = c[((size_t)zi * ny + li) * nx + ii];
                k2[((size_t)z * Ny + l) * Nx + i] = (omega / cc) * (omega / cc);
            }
        }
    }
    std::vector<double2> az, azh;
    if (dim == 3) {
        az.resize(Nz); azh.resize(Nz + 1);
        for (int z = 0; z < Nz; ++z) az[z] = d2(alpha_outer(g, z, Nz));
        for (int z = 0; z <= Nz; ++z) azh[z] = d2(alpha_outer(g, z - 0.5, Nz));
    }
    std::vector<double2> ax(Nx), axh(Nx + 1), ay(Ny), ayh(Ny + 1), cy(Ny), by(Ny);
    for (int i = 0; i < Nx; ++i) ax[i] = d2(alpha_outer(g, i, Nx));
    for (int i = 0; i <= Nx; ++i) axh[i] = d2(alpha_outer(g, i - 0.5, Nx));
    for (int l = 0; l < Ny; ++l) ay[l] = d2(alpha_outer(g, l, Ny));
    for (int l = 0; l <= Ny; ++l) ayh[l] = d2(alpha_outer(g, l - 0.5, Ny));
    const double ih2 = 1.0 / (h * h);
    for (int l = 0; l < Ny; ++l) {
        const cd a = alpha_outer(g, l, Ny);
        cy[l] = d2(-a * alpha_outer(g, l - 0.5, Ny) * ih2);
        by[l] = d2(-a * alpha_outer(g, l + 0.5, Ny) * ih2);
    }
    std::vector<double2> sax((size_t)J * WP, make_double2(0, 0)), saxh((size_t)J * (WP + 1), make_double2(0, 0));
    std::vector<int> scol((size_t)J * WP, 0), sW(J);
    for (int s = 0; s < J; ++s) {
        const auto& S = g.strips[s];
        sW[s] = S.W;
        for (int q = 0; q < S.W; ++q) {
            sax[(size_t)s * WP + q] = d2(alpha_strip(g, S, S.a + q));
            scol[(size_t)s * WP + q] = std::min(std::max(S.a + q, S.dom_lo), S.dom_hi - 1);
        }
        for (int q = 0; q <= S.W; ++q) saxh[(size_t)s * (WP + 1) + q] = d2(alpha_strip(g, S, S.a + q - 0.5));
    }
    // Robin transmission (Sec. 4.4): rho_j = (1 + i k h/2) / (1 - i k h/2) per row with k at
    // column beta_j, and the ghost-elimination terms -alpha_x(b) alpha_x(b -+ 1/2) rho / h^2
    // of the boundary columns b = beta_s (left side) and b = beta_{s+1} (right side)
    std::vector<double2> rob, rho;
    if (robin) {
        auto rho_at = [&](int l, int col) {
            const cd ikh2(0.0, 0.5 * std::sqrt(k2[(size_t)l * Nx + col]) * h);
            return (1.0 + ikh2) / (1.0 - ikh2);
        };
        rob.assign((size_t)J * Ny * 2, make_double2(0, 0));
        rho.assign((size_t)std::max(1, J - 1) * Ny, make_double2(0, 0));
        for (int s = 1; s < J; ++s)
            for (int l = 0; l < Ny; ++l) rho[(size_t)(s - 1) * Ny + l] = d2(rho_at(l, g.beta[s]));
        for (int s = 0; s < J; ++s) {
            const auto& S = g.strips[s];
            for (int l = 0; l < Ny; ++l) {
                if (S.lpad) {
                    const int b = S.dom_lo;
                    rob[((size_t)s * Ny + l) * 2] =
                        d2(-alpha_outer(g, b, Nx) * alpha_outer(g, b - 0.5, Nx) * rho_at(l, b) * ih2);
                }
                if (S.rpad) {
                    const int b = S.dom_hi - 1;
                    rob[((size_t)s * Ny + l) * 2 + 1] =
                        d2(-alpha_outer(g, b, Nx) * alpha_outer(g, b + 0.5, Nx) * rho_at(l, b) * ih2);
                }
            }
        }
    }
    // pairs of adjacent columns per interface (the pair stencil kernel relies on it)
    std::vector<int> rcols, redcols;
    for (int s = 1; s < J; ++s) {
        rcols.push_back(g.beta[s] - 1); rcols.push_back(g.beta[s]);
        redcols.push_back(g.beta[s]); redcols.push_back(g.beta[s] + 1);
    }
    rcols.push_back(0); redcols.push_back(0);   // never empty
    // interface windows: first column and k^2 on the window columns
    const int NI = std::max(1, J - 1);
    std::vector<int> bw(NI, 0);
    for (int s = 1; s < J; ++s) bw[s - 1] = g.beta[s] - 2;
    std::vector<double> k2w((size_t)Nz * Ny * NI * helm::IWIN, 0.0);
    for (size_t row = 0; row < (size_t)Nz * Ny; ++row)
        for (int s = 1; s < J; ++s)
            for (int c = 0; c < helm::IWIN; ++c)
                k2w[(row * NI + (s - 1)) * helm::IWIN + c] = k2[row * Nx + (bw[s - 1] + c)];
    // per strip, the strip-local columns the reduced sweeps read: beta_s .. beta_s+2 on the
    // left interface, beta_{s+1}-2 .. beta_{s+1} on the right one
    std::vector<int> tcol((size_t)J * 8, -1);
    for (int s = 0; s < J; ++s) {
        const auto& S = g.strips[s];
        if (S.lpad)
            for (int k = 0; k < 3; ++k) tcol[(size_t)s * 8 + k] = g.beta[s] + k - S.a;
        if (S.rpad)
            for (int k = 0; k < 3; ++k) tcol[(size_t)s * 8 + 3 + k] = g.beta[s + 1] - 2 + k - S.a;
    }
    // strips (slabs) whose operators coincide share one factorisation: the same width, PML
    // tables and target columns, and the same k^2 on every row (and z-plane) of
    // corresponding columns (a medium that does not vary with x makes every interior strip
    // of one width alike)
    std::vector<int> urep;
    H->fidx.assign(J, 0);
    auto same_strip = [&](int a, int b) {
        if (sW[a] != sW[b]) return false;
        const int W = sW[a];
        for (int q = 0; q < W; ++q) {
            const double2 x = sax[(size_t)a * WP + q], y = sax[(size_t)b * WP + q];
            if (x.x != y.x || x.y != y.y) return false;
        }
        for (int q = 0; q <= W; ++q) {
            const double2 x = saxh[(size_t)a * (WP + 1) + q], y = saxh[(size_t)b * (WP + 1) + q];
            if (x.x != y.x || x.y != y.y) return false;
        }
        for (int k = 0; k < 8; ++k)
            if (tcol[(size_t)a * 8 + k] != tcol[(size_t)b * 8 + k]) return false;
        for (size_t k = 0; robin && k < (size_t)Ny * 2; ++k) {
            const double2 x = rob[(size_t)a * Ny * 2 + k], y = rob[(size_t)b * Ny * 2 + k];
            if (x.x != y.x || x.y != y.y) return false;
        }
        for (int q = 0; q < W; ++q) {
            const int ca = scol[(size_t)a * WP + q], cb = scol[(size_t)b * WP + q];
            if (ca == cb) continue;
            for (size_t row = 0; row < (size_t)Nz * Ny; ++row)
                if (k2[row * Nx + ca] != k2[row * Nx + cb]) return false;
        }
        return true;
    };
    for (int s = 0; s < J; ++s) {
        int u = 0;
        while (u < (int)urep.size() && !same_strip(s, urep[u])) ++u;
        if (u == (int)urep.size()) urep.push_back(s);
        H->fidx[s] = u;
    }
    H->nfac = (int)urep.size();
    std::vector<double2> fsax((size_t)H->nfac * WP), fsaxh((size_t)H->nfac * (WP + 1));
    std::vector<int> fscol((size_t)H->nfac * WP), fsW(H->nfac), ftcol((size_t)H->nfac * 8);
    for (int u = 0; u < H->nfac; ++u) {
        const int r = urep[u];
        fsW[u] = sW[r];
        std::copy(sax.begin() + (size_t)r * WP, sax.begin() + (size_t)(r + 1) * WP, fsax.begin() + (size_t)u * WP);
        std::copy(saxh.begin() + (size_t)r * (WP + 1), saxh.begin() + (size_t)(r + 1) * (WP + 1),
                  fsaxh.begin() + (size_t)u * (WP + 1));
        std::copy(scol.begin() + (size_t)r * WP, scol.begin() + (size_t)(r + 1) * WP, fscol.begin() + (size_t)u * WP);
        std::copy(tcol.begin() + (size_t)r * 8, tcol.begin() + (size_t)(r + 1) * 8, ftcol.begin() + (size_t)u * 8);
    }
    auto& t = H->t;
    helm_status st = HELM_OK;
    struct Guard {
        helm_t& H; helm_status& st; bool armed = true;
        ~Guard() { if (armed && st != HELM_OK) { g_setup_err = H->err; helm_destroy(H); } }
    } guard{H, st};
    if ((st = upload(H, (void**)&t.k2, k2.data(), k2.size() * sizeof(double))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.ax, ax.data(), ax.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.axh, axh.data(), axh.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.ay, ay.data(), ay.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.ayh, ayh.data(), ayh.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.cy, cy.data(), cy.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.by, by.data(), by.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.sax, sax.data(), sax.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.saxh, saxh.data(), saxh.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.scol, scol.data(), scol.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.sW, sW.data(), sW.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.rcols, rcols.data(), rcols.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.redcols, redcols.data(), redcols.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.tcol, tcol.data(), tcol.size() * sizeof(int))) != HELM_OK) return st;
    if (robin) {
        if ((st = upload(H, (void**)&t.srob, rob.data(), rob.size() * sizeof(double2))) != HELM_OK) return st;
        if ((st = upload(H, (void**)&t.rho, rho.data(), rho.size() * sizeof(double2))) != HELM_OK) return st;
        if (opts->sweep == 1) {
            std::vector<int> par(Nx);
            for (int s = 0; s < J; ++s)
                for (int x = g.beta[s]; x < g.beta[s + 1]; ++x) par[x] = s & 1;
            if ((st = upload(H, (void**)&H->colpar, par.data(), par.size() * sizeof(int))) != HELM_OK) return st;
        }
    }
    H->tf = t;
    if (robin) {
        std::vector<double2> frob((size_t)H->nfac * Ny * 2);
        for (int u = 0; u < H->nfac; ++u)
            std::copy(rob.begin() + (size_t)urep[u] * Ny * 2, rob.begin() + (size_t)(urep[u] + 1) * Ny * 2,
                      frob.begin() + (size_t)u * Ny * 2);
        if ((st = upload(H, (void**)&H->tf.srob, frob.data(), frob.size() * sizeof(double2))) != HELM_OK)
            return st;
    }
    if ((st = upload(H, (void**)&H->tf.sax, fsax.data(), fsax.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&H->tf.saxh, fsaxh.data(), fsaxh.size() * sizeof(double2))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&H->tf.scol, fscol.data(), fscol.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&H->tf.sW, fsW.data(), fsW.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&H->tf.tcol, ftcol.data(), ftcol.size() * sizeof(int))) != HELM_OK) return st;
    H->gf = g;
    H->gf.J = H->nfac;
    H->gf.strips.clear();
    for (int u = 0; u < H->nfac; ++u) H->gf.strips.push_back(g.strips[urep[u]]);
    if ((st = upload(H, (void**)&t.bw, bw.data(), bw.size() * sizeof(int))) != HELM_OK) return st;
    if ((st = upload(H, (void**)&t.k2w, k2w.data(), k2w.size() * sizeof(double))) != HELM_OK) return st;
    if (dim == 3) {
        if ((st = upload(H, (void**)&t.az, az.data(), az.size() * sizeof(double2))) != HELM_OK) return st;
        if ((st = upload(H, (void**)&t.azh, azh.data(), azh.size() * sizeof(double2))) != HELM_OK) return st;
    }
    if ((st = dmalloc(H, &H->d_err, sizeof(int))) != HELM_OK) return st;
    H->err.clear();
    *out = H;
    return HELM_OK;
}

// 3-D: the inverses G_l of every slab, plane by plane (all slabs of a plane together)
helm_status factor3(helm_t H) {
    const auto& g = H->g;
    const size_t BB = (size_t)g.Bp * g.Bp;
    const bool single = H->prec != HELM_C128;
    const size_t esz = single ? sizeof(float2) : sizeof(double2);
    void* F = nullptr;
    const int nf = H->nfac;               // one factorisation per distinct slab operator
    CHK(dmalloc(H, &F, (size_t)nf * g.Ny * BB * esz));
    // F is freed on every early return (HIP errors included) unless it was handed to H
    struct FOwner {
        void*& p; bool kept = false;
        ~FOwner() { if (!kept) dfree(p); }
    } fown{F};
    auto keep_F = [&]() { H->F = F; fown.kept = true; };
    struct Bufs {
        std::vector<void*> p;
        ~Bufs() { for (void* q : p) dfree(q); }
    } bufs;
    auto alloc = [&](void** q, size_t bytes) -> helm_status {
        CHK(dmalloc(H, q, bytes));
        bufs.p.push_back(*q);
        return HELM_OK;
    };
    const size_t nb = helm::factor3_panel_width();
    double2 *S, *G64, *Tm, *Cm;
    int *perm, *pi;
    void* work32 = nullptr;
    helm_status st;
    helm::Fac3Args a;
    a.J = nf; a.Ny = g.Ny; a.Nz = g.Nz; a.Nx = g.Nx; a.Bp = g.Bp;
    a.sW = H->tf.sW; a.sax = H->tf.sax; a.saxh = H->tf.saxh; a.scol = H->tf.scol;
    a.ay = H->t.ay; a.ayh = H->t.ayh; a.az = H->t.az; a.azh = H->t.azh;
    a.cy = H->t.cy; a.by = H->t.by; a.k2 = H->t.k2;
    a.ih2 = 1.0 / (g.h * g.h);
    int herr = 0;
    // the sweeps read the stored complex64 inverses in 16-row panels (one contiguous run per
    // 16-row tile of a plane product instead of 16-entry pieces of every column)
    auto panelize = [&](void* Fp, void* work) -> hipError_t {
        auto run = [&]() {
            return helm::launch_factor3_panelize(static_cast<float2*>(Fp), (size_t)g.Ny * BB, nf, g.Ny, g.Bp,
                                                 static_cast<float2*>(work), H->st);
        };
        // timed apart from the factorisation (its own class), so that a factorisation stays
        // one timed unit
        return TIMED(H, helm::K_OTHER, run());
    };
    // HELM_FACTOR3_FP64=1 sends a complex64 factorisation straight to the FP64 route (the one
    // an ill-conditioned diagonal block would take), so that route can be exercised
    const char* force = std::getenv("HELM_FACTOR3_FP64");
    if (single && !(force && force[0] == '1')) {
        // complex64 blocked Gauss-Jordan in place in the stored factor; a diagonal block
        // that is singular or ill-conditioned sends the whole factorisation to the FP64
        // Gauss-Jordan with partial pivoting over the whole column below
        if ((st = alloc(&work32, helm::factor3_f32_work_bytes(nf, g.Bp))) != HELM_OK) return st;
        HIPCHK(hipMemsetAsync(H->d_err, 0, sizeof(int), H->st));
        // the slabs are independent.  FAC3_GROUPS streams (the handle's and streams of their
        // own, default priority) each factor one group of slabs at a time, all planes of a
        // group before the next, so that one stream's latency-bound diagonal inverses
        // overlap the other streams' update GEMMs.  Measured at 80^3 (16 slabs, 2 streams):
        // groups of 8 slabs 1130 ms, of 4 1226 ms, of 2 1590 ms (smaller groups keep the
        // updated matrices in the last-level cache but launch too few tiles), one stream
        // 1425 ms; 4 or 8 streams with one group each changed nothing
        constexpr int NGR = FAC3_GROUPS;
        const int batch = FAC3_BATCH > 0 ? std::min(FAC3_BATCH, nf) : (nf + NGR - 1) / NGR;
        const int ngroups = (nf + batch - 1) / batch;
        const int nst = std::min(NGR, ngroups);
        hipStream_t sts[NGR];
        sts[0] = H->st;
        for (int q = 1; q < nst; ++q) {
            if (!H->st_fac[q - 1]) HIPCHK(hipStreamCreateWithFlags(&H->st_fac[q - 1], hipStreamNonBlocking));
            sts[q] = H->st_fac[q - 1];
        }
        hipEvent_t evs[NGR] = {};
        struct Evs {
            hipEvent_t* e; int n;
            ~Evs() { for (int q = 0; q < n; ++q) if (e[q]) (void)hipEventDestroy(e[q]); }
        } evguard{evs, NGR};
        for (int q = 0; q < nst; ++q) HIPCHK(hipEventCreateWithFlags(&evs[q], hipEventDisableTiming));
        float2* F32 = static_cast<float2*>(F);
        const size_t stride = (size_t)g.Ny * BB;
        hipError_t e = TIMED(H, helm::K_FACTOR_CHUNKS, [&]() -> hipError_t {
            // fork: every group stream waits for the work queued so far on the handle's
            hipError_t r = hipEventRecord(evs[0], H->st);
            for (int q = 1; q < nst && r == hipSuccess; ++q) r = hipStreamWaitEvent(sts[q], evs[0], 0);
            for (int g0 = 0; g0 < ngroups && r == hipSuccess; g0 += nst)
                for (int l = 0; l < g.Ny && r == hipSuccess; ++l)
                    for (int q = 0; q < nst && r == hipSuccess; ++q) {
                        const int gi = g0 + q;
                        if (gi >= ngroups) continue;
                        const int s0 = gi * batch;
                        const int ns = std::min(batch, nf - s0);
                        r = helm::launch_factor3_plane_f32(a, l, F32, stride, work32, H->d_err, sts[q], s0, ns);
                    }
            // join
            for (int q = 1; q < nst && r == hipSuccess; ++q) {
                r = hipEventRecord(evs[q], sts[q]);
                if (r == hipSuccess) r = hipStreamWaitEvent(H->st, evs[q], 0);
            }
            return r;
        }());
        HIPCHK(e);
        HIPCHK(hipMemcpyAsync(&herr, H->d_err, sizeof(int), hipMemcpyDeviceToHost, H->st));
        HIPCHK(hipStreamSynchronize(H->st));
        H->factor_path = herr ? 0 : 1;
        if (trace_on())
            std::fprintf(stderr, "[helm] 3-D complex64 blocked Gauss-Jordan: %s\n",
                         herr ? "ill-conditioned diagonal block, redone in FP64" : "accepted");
        if (!herr) {
            void* pw = nullptr;
            if ((st = alloc(&pw, (size_t)nf * BB * sizeof(float2))) != HELM_OK) return st;
            HIPCHK(panelize(F, pw));
            HIPCHK(hipStreamSynchronize(H->st));
            keep_F();
            H->factored = true;
            return HELM_OK;
        }
    }
    H->factor_path = 0;
    if ((st = alloc((void**)&S, nf * BB * sizeof(double2))) != HELM_OK ||
        (st = alloc((void**)&G64, nf * BB * sizeof(double2))) != HELM_OK ||
        (st = alloc((void**)&Tm, (size_t)nf * g.Bp * nb * sizeof(double2))) != HELM_OK ||
        (st = alloc((void**)&Cm, (size_t)nf * g.Bp * nb * sizeof(double2))) != HELM_OK ||
        (st = alloc((void**)&perm, (size_t)nf * g.Bp * sizeof(int))) != HELM_OK ||
        (st = alloc((void**)&pi, (size_t)nf * g.Bp * sizeof(int))) != HELM_OK)
        return st;
    HIPCHK(hipMemsetAsync(H->d_err, 0, sizeof(int), H->st));
    // timed as one unit, like the complex64 route
    hipError_t e = TIMED(H, helm::K_FACTOR_CHUNKS, [&]() -> hipError_t {
        hipError_t r = hipSuccess;
        for (int l = 0; l < g.Ny && r == hipSuccess; ++l) {
            void* out = static_cast<char*>(F) + (size_t)l * BB * esz;
            r = helm::launch_factor3_plane(a, l, l > 0 ? G64 : nullptr, S, Tm, Cm, perm, pi, H->d_err, G64, out,
                                           single, (size_t)g.Ny * BB, H->st);
        }
        return r;
    }());
    HIPCHK(e);
    herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, H->d_err, sizeof(int), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    if (single && !herr) {
        // S (nf Bp^2 complex128 entries) is free now and holds the panel scratch
        HIPCHK(panelize(F, S));
        HIPCHK(hipStreamSynchronize(H->st));
    }
    keep_F();
    if (herr) return fail(H, HELM_ESINGULAR, "zero or non-finite pivot in a slab factorisation");
    H->factored = true;
    return HELM_OK;
}

helm_status helm_factor(helm_t H) {
    if (!H) return HELM_EINVAL;
    Range range("helm_factor");
    if (!H->t.k2) return fail(H, HELM_ESTATE, "helm_setup did not complete");
    const auto& g = H->g;
    // the captured reduced operator holds the factor addresses in its kernel arguments:
    // drop it before the factors are freed (it is captured again on the next solve)
    CHK(drop_graph(H));
    HIPCHK(hipStreamSynchronize(H->st));    // no queued work may still read the old factors
    H->factored = false;
    if (g.dim == 3) {
        dfree(H->F);
        H->F = nullptr;
        return factor3(H);
    }
    // The factor buffers keep their size for the handle's life: they are allocated (and
    // cleared: slots no factorisation writes must read as zero) once, and every later
    // factorisation overwrites the same slots.  The complex64 path keeps the FP64 factor as
    // workspace and receives each block rounded as it is stored.
    const size_t nel = (size_t)H->nfac * g.Ny * NSLOT * BLK;
    const size_t nsel = H->ch.G >= 2 ? (size_t)H->nfac * (H->ch.P - 1) * 2 * BLK : 0;
    const size_t ncomp = (size_t)H->nfac * g.Ny * 2 * 8 * WP;
    const bool single = H->prec != HELM_C128;
    const size_t esz = single ? sizeof(float2) : sizeof(double2);
    if (!H->F64) {
        CHK(dmalloc(H, &H->F64, nel * sizeof(double2)));
        if (single) CHK(dmalloc(H, &H->F, nel * esz));
        else H->F = H->F64;
        CHK(dmalloc(H, &H->Fc, ncomp * esz));
        if (single) CHK(dmalloc(H, &H->Fa, nel / NSLOT * esz));
        H->fac_m = 0;
    }
    if (H->fac_m != H->ch.m) {
        // first factorisation, or a new y-partition (autotuning): the slots a partition
        // leaves unwritten read as zero, and the propagators take its separator count
        HIPCHK(hipMemsetAsync(H->F64, 0, nel * sizeof(double2), H->st));
        if (single) HIPCHK(hipMemsetAsync(H->F, 0, nel * esz, H->st));
        if (H->Fs != H->Fs64) dfree(H->Fs);
        dfree(H->Fs64);
        dfree(H->Fw);
        H->Fs = H->Fs64 = nullptr;
        H->Fw = nullptr;
        if (nsel) {
            CHK(dmalloc(H, &H->Fs64, nsel * sizeof(double2)));
            if (single) CHK(dmalloc(H, &H->Fs, nsel * esz));
            else H->Fs = H->Fs64;
            if (single) CHK(dmalloc(H, &H->Fw, nsel * 2 * esz));     // 4 blocks per separator
        }
        H->fac_m = H->ch.m;
    }
    double2* F64 = H->F64;
    float2* F32 = single ? static_cast<float2*>(H->F) : nullptr;
    HIPCHK(hipMemsetAsync(H->d_err, 0, sizeof(int), H->st));
    // one factorisation per distinct strip operator (factor slots 0 .. nfac - 1)
    const auto& gf = H->gf;
    HIPCHK(TIMED(H, helm::K_FACTOR_CHUNKS, helm::launch_factor_chunks(H->tf, gf, H->ch, F64, F32, H->d_err, H->st)));
    HIPCHK(TIMED(H, helm::K_FACTOR_SEPS, helm::launch_factor_separators(H->tf, gf, H->ch, F64, F32, H->d_err, H->st)));
    if (nsel)
        HIPCHK(TIMED(H, helm::K_FACTOR_SEPS,
                     helm::launch_factor_propagators(H->tf, gf, H->ch, F64, H->Fs64,
                                                     single ? static_cast<float2*>(H->Fs) : nullptr, H->st)));
    if (single) {
        HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_extract_targets<float2>(F32, static_cast<float2*>(H->Fc),
                                                                           H->tf.tcol, gf, H->ch, H->st)));
        HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_swizzle_factors(F32, static_cast<const float2*>(H->Fs),
                                                                   static_cast<float2*>(H->Fa),
                                                                   static_cast<float2*>(H->Fw), gf, H->ch,
                                                                   H->nfac, H->st)));
    }
    else
        HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_extract_targets<double2>(F64, static_cast<double2*>(H->Fc),
                                                                            H->tf.tcol, gf, H->ch, H->st)));
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, H->d_err, sizeof(int), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    if (herr & 1) return fail(H, HELM_ESINGULAR, "zero or non-finite pivot in a strip factorisation");
    if (herr & 2)
        return fail(H, HELM_ESINGULAR, "a strip block is numerically singular (1-norm condition estimate "
                                       "above 1e13): the strip operator is at or near a resonance");
    H->factored = true;
    return HELM_OK;
}

helm_status helm_solve(helm_t H, int nrhs, const void* rhs, void* u, double tol, int* iters,
                       double* relres) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_solve before helm_factor");
    if (nrhs < 1 || !rhs || !u) return fail(H, HELM_EINVAL, "nrhs >= 1 and non-null rhs, u required");
    if (!(tol > 0)) return fail(H, HELM_EINVAL, "tol must be positive");
    H->stat_ap = 0;
    H->stat_panel = H->stat_panel_full = 0;
    Range range("helm_solve");
    const auto t0 = std::chrono::steady_clock::now();
    helm_status s = solve_impl(H, nrhs, static_cast<const double2*>(rhs), static_cast<double2*>(u),
                               tol, iters, relres);
    const auto t1 = std::chrono::steady_clock::now();
    H->stat_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return s;
}

helm_status helm_autotune(helm_t H, int nrhs, const void* rhs, const int* cand, int ncand, int reps,
                          int* best, double* ms) {
    if (!H) return HELM_EINVAL;
    if (!H->t.k2) return fail(H, HELM_ESTATE, "helm_setup did not complete");
    if (nrhs < 1 || !rhs || !cand || ncand < 1 || reps < 1)
        return fail(H, HELM_EINVAL, "helm_autotune: nrhs, reps, ncand >= 1 and non-null rhs, cand required");
    for (int c = 0; c < ncand; ++c)
        if (cand[c] < 2) return fail(H, HELM_EINVAL, "helm_autotune: candidate chunk sizes must be >= 2");
    const auto& g = H->g;
    if (g.dim == 3) {
        // a slab is one chunk: nothing to choose
        if (best) *best = H->ch.m;
        if (ms) for (int c = 0; c < ncand; ++c) ms[c] = 0.0;
        if (!H->factored) return helm_factor(H);
        return HELM_OK;
    }
    const bool reduced = H->mode == HELM_REDUCED && g.J >= 2;
    const int nred = 2 * (g.J - 1);
    CHK(ensure_sweep_ws(H, nrhs));
    // the operator one GMRES iteration applies: Algorithm 3 on the right-hand sides'
    // reduced columns (REDUCED), or P followed by A (FULL)
    const size_t in_bytes = reduced ? (size_t)nrhs * g.Nrow() * nred * sizeof(double2) : field_bytes(H, nrhs);
    double2 *xin = nullptr, *xout = nullptr;
    struct Bufs { double2** a; double2** b; ~Bufs() { dfree(*a); dfree(*b); } } bufs{&xin, &xout};
    CHK(dmalloc(H, &xin, in_bytes));
    CHK(dmalloc(H, &xout, in_bytes));
    if (reduced)
        HIPCHK(helm::launch_gather_cols(static_cast<const double2*>(rhs), red_cols(H), nred, nrhs, g.Nrow(),
                                        g.Nx, xin, H->st));
    else
        HIPCHK(hipMemcpyAsync(xin, rhs, in_bytes, hipMemcpyDeviceToDevice, H->st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } ev{e0, e1};
    auto apply = [&]() -> helm_status {
        if (reduced) return apply_AP_red(H, nrhs, xin, xout);
        CHK(apply_P_any(H, nrhs, xin, H->wk.PF));
        HIPCHK(helm::launch_apply_A(H->t, g, nrhs, H->wk.PF, nullptr, xout, H->st));
        return HELM_OK;
    };
    int bi = -1;
    double bms = 0.0;
    for (int c = 0; c < ncand; ++c) {
        set_chunks(H, cand[c]);
        CHK(helm_factor(H));
        CHK(apply());                      // warm-up (first touch of the layout)
        HIPCHK(hipEventRecord(e0, H->st));
        for (int r = 0; r < reps; ++r) CHK(apply());
        HIPCHK(hipEventRecord(e1, H->st));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        const double per = (double)t / reps;
        if (ms) ms[c] = per;
        if (bi < 0 || per < bms) { bi = c; bms = per; }
    }
    if (best) *best = cand[bi];
    if (cand[bi] != H->ch.m) {
        set_chunks(H, cand[bi]);
        CHK(helm_factor(H));
    }
    HIPCHK(hipStreamSynchronize(H->st));
    return HELM_OK;
}

helm_status helm_solve_batch(int nprob, const helm_t* H, const int* nrhs, const void* const* rhs,
                             void* const* u, double tol, int* iters, double* relres) {
    if (nprob < 1 || !H || !nrhs || !rhs || !u) return HELM_EINVAL;
    std::vector<long> off(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        if (!H[p]) return HELM_EINVAL;
        for (int q = 0; q < p; ++q)
            if (H[q] == H[p]) return fail(H[p], HELM_EINVAL, "helm_solve_batch: a handle is listed twice");
        if (nrhs[p] < 1) return fail(H[p], HELM_EINVAL, "helm_solve_batch: nrhs must be >= 1");
        off[p + 1] = off[p] + nrhs[p];
    }
    // 2-D complex64 problems on the double sweep fuse their strip solves: their host threads
    // meet in a Fuser, which launches the strip solves of a round on a stream of its own
    // (ordered against each problem's stream by events), one launch per phase
    std::vector<int> fuse;
    for (int p = 0; p < nprob; ++p)
        if (H[p]->batch_fuse && H[p]->factored && H[p]->g.dim == 2 && H[p]->prec == HELM_MIXED_C64 &&
            H[p]->sweep == 0 && !H[p]->timer && H[p]->dev == H[0]->dev)
            fuse.push_back(p);
    if (fuse.size() < 2) fuse.clear();
    Fuser fz;
    if (!fuse.empty()) {
        if (hipSetDevice(H[fuse[0]]->dev) != hipSuccess) return fail(H[fuse[0]], HELM_EHIP, "hipSetDevice failed");
        if (hipStreamCreateWithFlags(&fz.st, hipStreamNonBlocking) != hipSuccess)
            return fail(H[fuse[0]], HELM_EHIP, "stream creation failed");
        if (hipEventCreateWithFlags(&fz.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(fz.st);
            return fail(H[fuse[0]], HELM_EHIP, "event creation failed");
        }
        for (int p : fuse) {
            H[p]->fuser = &fz;
            fz.join();
        }
    }
    std::vector<helm_status> st(nprob, HELM_OK);
    std::vector<std::thread> th;
    th.reserve(nprob);
    for (int p = 0; p < nprob; ++p) {
        th.emplace_back([&, p]() {
            struct Leave {
                Fuser* f;
                ~Leave() { if (f) f->leave(); }
            } leave{H[p]->fuser};
            if (hipSetDevice(H[p]->dev) != hipSuccess) {
                st[p] = fail(H[p], HELM_EHIP, "hipSetDevice failed");
                return;
            }
            st[p] = helm_solve(H[p], nrhs[p], rhs[p], u[p], tol, iters ? iters + off[p] : nullptr,
                               relres ? relres + off[p] : nullptr);
        });
    }
    for (auto& t : th) t.join();
    for (int p = 0; p < nprob; ++p) H[p]->stat_fused = H[p]->stat_unfused = 0;
    if (!fuse.empty()) {
        hipError_t e = hipStreamSynchronize(fz.st);
        for (int p : fuse) {
            const hipError_t e2 = hipStreamSynchronize(H[p]->st);
            if (e == hipSuccess) e = e2;
            H[p]->fuser = nullptr;
            H[p]->stat_fused = fz.fused_launches;
            H[p]->stat_unfused = fz.single_launches;
        }
        (void)hipEventDestroy(fz.done);
        (void)hipStreamDestroy(fz.st);
        if (e != hipSuccess) return fail(H[fuse[0]], HELM_EHIP, hipGetErrorString(e));
    }
    for (int p = 0; p < nprob; ++p)
        if (st[p] != HELM_OK) return st[p];
    return HELM_OK;
}

helm_status helm_grad(helm_t H, int nsrc, const void* src, int nrec, const int64_t* rec,
                      const void* d, double tol, double* misfit, double* grad, int* iters) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_grad before helm_factor");
    if (nsrc < 1 || nrec < 1 || !src || !rec || !d || !misfit || !grad)
        return fail(H, HELM_EINVAL, "nsrc, nrec >= 1 and non-null src, rec, d, misfit, grad required");
    if (!(tol > 0)) return fail(H, HELM_EINVAL, "tol must be positive");
    const auto& g = H->g;
    if (g.dim != 2) return fail(H, HELM_EINVAL, "helm_grad supports the 2-D problem only");
    const long field = (long)g.Nx * g.Ny;
    // receivers: validated on the host, grouped by point (repeated receivers add up)
    std::vector<int64_t> hrec(nrec);
    HIPCHK(hipMemcpyAsync(hrec.data(), rec, nrec * sizeof(int64_t), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    std::vector<int> order(nrec);
    for (int k = 0; k < nrec; ++k) {
        if (hrec[k] < 0 || hrec[k] >= field)
            return fail(H, HELM_EINVAL, "receiver index " + std::to_string(hrec[k]) +
                                            " outside the padded grid [0, N_x N_y)");
        order[k] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hrec[a] < hrec[b]; });
    std::vector<long> upt;
    std::vector<int> ustart;
    for (int t = 0; t < nrec; ++t) {
        if (t == 0 || hrec[order[t]] != hrec[order[t - 1]]) {
            upt.push_back((long)hrec[order[t]]);
            ustart.push_back(t);
        }
    }
    ustart.push_back(nrec);
    const int nu = (int)upt.size();

    struct Bufs {
        std::vector<void*> p;
        ~Bufs() { for (void* q : p) dfree(q); }
    } bufs;
    auto alloc = [&](void** q, size_t bytes) -> helm_status {
        CHK(dmalloc(H, q, bytes));
        bufs.p.push_back(*q);
        return HELM_OK;
    };
    double2 *U, *Q, *Z, *r;
    long *dupt;
    int *dustart, *duidx;
    double* dmis;
    CHK(alloc((void**)&U, field_bytes(H, nsrc)));
    CHK(alloc((void**)&Q, field_bytes(H, nsrc)));
    CHK(alloc((void**)&Z, field_bytes(H, nsrc)));
    CHK(alloc((void**)&r, (size_t)nsrc * nrec * sizeof(double2)));
    CHK(alloc((void**)&dupt, nu * sizeof(long)));
    CHK(alloc((void**)&dustart, (nu + 1) * sizeof(int)));
    CHK(alloc((void**)&duidx, nrec * sizeof(int)));
    CHK(alloc((void**)&dmis, sizeof(double)));
    HIPCHK(hipMemcpyAsync(dupt, upt.data(), nu * sizeof(long), hipMemcpyHostToDevice, H->st));
    HIPCHK(hipMemcpyAsync(dustart, ustart.data(), (nu + 1) * sizeof(int), hipMemcpyHostToDevice, H->st));
    HIPCHK(hipMemcpyAsync(duidx, order.data(), nrec * sizeof(int), hipMemcpyHostToDevice, H->st));

    std::vector<int> it1(nsrc), it2(nsrc);
    std::vector<double> rr1(nsrc), rr2(nsrc);
    // forward fields u_s = A^{-1} f_s
    helm_status s1 = solve_impl(H, nsrc, static_cast<const double2*>(src), U, tol, it1.data(), rr1.data());
    if (s1 != HELM_OK && s1 != HELM_ENOCONV) return s1;
    // r = R u - d, misfit, adjoint right-hand side D conj(R^T r)
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_rec_residual(U, field, reinterpret_cast<const long*>(rec), nrec,
                                                             static_cast<const double2*>(d), nsrc, r, H->st)));
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_half_sumsq(r, (long)nsrc * nrec, dmis, H->st)));
    HIPCHK(hipMemsetAsync(Q, 0, field_bytes(H, nsrc), H->st));
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_adjoint_rhs(r, nrec, nsrc, dupt, dustart, duidx, nu, H->t, g, Q,
                                                            H->st)));
    // z = A^{-1} D conj(q), conj(lambda) = z / D
    helm_status s2 = solve_impl(H, nsrc, Q, Z, tol, it2.data(), rr2.data());
    if (s2 != HELM_OK && s2 != HELM_ENOCONV) return s2;
    HIPCHK(TIMED(H, helm::K_OTHER, helm::launch_grad_m(U, Z, nsrc, H->t, g, grad, H->st)));
    HIPCHK(hipMemcpyAsync(misfit, dmis, sizeof(double), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    if (iters)
        for (int k = 0; k < nsrc; ++k) { iters[k] = it1[k]; iters[nsrc + k] = it2[k]; }
    if (s1 != HELM_OK || s2 != HELM_OK)
        return fail(H, HELM_ENOCONV, "a forward or adjoint solve did not reach the tolerance");
    return HELM_OK;
}

helm_status helm_apply_P(helm_t H, int nrhs, const void* f, void* out) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_apply_P before helm_factor");
    if (nrhs < 1 || !f || !out) return fail(H, HELM_EINVAL, "bad arguments");
    CHK(ensure_sweep_ws(H, nrhs));
    return apply_P_any(H, nrhs, static_cast<const double2*>(f), static_cast<double2*>(out));
}

helm_status helm_apply_AP_reduced(helm_t H, int nrhs, const void* psi, void* out) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_apply_AP_reduced before helm_factor");
    if (nrhs < 1 || !psi || !out) return fail(H, HELM_EINVAL, "bad arguments");
    if (H->g.J < 2) return fail(H, HELM_EINVAL, "the reduced space is empty for J = 1");
    if (H->trans == 1) return fail(H, HELM_EINVAL, "the reduced form is built for the PML transmission");
    return apply_AP_red(H, nrhs, static_cast<const double2*>(psi), static_cast<double2*>(out));
}

helm_status helm_restart_rhs_reduced(helm_t H, int nrhs, const void* r, void* b) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_restart_rhs_reduced before helm_factor");
    if (H->g.J < 2) return fail(H, HELM_EINVAL, "the reduced space is empty for J = 1");
    if (nrhs < 1 || !r || !b) return fail(H, HELM_EINVAL, "bad arguments");
    if (H->trans == 1 || H->sweep == 1)
        return fail(H, HELM_EINVAL, "the restart right-hand side is built for the double sweep with PML transmission");
    return restart_rhs_reduced(H, nrhs, static_cast<const double2*>(r), static_cast<double2*>(b));
}

helm_status helm_apply_A(helm_t H, int nrhs, const void* u, const void* f, void* out) {
    if (!H) return HELM_EINVAL;
    if (!H->t.k2) return fail(H, HELM_ESTATE, "helm_setup did not complete");
    if (nrhs < 1 || !u || !out) return fail(H, HELM_EINVAL, "bad arguments");
    HIPCHK(TIMED(H, helm::K_STENCIL, helm::launch_apply_A(H->t, H->g, nrhs, static_cast<const double2*>(u),
                                static_cast<const double2*>(f), static_cast<double2*>(out), H->st)));
    return HELM_OK;
}

helm_status helm_strip_solve(helm_t H, int strip, int nrhs, const void* r, void* x) {
    if (!H) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_strip_solve before helm_factor");
    if (strip < 0 || strip >= H->g.J || nrhs < 1 || !r || !x)
        return fail(H, HELM_EINVAL, "bad arguments");
    CHK(ensure_sweep_ws(H, nrhs));
    return helm::strip_solve_into(H, strip, nrhs, r, x, nullptr);
}

helm_status helm_get_dims3(helm_t H, int* N_x, int* N_y, int* N_z, int* J) {
    if (!H) return HELM_EINVAL;
    if (N_x) *N_x = H->g.Nx;
    if (N_y) *N_y = H->g.Ny;
    if (N_z) *N_z = H->g.Nz;
    if (J) *J = H->g.J;
    return HELM_OK;
}

helm_status helm_get_dims(helm_t H, int* N_x, int* N_y, int* J) {
    if (!H) return HELM_EINVAL;
    if (N_x) *N_x = H->g.Nx;
    if (N_y) *N_y = H->g.Ny;
    if (J) *J = H->g.J;
    return HELM_OK;
}

helm_status helm_get_partition(helm_t H, int* beta, int* strip_first, int* strip_width) {
    if (!H || H->g.beta.empty()) return HELM_EINVAL;
    for (int s = 0; s <= H->g.J; ++s) if (beta) beta[s] = H->g.beta[s];
    for (int s = 0; s < H->g.J && s < (int)H->g.strips.size(); ++s) {
        if (strip_first) strip_first[s] = H->g.strips[s].a;
        if (strip_width) strip_width[s] = H->g.strips[s].W;
    }
    return HELM_OK;
}

helm_status helm_get_chunks(helm_t H, int* rows_per_chunk, int* nchunks) {
    if (!H) return HELM_EINVAL;
    if (rows_per_chunk) *rows_per_chunk = H->ch.m;
    if (nchunks) *nchunks = H->ch.P;
    return HELM_OK;
}

helm_status helm_get_stats(helm_t H, int* ap_applies, int* restarts, double* solve_ms) {
    if (!H) return HELM_EINVAL;
    if (ap_applies) *ap_applies = H->stat_ap;
    if (restarts) *restarts = H->stat_restarts;
    if (solve_ms) *solve_ms = H->stat_ms;
    return HELM_OK;
}

helm_status helm_get_panel_stats(helm_t H, long long* rhs_applied, long long* rhs_applied_full) {
    if (!H) return HELM_EINVAL;
    if (rhs_applied) *rhs_applied = H->stat_panel;
    if (rhs_applied_full) *rhs_applied_full = H->stat_panel_full;
    return HELM_OK;
}

helm_status helm_get_fusion_stats(helm_t H, long long* fused, long long* unfused) {
    if (!H) return HELM_EINVAL;
    if (fused) *fused = H->stat_fused;
    if (unfused) *unfused = H->stat_unfused;
    return HELM_OK;
}

helm_status helm_get_factor_slots(helm_t H, int* slots, int* strip_slot) {
    if (!H || !slots) return HELM_EINVAL;
    if (!H->t.k2) return fail(H, HELM_ESTATE, "helm_setup did not complete");
    *slots = H->nfac;
    if (strip_slot)
        for (int s = 0; s < H->g.J; ++s) strip_slot[s] = H->fidx[s];
    return HELM_OK;
}

helm_status helm_get_factor_path(helm_t H, int* path) {
    if (!H || !path) return HELM_EINVAL;
    if (!H->factored) return fail(H, HELM_ESTATE, "helm_get_factor_path before helm_factor");
    *path = H->g.dim == 3 ? H->factor_path : 0;
    return HELM_OK;
}

helm_status helm_set_kernel_timing(helm_t H, int enable) {
    if (!H) return HELM_EINVAL;
    if (enable) {
        if (!H->timer) H->timer = new EventTimer();
        HIPCHK(H->st ? hipStreamSynchronize(H->st) : hipDeviceSynchronize());
        H->timer->reset();
        H->timer->mask = (unsigned)enable & 0xFFu;
    } else if (H->timer) {
        HIPCHK(H->st ? hipStreamSynchronize(H->st) : hipDeviceSynchronize());
        delete H->timer;
        H->timer = nullptr;
    }
    return HELM_OK;
}

helm_status helm_get_kernel_times(helm_t H, int nclass, int* launches, double* total_ms) {
    if (!H || nclass < 0) return HELM_EINVAL;
    if (!H->timer) return fail(H, HELM_ESTATE, "kernel timing is not enabled");
    HIPCHK(H->st ? hipStreamSynchronize(H->st) : hipDeviceSynchronize());
    H->timer->collect();
    for (int c = 0; c < nclass; ++c) {
        const bool ok = c < helm::K_NCLASS;
        if (launches) launches[c] = ok ? (int)H->timer->counts[c] : 0;
        if (total_ms) total_ms[c] = ok ? H->timer->ms[c] : 0.0;
    }
    return HELM_OK;
}

const char* helm_last_error(helm_t H) { return H ? H->err.c_str() : g_setup_err.c_str(); }

void helm_destroy(helm_t H) {
    if (!H) return;
    if (H->st) (void)hipStreamSynchronize(H->st);
    else (void)hipDeviceSynchronize();
    for (auto& e : H->apg)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (H->fuse_ev) (void)hipEventDestroy(H->fuse_ev);
    if (H->cap_st) (void)hipStreamDestroy(H->cap_st);
    for (hipStream_t q : H->st_c)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : H->ev_c)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : H->st_fac)
        if (q) (void)hipStreamDestroy(q);
    free_work(H->wk);
    delete H->timer;
    if (H->F != H->F64) dfree(H->F);
    if (H->Fs != H->Fs64) dfree(H->Fs);
    dfree(H->F64);
    dfree(H->Fs64);
    dfree(H->Fc);
    dfree(H->Fa);
    dfree(H->Fw);
    dfree(H->d_err);
    for (void* p : H->owned) dfree(p);
    delete H;
}

}  // extern "C"
