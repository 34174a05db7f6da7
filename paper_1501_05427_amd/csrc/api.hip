// C ABI of the library: argument validation, the per-handle workspace and the host-side
// orchestration of the kernels (covariance products, ULISSE iterations, gradient
// assembly, SGLD update).  Nothing here computes on the host beyond launch shapes.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <vector>

#include "gp_common.h"
#include "internal.h"
#include "learned.h"
#include "solver.h"
#include "ulisse_gp.h"

using namespace gpk;

namespace {

thread_local char g_err[512] = "";

gp_status fail(gp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define GP_HIP(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(GP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define GP_CHECK(cond, ...)                                  \
    do {                                                     \
        if (!(cond)) return fail(GP_EINVAL, __VA_ARGS__);    \
    } while (0)

enum Slot {
    kSlotZ, kSlotKP, kSlotVP, kSlotPart, kSlotQ, kSlotS, kSlotE, kSlotD, kSlotP1, kSlotP2,
    kSlotCounter, kSlotActive, kSlotState, kSlotStats, kSlotR, kSlotB, kSlotSt, kSlotS0,
    kSlotA32, kSlotB32, kSlotGpart, kSlotWork, kSlotVH, kSlotVL, kSlotGbatch, kSlotGvec,
    kSlotRatio, kSlotRunStats, kSlotZp, kSlotUtv, kSlotHW, kSlotP3, kSlotY0, kSlotY1,
    kSlotY2, kSlotGram, kSlotGpart2, kSlotSmall, kSlotMlp, kSlotIcgB, kSlotIcgZ, kSlotIcgSt,
    kSlotIcgKP, kSlotTuneV, kSlotTunePart, kSlotTuneVH, kSlotTuneVL, kSlotAH, kSlotAL, kSlotBH,
    kSlotBL, kSlotRD, kSlotRPart, kSlotRFlag, kSlotProbe, kSlotBroken, kNumSlots
};
// Solves nest one level (the inner CG of the shifted preconditioner): the inner solve's
// buffers live in a second set of slots, offset by kNumSlots.
constexpr int kLevels = 2;

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

struct gp_handle {
    int device = 0;
    uint64_t seed = 0;
    void* buf[kLevels * kNumSlots] = {};
    size_t bytes[kLevels * kNumSlots] = {};
    // two words per solve level: systems still running after iteration it (it % 2)
    int* pinned = nullptr;
    double* pinned_d = nullptr;  // one word read back by sgld_run (Langevin-phase ratio)
    hipEvent_t ev[2 * kLevels] = {};
    // kernel timing (gp_profile)
    bool prof = false;
    std::vector<hipEvent_t> pool;
    std::vector<hipEvent_t> kmv_ev, dq_ev;  // start/stop pairs
    std::vector<hipEvent_t> kmv_main_ev;    // start / end-of-main-kernel pairs of the products
    int64_t solves = 0, passes = 0;
    // set only by the batched path: step word and step size read from device memory
    const uint64_t* dyn_step = nullptr;
    const uint64_t* dyn_probe_step = nullptr;
    const double* dyn_eps = nullptr;
    // autotuner: (n_pad, d, mp, prec) -> shape code of the covariance product (0 symmetric,
    // c > 0 split-K for about c workgroups); pins apply always, tuned entries with autotune
    bool autotune = false;
    std::map<std::array<int64_t, 4>, int> tuned;
    std::map<std::array<int64_t, 4>, int> pinned_shape;
    // work table of the gradient reduction currently in the workspace
    int64_t work_npad = -1;
    int work_L = -1;
    void* work_ptr = nullptr;
};

namespace {

// Grow-only workspace slot; growing waits for the device so no queued kernel still uses
// the old buffer.  Fresh buffers are zeroed.
gp_status ensure(gp_handle* h, int slot, size_t bytes, void** out) {
    bytes = std::max<size_t>(bytes, 256);
    if (h->bytes[slot] < bytes) {
        GP_HIP(hipDeviceSynchronize());
        if (h->buf[slot]) GP_HIP(hipFree(h->buf[slot]));
        h->buf[slot] = nullptr;
        h->bytes[slot] = 0;
        const size_t rb = (size_t)round_up((int64_t)bytes, 1 << 16);
        if (hipMalloc(&h->buf[slot], rb) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GP_ENOMEM, "workspace allocation of %zu bytes failed", rb);
        }
        GP_HIP(hipMemset(h->buf[slot], 0, rb));
        h->bytes[slot] = rb;
    }
    *out = h->buf[slot];
    return GP_OK;
}

template <typename T>
gp_status ws(gp_handle* h, int slot, size_t count, T** out) {
    void* p = nullptr;
    gp_status st = ensure(h, slot, count * sizeof(T), &p);
    *out = static_cast<T*>(p);
    return st;
}

#define GP_TRY(expr)                    \
    do {                                \
        gp_status s_ = (expr);          \
        if (s_ != GP_OK) return s_;     \
    } while (0)

hipEvent_t take_event(gp_handle* h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Record a start event before a timed launch (nullptr when timing is off).
hipEvent_t prof_start(gp_handle* h, hipStream_t s) {
    if (!h->prof) return nullptr;
    hipEvent_t e = take_event(h);
    if (e) (void)hipEventRecord(e, s);
    return e;
}

void prof_stop(gp_handle* h, hipEvent_t start, std::vector<hipEvent_t>& into, hipStream_t s) {
    if (!start) return;
    hipEvent_t e = take_event(h);
    if (!e) return;
    (void)hipEventRecord(e, s);
    into.push_back(start);
    into.push_back(e);
}

// A second start and an end event for the main product kernel (nullptr when timing is off).
void prof_main(gp_handle* h, hipStream_t s, hipEvent_t* start, hipEvent_t* end) {
    *start = prof_start(h, s);
    *end = *start ? take_event(h) : nullptr;
    if (*start && !*end) {
        h->pool.push_back(*start);
        *start = nullptr;
    }
}

void prof_main_keep(gp_handle* h, hipEvent_t start, hipEvent_t end) {
    if (!start) return;
    h->kmv_main_ev.push_back(start);
    h->kmv_main_ev.push_back(end);
}

void prof_drop_last(gp_handle* h, std::vector<hipEvent_t>& v) {
    if (v.size() < 2) return;
    h->pool.push_back(v.back());
    v.pop_back();
    h->pool.push_back(v.back());
    v.pop_back();
}

gp_status check_handle(gp_handle* h) {
    GP_CHECK(h != nullptr, "null handle");
    GP_HIP(hipSetDevice(h->device));
    return GP_OK;
}

gp_status check_data(const gp_data& X) {
    GP_CHECK(X.X != nullptr, "X is null");
    GP_CHECK(aligned(X.X, 4), "X must be 4-byte aligned");
    GP_CHECK(X.n >= 1 && X.n <= (int64_t(1) << 26), "n = %lld outside [1, 2^26]", (long long)X.n);
    GP_CHECK(X.d >= 1 && X.d <= kMaxD, "d = %d outside [1, 16]", X.d);
    GP_CHECK(X.ldx >= X.d, "ldx = %lld < d", (long long)X.ldx);
    return GP_OK;
}

gp_status check_params(const ulisse_params* p) {
    GP_CHECK(p != nullptr, "params is null");
    GP_CHECK(p->q >= 0.0, "q must be >= 0");
    GP_CHECK(p->rate > 0.0, "rate must be > 0");
    GP_CHECK(p->eps >= 0.0, "eps must be >= 0");
    GP_CHECK(p->max_iter >= 1, "max_iter must be >= 1");
    GP_CHECK(p->refresh >= 0 && p->refresh <= 30, "refresh must be in [0, 30]");
    GP_CHECK(p->prec == GP_FP32 || p->prec == GP_BF16_SPLIT_V || p->prec == GP_BF16_SPLIT_KV,
             "unknown precision");
    return GP_OK;
}

// psi -> KParams and scaled inputs in the workspace.
gp_status prep(gp_handle* h, const gp_data& X, const double* psi, int64_t n_pad, float** Z,
               KParams** kp, hipStream_t s) {
    GP_CHECK(psi != nullptr && aligned(psi, 8), "psi must be a non-null 8-byte aligned pointer");
    GP_TRY(ws(h, kSlotZ, (size_t)n_pad * dpad(X.d), Z));
    GP_TRY(ws(h, kSlotKP, 1, kp));
    GP_HIP(launch_prep(X.X, X.n, X.d, X.ldx, psi, *Z, n_pad, *kp, s));
    return GP_OK;
}

// The ULISSE iterations for m systems whose right-hand sides are B (ld ldb); Z and kp
// already prepared.
gp_status check_precond(const gp_precond* pc, int64_t n) {
    if (pc == nullptr) return GP_OK;
    GP_CHECK(pc->U != nullptr && aligned(pc->U, 4) && pc->ldu >= n, "preconditioner U null, misaligned or ldu < n");
    GP_CHECK(pc->k == 16 || pc->k == 32 || pc->k == 64, "preconditioner rank must be 16, 32 or 64");
    GP_CHECK(pc->coef != nullptr && aligned(pc->coef, 8), "preconditioner coef null or misaligned");
    GP_CHECK(pc->warm_start == 0 || pc->warm_start == 1, "preconditioner warm_start must be 0 or 1");
    GP_CHECK(!pc->warm_start || (pc->c != nullptr && aligned(pc->c, 8)),
             "a preconditioner warm start needs its coefficients c (8-byte aligned)");
    return GP_OK;
}

// Split-K candidates of the autotuner (workgroup targets; duplicates after rounding are
// skipped) and the timing of one candidate: a warm-up launch, then kTuneReps launches.
constexpr int kTuneTargets[] = {256, 512, 1024, 2048, 4096, 8192};
constexpr int kTuneReps = 3;
constexpr int kTuneMaxSplit = 64;
constexpr int kTuneMaxCode = 1 << 20;
constexpr const char* kTuneHeader = "ulisse_gp shape cache v1";

// A candidate of the autotuner: 0 = the symmetric product, else the split-K product for
// about that many workgroups.
KmvShape shape_of_code(int64_t n, int d, int m, gp_precision prec, int code) {
    return code == 0 ? kmv_shape_sym(n, d, m, prec) : kmv_shape_target(n, d, m, prec, code);
}

// The shape of the covariance products for (n, d, m, prec): the default, or with the
// autotuner on, the fastest of the candidates (the symmetric product where it applies and
// the split-K factors), timed once per shape on this handle with the prepared Z and kp
// (the timing synchronises the stream).
std::array<int64_t, 4> tune_key(const KmvShape& base, int d, gp_precision prec) {
    return std::array<int64_t, 4>{base.n_pad, d, base.mp, (int64_t)prec};
}

// The shape code a product of (n, d, m, prec) takes without timing anything: the pin, else
// the tuned entry when the autotuner is on, else the default's; -1 when it must be timed.
int resolved_code(const gp_handle* h, int64_t n, int d, int m, gp_precision prec) {
    const KmvShape base = kmv_shape(n, d, m, prec);
    const auto key = tune_key(base, d, prec);
    auto p = h->pinned_shape.find(key);
    if (p != h->pinned_shape.end()) return p->second;
    if (!h->autotune) return kmv_default_code(n, d, m, prec);
    auto it = h->tuned.find(key);
    return it == h->tuned.end() ? -1 : it->second;
}

gp_status shape_for(gp_handle* h, int64_t n, int d, int m, gp_precision prec, const float* Z,
                    const KParams* kp, hipStream_t s, KmvShape* out) {
    const KmvShape base = kmv_shape(n, d, m, prec);
    const int code = resolved_code(h, n, d, m, prec);
    if (code >= 0) {
        *out = shape_of_code(n, d, m, prec, code);
        return GP_OK;
    }
    const auto key = tune_key(base, d, prec);
    const bool b16 = uses_bf16(base, prec);
    const KmvShape sym = kmv_shape_sym(n, d, m, prec);
    const bool has_sym = sym.sym;
    size_t part_floats = has_sym ? kmv_part_floats(sym) : 0;
    // V for every candidate: the symmetric product may pad to more columns than split-K
    const size_t v_floats = (size_t)base.n_pad * (size_t)std::max(base.mp, has_sym ? sym.mp : 0);
    for (int target : kTuneTargets) {
        const KmvShape sh = kmv_shape_target(n, d, m, prec, target);
        if (sh.split <= kTuneMaxSplit) part_floats = std::max(part_floats, kmv_part_floats(sh));
    }
    float *V, *part;
    uint16_t *VH = nullptr, *VL = nullptr;
    GP_TRY(ws(h, kSlotTuneV, v_floats, &V));
    GP_TRY(ws(h, kSlotTunePart, part_floats, &part));
    if (b16) {
        GP_TRY(ws(h, kSlotTuneVH, v_floats, &VH));
        GP_TRY(ws(h, kSlotTuneVL, v_floats, &VL));
    }
    hipEvent_t e0, e1;
    GP_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GP_EDEVICE, "event creation failed");
    }
    int best_target = kmv_default_code(n, d, m, prec), last_split = -1;
    float best_ms = 1e30f;
    gp_status st = GP_OK;
    std::vector<int> codes;
    if (has_sym) codes.push_back(0);
    for (int target : kTuneTargets) codes.push_back(target);
    for (int target : codes) {
        const KmvShape sh = shape_of_code(n, d, m, prec, target);
        if (!sh.sym) {
            if (sh.split == last_split || sh.split > kTuneMaxSplit) continue;
            last_split = sh.split;
        }
        hipError_t e = launch_kmv_partials(sh, d, Z, V, VH, VL, kp, part, nullptr, prec, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < kTuneReps && e == hipSuccess; ++r)
            e = launch_kmv_partials(sh, d, Z, V, VH, VL, kp, part, nullptr, prec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = fail(GP_EDEVICE, "autotuner launch failed: %s", hipGetErrorString(e));
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best_target = target;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GP_OK) return st;
    h->tuned[key] = best_target;
    *out = shape_of_code(n, d, m, prec, best_target);
    return GP_OK;
}

gp_status check_shift(const gp_shift_precond* sp) {
    if (sp == nullptr) return GP_OK;
    GP_CHECK(std::isfinite(sp->delta) && sp->delta > 0.0, "shift delta must be finite and > 0");
    GP_CHECK(std::isfinite(sp->eps_inner) && sp->eps_inner >= 0.0, "eps_inner must be >= 0");
    GP_CHECK(sp->max_inner >= 1, "max_inner must be >= 1");
    GP_CHECK(sp->prec_inner == GP_FP32 || sp->prec_inner == GP_BF16_SPLIT_V ||
                 sp->prec_inner == GP_BF16_SPLIT_KV,
             "unknown inner precision");
    return GP_OK;
}

// One ULISSE solve in three phases, so that the batched path can capture each phase in a
// graph: begin() sets up buffers, the initial residual and state; step() launches one
// iteration of every running system (its kernels do nothing once none runs); end() copies
// the last CG iterates out.  run() is the eager loop: it polls the device's count of running
// systems one iteration behind the launches.
struct Solve {
    gp_handle* h = nullptr;
    int level = 0, so = 0;
    int64_t n = 0;
    int d = 0, m = 0;
    const float* Z = nullptr;
    const KParams* kp = nullptr;
    ulisse_params p{};
    const gp_precond* pc = nullptr;
    const gp_shift_precond* sp = nullptr;
    hipStream_t s = nullptr;
    KmvShape sh{};
    bool b16 = false;
    SolverArgs a{};
    SysState* states = nullptr;
    uint16_t *DH = nullptr, *DL = nullptr;
    float* kpart = nullptr;
    float* Bin = nullptr;
    double *Zin = nullptr, *Stin = nullptr;
    KParams* kp_in = nullptr;
    ulisse_params ip{};
    int it = 0;  // iterations launched
    // residual replacement: FP32 product of fp32(s) every p.refresh iterations
    KmvShape sh32{};
    float* D32 = nullptr;
    float* kpart32 = nullptr;

    gp_status product(const int* n_active) {
        // the BF16 modes split the FP32 direction into hi + lo halves before each product
        if (b16) GP_HIP(launch_split_bf16(a.D, sh.n_pad * sh.mp, DH, DL, s));
        hipEvent_t t0 = prof_start(h, s), m0, m1;
        prof_main(h, s, &m0, &m1);
        GP_HIP(launch_kmv_partials(sh, d, Z, a.D, DH, DL, kp, kpart, n_active, p.prec, s, m1));
        prof_stop(h, t0, h->kmv_ev, s);
        prof_main_keep(h, m0, m1);
        return GP_OK;
    }

    gp_status run_inner(int first);

    gp_status begin(const float* B, int64_t ldb, const double* S0, double* St, ulisse_sysstat* stats) {
        if (level >= kLevels || (sp != nullptr && level + 1 >= kLevels))
            return fail(GP_EUNSUPPORTED, "solves nest at most %d levels", kLevels);
        so = level * kNumSlots;  // this level's workspace slots
        GP_TRY(shape_for(h, n, d, m, p.prec, Z, kp, s, &sh));
        b16 = uses_bf16(sh, p.prec);
        const int64_t n_pad = sh.n_pad;
        a = SolverArgs{};
        a.n = n;
        a.n_pad = n_pad;
        a.m = m;
        a.mp = sh.mp;
        a.split = sh.split;
        a.nb = solver_blocks(n);
        a.ldb = ldb;
        a.B = B;
        a.S0 = S0;
        GP_TRY(ws(h, kSlotPart + so, kmv_part_floats(sh), &kpart));
        GP_TRY(ws(h, kSlotQ + so, (size_t)n_pad * m, &a.Q));
        GP_TRY(ws(h, kSlotS + so, (size_t)n_pad * m, &a.S));
        GP_TRY(ws(h, kSlotE + so, (size_t)n_pad * m, &a.E));
        GP_TRY(ws(h, kSlotD + so, (size_t)n_pad * sh.mp, &a.D));
        GP_TRY(ws(h, kSlotP1 + so, (size_t)a.nb * m, &a.part));
        GP_TRY(ws(h, kSlotP2 + so, (size_t)a.nb * m, &a.part2));
        GP_TRY(ws(h, kSlotActive + so, 1, &a.n_active));
        GP_TRY(ws(h, kSlotState + so, (size_t)2 * m, &states));
        a.state = states;
        if (stats == nullptr) GP_TRY(ws(h, kSlotStats + so, (size_t)m, &stats));
        a.St = St;
        a.kpart = kpart;
        a.kp = kp;
        a.stats = stats;
        a.q = p.q;
        a.rate = p.rate;
        a.eps = p.eps;
        a.eps_relative = p.eps_relative;
        a.max_iter = p.max_iter;
        a.two_track = p.two_track_first ? 1 : 0;
        a.seed = h->seed;
        a.rng_stream = p.rng_stream;
        a.rng_counter = p.rng_counter;
        a.counter_dev = level == 0 ? h->dyn_step : nullptr;
        if (pc != nullptr) {
            a.pcm = 1;
            a.U = pc->U;
            a.ldu = pc->ldu;
            a.pk = pc->k;
            a.coef = pc->coef;
            a.nb256 = pc_chunks(n);
            GP_TRY(ws(h, kSlotZp + so, (size_t)n_pad * m, &a.Zp));
            GP_TRY(ws(h, kSlotUtv + so, (size_t)a.nb256 * pc->k * m, &a.utv_part));
            GP_TRY(ws(h, kSlotHW + so, (size_t)pc->k * m, &a.HW));
            GP_TRY(ws(h, kSlotP3 + so, (size_t)a.nb256 * m, &a.part3));
        }
        // J = K + delta I: inner solves on the shifted covariance, one level down
        if (sp != nullptr) {
            a.pcm = 2;
            a.nb256 = pc_chunks(n);
            GP_TRY(ws(h, kSlotZp + so, (size_t)n_pad * m, &a.Zp));
            GP_TRY(ws(h, kSlotP3 + so, (size_t)a.nb256 * m, &a.part3));
            GP_TRY(ws(h, kSlotIcgB + so, (size_t)n_pad * m, &Bin));
            GP_TRY(ws(h, kSlotIcgZ + so, (size_t)n * m, &Zin));
            GP_TRY(ws(h, kSlotIcgSt + so, (size_t)n * m, &Stin));
            GP_TRY(ws(h, kSlotIcgKP + so, 1, &kp_in));
            GP_HIP(launch_shift_kp(kp, sp->delta, kp_in, s));
            ip = ulisse_params{};
            ip.q = 0.0;  // no truncation: the inner run is plain CG
            ip.rate = 1.0;
            ip.eps = sp->eps_inner;
            ip.eps_relative = 1;
            ip.max_iter = sp->max_inner;
            ip.prec = sp->prec_inner;
        }
        if (b16) {
            GP_TRY(ws(h, kSlotVH + so, (size_t)n_pad * sh.mp, &DH));
            GP_TRY(ws(h, kSlotVL + so, (size_t)n_pad * sh.mp, &DL));
        }
        if (p.refresh > 0) {
            sh32 = kmv_shape(n, d, m, GP_FP32);
            GP_TRY(ws(h, kSlotRD + so, (size_t)n_pad * sh32.mp, &D32));
            GP_TRY(ws(h, kSlotRPart + so, kmv_part_floats(sh32), &kpart32));
            int* fl;
            GP_TRY(ws(h, kSlotRFlag + so, (size_t)m + 1, &fl));
            a.rflag = fl;
            a.rcount = fl + m;
            a.refresh = p.refresh;
        }
        GP_HIP(launch_zero(a.D, (size_t)n_pad * sh.mp * sizeof(float), s));
        const int warm = S0 != nullptr;
        if (warm) {
            GP_HIP(launch_pack_f64(S0, n, m, a.D, n_pad, s));
            GP_TRY(product(nullptr));
            h->passes += 1;
        }
        GP_HIP(solver_init(a, warm, s));
        if (pc != nullptr) GP_HIP(launch_pc_step(a, 1, s));
        if (sp != nullptr) GP_TRY(run_inner(1));
        GP_HIP(solver_init_state(a, s));
        it = 0;
        return GP_OK;
    }

    gp_status step() {
        GP_TRY(product(a.n_active));
        GP_HIP(solver_reduce(a, s));
        GP_HIP(solver_update(a, s));
        if (p.refresh > 0) {
            // residual replacement, decided on the device: e = b - K s with an FP32 product
            // for the systems whose residual has fallen by 2^refresh (the product and the
            // replacement do nothing when no system replaces)
            GP_HIP(solver_refresh_pack(a, D32, s));
            GP_HIP(launch_kmv_partials(sh32, d, Z, D32, nullptr, nullptr, kp, kpart32, a.rcount,
                                       GP_FP32, s));
            GP_HIP(solver_refresh(a, kpart32, sh32.split, sh32.mp, s));
        }
        if (pc != nullptr) GP_HIP(launch_pc_step(a, 0, s));
        if (sp != nullptr) GP_TRY(run_inner(0));
        SysState* next = states + ((it + 1) & 1) * m;
        GP_HIP(solver_direction(a, next, s));
        a.state = next;
        ++it;
        return GP_OK;
    }

    gp_status run() {
        int* pinned = h->pinned + 2 * level;
        hipEvent_t* ev = h->ev + 2 * level;
        for (int k = 0; k <= p.max_iter; ++k) {
            GP_TRY(step());
            GP_HIP(hipMemcpyAsync(pinned + (k & 1), a.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
            GP_HIP(hipEventRecord(ev[k & 1], s));
            h->passes += 1;
            if (sp != nullptr) {
                // the inner runs synchronise anyway: stop before launching another one
                GP_HIP(hipEventSynchronize(ev[k & 1]));
                if (pinned[k & 1] == 0) break;
            } else if (k >= 1) {
                GP_HIP(hipEventSynchronize(ev[(k - 1) & 1]));
                if (pinned[(k - 1) & 1] == 0) {
                    // this iteration's launches found no running system and did nothing
                    if (h->prof) {
                        prof_drop_last(h, h->kmv_ev);
                        prof_drop_last(h, h->kmv_main_ev);
                    }
                    h->passes -= 1;
                    break;
                }
            }
        }
        return GP_OK;
    }

    // After run(): the number of systems that broke down (synchronises the stream).
    gp_status broken_count(int* out) {
        int* cnt;
        GP_TRY(ws(h, kSlotBroken + so, 1, &cnt));
        GP_HIP(launch_count_flag(a.stats, m, ULISSE_BREAKDOWN, cnt, s));
        int* pinned = h->pinned + 2 * level;
        GP_HIP(hipMemcpyAsync(pinned, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        *out = *pinned;
        return GP_OK;
    }

    gp_status end(double* S_cg) {
        if (level == 0) h->solves += 1;
        if (S_cg != nullptr) GP_HIP(solver_copy_s(a, S_cg, s));
        return GP_OK;
    }
};

// z = J^-1 e by the inner run (its last CG iterate), then Zp, e^T z and (first) d = z
gp_status Solve::run_inner(int first) {
    GP_HIP(launch_icg_rhs(a, Bin, first, s));
    Solve in;
    in.h = h;
    in.level = level + 1;
    in.n = n;
    in.d = d;
    in.m = m;
    in.Z = Z;
    in.kp = kp_in;
    in.p = ip;
    in.s = s;
    GP_TRY(in.begin(Bin, sh.n_pad, nullptr, Stin, nullptr));
    GP_TRY(in.run());
    GP_TRY(in.end(Zin));
    GP_HIP(launch_icg_finish(a, Zin, first, s));
    return GP_OK;
}

gp_status solve_core(gp_handle* h, int64_t n, int d, const float* Z, const KParams* kp,
                     const float* B, int64_t ldb, int m, const double* S0,
                     const ulisse_params& p, double* St, double* S_cg, ulisse_sysstat* stats,
                     hipStream_t s, const gp_precond* pc = nullptr,
                     const gp_shift_precond* sp = nullptr) {
    Solve sv;
    auto solve = [&](const ulisse_params& pr) -> gp_status {
        sv = Solve{};
        sv.h = h;
        sv.n = n;
        sv.d = d;
        sv.m = m;
        sv.Z = Z;
        sv.kp = kp;
        sv.p = pr;
        sv.pc = pc;
        sv.sp = sp;
        sv.s = s;
        GP_TRY(sv.begin(B, ldb, S0, St, stats));
        return sv.run();
    };
    GP_TRY(solve(p));
    if (sv.b16) {
        // BF16 rounding can leave K indefinite (CG breaks down): the whole solve again in
        // FP32 from the same warm starts with the same draws
        int broken = 0;
        GP_TRY(sv.broken_count(&broken));
        if (broken > 0) {
            ulisse_params p32 = p;
            p32.prec = GP_FP32;
            p32.refresh = 0;
            GP_TRY(solve(p32));
            GP_HIP(launch_or_flag(sv.a.stats, m, ULISSE_FP32_RERUN, s));
        }
    }
    return sv.end(S_cg);
}

// One stochastic gradient estimate in phases around its solve: begin() prepares Z, the
// right-hand sides (y and the probes) and the warm starts and begins the solve; end() takes
// the last CG iterates out and runs the fused gradient reduction.
struct Grad {
    gp_handle* h = nullptr;
    gp_data X{};
    const double* psi = nullptr;
    const float* y = nullptr;
    const float* R = nullptr;
    int nr = 0, kind = 0;
    ulisse_params p{};
    double* S_warm = nullptr;
    double* g = nullptr;
    ulisse_sysstat* stats = nullptr;
    hipStream_t s = nullptr;
    float* Z = nullptr;
    KParams* kp = nullptr;
    float* Bm = nullptr;
    double* St = nullptr;
    Solve sv;

    gp_status begin(const gp_precond* pc, const gp_shift_precond* sp) {
        const int64_t n = X.n;
        const int m = 1 + nr;
        GP_TRY(prep(h, X, psi, round_up(n, kRowPad), &Z, &kp, s));
        GP_TRY(ws(h, kSlotB, (size_t)n * m, &Bm));
        GP_HIP(hipMemcpyAsync(Bm, y, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (R == nullptr) {
            GP_HIP(launch_probes(n, nr, kind, h->seed, p.rng_stream, p.rng_counter, Bm + n, n, s,
                                 h->dyn_step));
        } else {
            GP_HIP(hipMemcpyAsync(Bm + n, R, (size_t)n * nr * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
        const double* S0 = nullptr;
        if (pc != nullptr && pc->warm_start) {
            // y starts from U c (the caller's warm start when the preconditioner falls
            // back); the probes from their warm starts when the probes are the caller's
            double* S0b;
            GP_TRY(ws(h, kSlotS0, (size_t)n * m, &S0b));
            if (S_warm != nullptr && R != nullptr)
                GP_HIP(hipMemcpyAsync(S0b, S_warm, (size_t)n * m * sizeof(double), hipMemcpyDeviceToDevice, s));
            else
                GP_HIP(launch_zero(S0b, (size_t)n * m * sizeof(double), s));
            GP_HIP(launch_pc_warm(pc->U, pc->ldu, pc->k, n, pc->c, pc->coef, S_warm, S0b, s));
            S0 = S0b;
        } else if (S_warm != nullptr) {
            if (R == nullptr) {
                double* S0b;
                GP_TRY(ws(h, kSlotS0, (size_t)n * m, &S0b));
                GP_HIP(launch_zero(S0b, (size_t)n * m * sizeof(double), s));
                GP_HIP(hipMemcpyAsync(S0b, S_warm, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                S0 = S0b;
            } else {
                S0 = S_warm;
            }
        }
        GP_TRY(ws(h, kSlotSt, (size_t)n * (m + 1), &St));
        ulisse_params ps = p;
        ps.two_track_first = 1;
        sv = Solve{};
        sv.h = h;
        sv.n = n;
        sv.d = X.d;
        sv.m = m;
        sv.Z = Z;
        sv.kp = kp;
        sv.p = ps;
        sv.pc = pc;
        sv.sp = sp;
        sv.s = s;
        return sv.begin(Bm, n, S0, St, stats);
    }

    // The fused reduction's work table, uploaded when the shape changes (this synchronises:
    // done before any graph capture).
    gp_status work_table(const DquadShape& dq, int2** work) {
        GP_TRY(ws(h, kSlotWork, (size_t)dq.nwg, work));
        if (h->work_npad != dq.n_pad || h->work_L != dq.chunk || h->work_ptr != (void*)*work) {
            std::vector<int2> tab;
            dquad_work(dq, tab);
            GP_HIP(hipStreamSynchronize(s));
            GP_HIP(hipMemcpy(*work, tab.data(), tab.size() * sizeof(int2), hipMemcpyHostToDevice));
            h->work_npad = dq.n_pad;
            h->work_L = dq.chunk;
            h->work_ptr = *work;
        }
        return GP_OK;
    }

    gp_status end() {
        const int64_t n = X.n;
        const int d = X.d;
        const int m = 1 + nr;
        GP_TRY(sv.end(S_warm));
        const float* Rp = Bm + n;
        const DquadShape dq = dquad_shape(n, d, m);
        double* gpart;
        GP_TRY(ws(h, kSlotGpart, (size_t)dq.nwg * (d + 1), &gpart));
        int2* work;
        GP_TRY(work_table(dq, &work));
        if (sv.b16) {
            // BF16 product modes: the G tiles from split BF16 operands as well
            uint16_t *AH, *AL, *BH, *BL;
            GP_TRY(ws(h, kSlotAH, (size_t)dq.n_pad * dq.mqb, &AH));
            GP_TRY(ws(h, kSlotAL, (size_t)dq.n_pad * dq.mqb, &AL));
            GP_TRY(ws(h, kSlotBH, (size_t)dq.n_pad * dq.mqb, &BH));
            GP_TRY(ws(h, kSlotBL, (size_t)dq.n_pad * dq.mqb, &BL));
            GP_HIP(launch_build_ab_bf16(St, Rp, n, n, nr, AH, AL, BH, BL, dq.n_pad, dq.mqb, s));
            hipEvent_t t0 = prof_start(h, s);
            GP_HIP(launch_dquad_bf16(dq, d, Z, AH, AL, BH, BL, kp, work, gpart, s));
            prof_stop(h, t0, h->dq_ev, s);
        } else {
            float *A32, *B32;
            GP_TRY(ws(h, kSlotA32, (size_t)dq.n_pad * dq.mq4, &A32));
            GP_TRY(ws(h, kSlotB32, (size_t)dq.n_pad * dq.mq4, &B32));
            GP_HIP(launch_build_ab(St, Rp, n, n, nr, A32, B32, dq.n_pad, dq.mq4, s));
            hipEvent_t t0 = prof_start(h, s);
            GP_HIP(launch_dquad(dq, d, Z, A32, B32, kp, work, gpart, s));
            prof_stop(h, t0, h->dq_ev, s);
        }
        double* dpart;
        GP_TRY(ws(h, kSlotP2, (size_t)solver_blocks(n), &dpart));
        GP_HIP(launch_grad_finish(St, Rp, n, n, nr, gpart, dq.nwg, d, kp, dpart, g, s));
        return GP_OK;
    }
};

// Bodies of the solve and gradient entry points, shared by their preconditioned forms.
gp_status solve_entry(gp_handle* h, gp_data X, const double* psi, const float* B, int32_t m,
                      int64_t ldb, const double* S0, const ulisse_params* params,
                      const gp_precond* pc, const gp_shift_precond* sp, double* S_tilde,
                      double* S_cg, ulisse_sysstat* stats, void* stream);
gp_status grad_entry(gp_handle* h, gp_data X, const double* psi, const float* y,
                     const float* R, int32_t n_probes, int32_t probe_kind,
                     const ulisse_params* params, const gp_precond* pc,
                     const gp_shift_precond* sp, double* S_warm, double* g,
                     ulisse_sysstat* stats, void* stream);

}  // namespace

extern "C" {

const char* gp_last_error(void) { return g_err; }

gp_status gp_create(gp_handle** out, int device, uint64_t seed) {
    GP_CHECK(out != nullptr, "null output pointer");
    int count = 0;
    GP_HIP(hipGetDeviceCount(&count));
    GP_CHECK(device >= 0 && device < count, "device %d not present (%d devices)", device, count);
    GP_HIP(hipSetDevice(device));
    gp_handle* h = new gp_handle();
    h->device = device;
    h->seed = seed;
    bool ok = hipHostMalloc((void**)&h->pinned, 2 * kLevels * sizeof(int), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&h->pinned_d, sizeof(double), hipHostMallocDefault) == hipSuccess;
    for (int i = 0; ok && i < 2 * kLevels; ++i)
        ok = hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        gp_destroy(h);
        return fail(GP_EDEVICE, "handle setup failed: %s", hipGetErrorString(hipGetLastError()));
    }
    for (int i = 0; i < 2 * kLevels; ++i) h->pinned[i] = 1;
    *out = h;
    return GP_OK;
}

void gp_destroy(gp_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < kLevels * kNumSlots; ++i)
        if (h->buf[i]) (void)hipFree(h->buf[i]);
    for (int i = 0; i < 2 * kLevels; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->pinned_d) (void)hipHostFree(h->pinned_d);
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->kmv_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->kmv_main_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->dq_ev) (void)hipEventDestroy(e);
    delete h;
}

gp_status gp_kmv(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                 int64_t ldv, float* out, int64_t ldo, gp_precision prec, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_CHECK(m >= 1 && m <= kMaxSys, "m = %d outside [1, 64]", m);
    GP_CHECK(V != nullptr && out != nullptr && aligned(V, 4) && aligned(out, 4), "V/out null or misaligned");
    GP_CHECK(ldv >= X.n && ldo >= X.n, "ldv and ldo must be >= n");
    GP_CHECK(prec == GP_FP32 || prec == GP_BF16_SPLIT_V || prec == GP_BF16_SPLIT_KV, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    float* Z;
    KParams* kp;
    GP_TRY(prep(h, X, psi, round_up(X.n, kRowPad), &Z, &kp, s));
    KmvShape sh;
    GP_TRY(shape_for(h, X.n, X.d, m, prec, Z, kp, s, &sh));
    float *Vp, *part;
    GP_TRY(ws(h, kSlotVP, (size_t)sh.n_pad * sh.mp, &Vp));
    GP_TRY(ws(h, kSlotPart, kmv_part_floats(sh), &part));
    GP_HIP(launch_pack(V, X.n, m, ldv, Vp, sh.n_pad, sh.mp, s));
    uint16_t *VH = nullptr, *VL = nullptr;
    if (uses_bf16(sh, prec)) {
        GP_TRY(ws(h, kSlotVH, (size_t)sh.n_pad * sh.mp, &VH));
        GP_TRY(ws(h, kSlotVL, (size_t)sh.n_pad * sh.mp, &VL));
        GP_HIP(launch_split_bf16(Vp, sh.n_pad * sh.mp, VH, VL, s));
    }
    hipEvent_t t0 = prof_start(h, s), m0, m1;
    prof_main(h, s, &m0, &m1);
    GP_HIP(launch_kmv_partials(sh, X.d, Z, Vp, VH, VL, kp, part, nullptr, prec, s, m1));
    prof_stop(h, t0, h->kmv_ev, s);
    prof_main_keep(h, m0, m1);
    GP_HIP(launch_kmv_reduce(sh, part, Vp, kp, X.n, m, out, ldo, s));
    return GP_OK;
}

gp_status gp_kmv_noalloc(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                         int64_t ldv, float* out, int64_t ldo, gp_precision prec, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_CHECK(m >= 1 && m <= kMaxSys, "m = %d outside [1, 64]", m);
    GP_CHECK(V != nullptr && out != nullptr && aligned(V, 4) && aligned(out, 4), "V/out null or misaligned");
    GP_CHECK(ldv >= X.n && ldo >= X.n, "ldv and ldo must be >= n");
    GP_CHECK(psi != nullptr && aligned(psi, 8), "psi must be a non-null 8-byte aligned pointer");
    GP_CHECK(prec == GP_FP32 || prec == GP_BF16_SPLIT_V || prec == GP_BF16_SPLIT_KV, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    // the largest split-K (at most the default shape's) whose buffers fit in the scratch
    auto align = [](size_t b) { return (b + 255) / 256 * 256; };
    auto footprint = [&](const KmvShape& sh, bool b16) {
        size_t b = align((size_t)sh.n_pad * dpad(X.d) * sizeof(float)) + align(sizeof(KParams)) +
                   align((size_t)sh.n_pad * sh.mp * sizeof(float)) +
                   align((size_t)sh.split * sh.mp * sh.n_pad * sizeof(float));
        if (b16) b += 2 * align((size_t)sh.n_pad * sh.mp * sizeof(uint16_t));
        return b;
    };
    KmvShape sh = kmv_shape_target(X.n, X.d, m, prec, 2048);  // split-K: the symmetric form needs far more
    bool b16 = uses_bf16(sh, prec);
    for (int target = 1024; footprint(sh, b16) > kNoAllocScratchBytes && sh.split > 1; target /= 2) {
        sh = kmv_shape_target(X.n, X.d, m, prec, target);
        b16 = uses_bf16(sh, prec);
    }
    if (footprint(sh, b16) > kNoAllocScratchBytes)
        return fail(GP_EINVAL, "gp_kmv_noalloc: n = %lld, d = %d, m = %d needs %zu bytes of scratch, more "
                    "than its fixed %zu", (long long)X.n, X.d, m, footprint(sh, b16), kNoAllocScratchBytes);
    void* base = nullptr;
    {
        const hipError_t e = noalloc_scratch(h->device, &base);
        if (e != hipSuccess) return fail(GP_EDEVICE, "scratch address lookup failed: %s", hipGetErrorString(e));
    }
    unsigned char* p = static_cast<unsigned char*>(base);
    auto take = [&](size_t bytes) {
        void* q = p;
        p += align(bytes);
        return q;
    };
    float* Z = static_cast<float*>(take((size_t)sh.n_pad * dpad(X.d) * sizeof(float)));
    KParams* kp = static_cast<KParams*>(take(sizeof(KParams)));
    float* Vp = static_cast<float*>(take((size_t)sh.n_pad * sh.mp * sizeof(float)));
    float* part = static_cast<float*>(take((size_t)sh.split * sh.mp * sh.n_pad * sizeof(float)));
    uint16_t *VH = nullptr, *VL = nullptr;
    if (b16) {
        VH = static_cast<uint16_t*>(take((size_t)sh.n_pad * sh.mp * sizeof(uint16_t)));
        VL = static_cast<uint16_t*>(take((size_t)sh.n_pad * sh.mp * sizeof(uint16_t)));
    }
    // every scratch word read below is written first in this call (Z, kp by prep; Vp by
    // pack; VH, VL by the split; each chunk's partials by the product), so nothing needs
    // clearing between calls
    GP_HIP(launch_prep(X.X, X.n, X.d, X.ldx, psi, Z, sh.n_pad, kp, s));
    GP_HIP(launch_pack(V, X.n, m, ldv, Vp, sh.n_pad, sh.mp, s));
    if (b16) GP_HIP(launch_split_bf16(Vp, sh.n_pad * sh.mp, VH, VL, s));
    GP_HIP(launch_kmv_partials(sh, X.d, Z, Vp, VH, VL, kp, part, nullptr, prec, s));
    GP_HIP(launch_kmv_reduce(sh, part, Vp, kp, X.n, m, out, ldo, s));
    return GP_OK;
}

gp_status gp_dkmv(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                  int64_t ldv, float* out, int64_t ldo, int64_t block_stride,
                  gp_precision prec, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_CHECK(m >= 1 && m <= kMaxSys, "m = %d outside [1, 64]", m);
    GP_CHECK(V != nullptr && out != nullptr && aligned(V, 4) && aligned(out, 4), "V/out null or misaligned");
    GP_CHECK(ldv >= X.n && ldo >= X.n, "ldv and ldo must be >= n");
    GP_CHECK(block_stride >= ldo * m, "block_stride must be >= ldo * m");
    if (prec != GP_FP32) return fail(GP_EUNSUPPORTED, "gp_dkmv computes in GP_FP32 only");
    hipStream_t s = (hipStream_t)stream;
    const KmvShape sh = dkmv_shape(X.n, X.d, m);
    float* Z;
    KParams* kp;
    GP_TRY(prep(h, X, psi, sh.n_pad, &Z, &kp, s));
    const int mtot = (int)round_up(m, sh.mp);
    float *Vp, *part;
    GP_TRY(ws(h, kSlotVP, (size_t)sh.n_pad * mtot, &Vp));
    GP_TRY(ws(h, kSlotPart, dkmv_part_floats(sh, X.d), &part));
    GP_HIP(launch_pack(V, X.n, m, ldv, Vp, sh.n_pad, mtot, s));
    GP_HIP(launch_dkmv(sh, X.d, Z, Vp, kp, part, X.n, m, out, ldo, block_stride, s));
    return GP_OK;
}

gp_status ulisse_solve(gp_handle* h, gp_data X, const double* psi, const float* B,
                       int32_t m, int64_t ldb, const double* S0, const ulisse_params* params,
                       double* S_tilde, double* S_cg, ulisse_sysstat* stats, void* stream) {
    return ulisse_solve_pc(h, X, psi, B, m, ldb, S0, params, nullptr, S_tilde, S_cg, stats, stream);
}

gp_status ulisse_solve_pc(gp_handle* h, gp_data X, const double* psi, const float* B,
                          int32_t m, int64_t ldb, const double* S0, const ulisse_params* params,
                          const gp_precond* pc, double* S_tilde, double* S_cg,
                          ulisse_sysstat* stats, void* stream) {
    return solve_entry(h, X, psi, B, m, ldb, S0, params, pc, nullptr, S_tilde, S_cg, stats, stream);
}

gp_status ulisse_solve_shift_pc(gp_handle* h, gp_data X, const double* psi, const float* B,
                                int32_t m, int64_t ldb, const double* S0,
                                const ulisse_params* params, const gp_shift_precond* sp,
                                double* S_tilde, double* S_cg, ulisse_sysstat* stats,
                                void* stream) {
    if (sp == nullptr) return fail(GP_EINVAL, "shift preconditioner is null");
    return solve_entry(h, X, psi, B, m, ldb, S0, params, nullptr, sp, S_tilde, S_cg, stats, stream);
}

gp_status gp_stoch_grad(gp_handle* h, gp_data X, const double* psi, const float* y,
                        const float* R, int32_t n_probes, int32_t probe_kind,
                        const ulisse_params* params, double* S_warm, double* g,
                        ulisse_sysstat* stats, void* stream) {
    return gp_stoch_grad_pc(h, X, psi, y, R, n_probes, probe_kind, params, nullptr, S_warm, g,
                            stats, stream);
}

gp_status gp_stoch_grad_pc(gp_handle* h, gp_data X, const double* psi, const float* y,
                           const float* R, int32_t n_probes, int32_t probe_kind,
                           const ulisse_params* params, const gp_precond* pc, double* S_warm,
                           double* g, ulisse_sysstat* stats, void* stream) {
    return grad_entry(h, X, psi, y, R, n_probes, probe_kind, params, pc, nullptr, S_warm, g,
                      stats, stream);
}

gp_status gp_stoch_grad_shift_pc(gp_handle* h, gp_data X, const double* psi, const float* y,
                                 const float* R, int32_t n_probes, int32_t probe_kind,
                                 const ulisse_params* params, const gp_shift_precond* sp,
                                 double* S_warm, double* g, ulisse_sysstat* stats,
                                 void* stream) {
    if (sp == nullptr) return fail(GP_EINVAL, "shift preconditioner is null");
    return grad_entry(h, X, psi, y, R, n_probes, probe_kind, params, nullptr, sp, S_warm, g,
                      stats, stream);
}

}  // extern "C"

namespace {

gp_status solve_entry(gp_handle* h, gp_data X, const double* psi, const float* B, int32_t m,
                      int64_t ldb, const double* S0, const ulisse_params* params,
                      const gp_precond* pc, const gp_shift_precond* sp, double* S_tilde,
                      double* S_cg, ulisse_sysstat* stats, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_TRY(check_params(params));
    GP_CHECK(m >= 1 && m + (params->two_track_first ? 1 : 0) <= kMaxSys, "too many systems");
    GP_CHECK(B != nullptr && aligned(B, 4) && ldb >= X.n, "B null, misaligned or ldb < n");
    GP_CHECK(S_tilde != nullptr && aligned(S_tilde, 8), "S_tilde null or misaligned");
    GP_CHECK(S0 == nullptr || aligned(S0, 8), "S0 misaligned");
    GP_CHECK(S_cg == nullptr || aligned(S_cg, 8), "S_cg misaligned");
    GP_TRY(check_precond(pc, X.n));
    GP_TRY(check_shift(sp));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_pad = round_up(X.n, kRowPad);
    float* Z;
    KParams* kp;
    GP_TRY(prep(h, X, psi, n_pad, &Z, &kp, s));
    if (pc != nullptr && pc->warm_start) {
        // system 0 starts from U c (from its column of S0 when the preconditioner falls back)
        double* S0b;
        GP_TRY(ws(h, kSlotS0, (size_t)X.n * m, &S0b));
        if (S0 != nullptr)
            GP_HIP(hipMemcpyAsync(S0b, S0, (size_t)X.n * m * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
            GP_HIP(launch_zero(S0b, (size_t)X.n * m * sizeof(double), s));
        GP_HIP(launch_pc_warm(pc->U, pc->ldu, pc->k, X.n, pc->c, pc->coef, S0, S0b, s));
        S0 = S0b;
    }
    return solve_core(h, X.n, X.d, Z, kp, B, ldb, m, S0, *params, S_tilde, S_cg, stats, s, pc, sp);
}

gp_status grad_entry(gp_handle* h, gp_data X, const double* psi, const float* y,
                     const float* R, int32_t n_probes, int32_t probe_kind,
                     const ulisse_params* params, const gp_precond* pc,
                     const gp_shift_precond* sp, double* S_warm, double* g,
                     ulisse_sysstat* stats, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_TRY(check_params(params));
    GP_CHECK(n_probes >= 1 && n_probes + 2 <= kMaxSys, "n_probes = %d outside [1, 62]", n_probes);
    GP_CHECK(probe_kind == 0 || probe_kind == 1, "probe_kind must be 0 or 1");
    GP_CHECK(y != nullptr && aligned(y, 4), "y null or misaligned");
    GP_CHECK(R == nullptr || aligned(R, 4), "R misaligned");
    GP_CHECK(g != nullptr && aligned(g, 8), "g null or misaligned");
    GP_CHECK(S_warm == nullptr || aligned(S_warm, 8), "S_warm misaligned");
    GP_TRY(check_precond(pc, X.n));
    GP_TRY(check_shift(sp));
    Grad gr;
    gr.h = h;
    gr.X = X;
    gr.psi = psi;
    gr.y = y;
    gr.R = R;
    gr.nr = n_probes;
    gr.kind = probe_kind;
    gr.p = *params;
    gr.S_warm = S_warm;
    gr.g = g;
    gr.stats = stats;
    gr.s = (hipStream_t)stream;
    GP_TRY(gr.begin(pc, sp));
    GP_TRY(gr.sv.run());
    if (gr.sv.b16) {
        // as in solve_core: a breakdown under BF16 products reruns the solve in FP32 (same
        // probes, warm starts and draws); the gradient reduction then runs in FP32 too
        int broken = 0;
        GP_TRY(gr.sv.broken_count(&broken));
        if (broken > 0) {
            gr.p.prec = GP_FP32;
            gr.p.refresh = 0;
            GP_TRY(gr.begin(pc, sp));
            GP_TRY(gr.sv.run());
            GP_HIP(launch_or_flag(gr.sv.a.stats, gr.sv.m, ULISSE_FP32_RERUN, gr.s));
        }
    }
    return gr.end();
}

}  // namespace

extern "C" {

gp_status sgld_run(gp_handle* h, gp_data X, double* psi, const float* y,
                   const ulisse_params* params, const gp_prior* prior, const double* M_chol,
                   const sgld_schedule* sched, sgld_state* state, int32_t T, double* S_warm,
                   float* R, double* trace, double* eps_trace, double* ratio_trace,
                   void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_TRY(check_params(params));
    GP_CHECK(sched != nullptr && state != nullptr, "schedule and state are required");
    GP_CHECK(sched->batch >= 2 && sched->probe_period >= 1 && T >= 0, "batch >= 2, probe_period >= 1, T >= 0");
    GP_CHECK(sched->n_probes >= 1 && sched->n_probes + 2 <= kMaxSys, "n_probes outside [1, 62]");
    GP_CHECK(sched->probe_kind == 0 || sched->probe_kind == 1, "probe_kind must be 0 or 1");
    GP_CHECK(state->t >= 0, "state->t must be >= 0");
    GP_CHECK(S_warm != nullptr && R != nullptr && psi != nullptr && y != nullptr,
             "psi, y, S_warm and R are required");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = X.n;
    const int P = X.d + 2;
    const int nr = sched->n_probes;
    double *G, *gvec, *ratio_dev;
    ulisse_sysstat* st;
    GP_TRY(ws(h, kSlotGbatch, (size_t)sched->batch * P, &G));
    GP_TRY(ws(h, kSlotGvec, (size_t)P, &gvec));
    GP_TRY(ws(h, kSlotRatio, 1, &ratio_dev));
    GP_TRY(ws(h, kSlotRunStats, (size_t)(1 + nr), &st));
    std::vector<double> eps_h, ratio_h;
    eps_h.reserve(T);
    for (int32_t k = 0; k < T; ++k) {
        const int64_t t = state->t;
        if (t % sched->probe_period == 0) {
            GP_HIP(launch_probes(n, nr, sched->probe_kind, h->seed, params->rng_stream,
                                 (uint64_t)(t / sched->probe_period), R, n, s));
            GP_HIP(hipMemsetAsync(S_warm + n, 0, (size_t)n * nr * sizeof(double), s));
        }
        ulisse_params p = *params;
        p.rng_counter = (uint64_t)t;
        GP_TRY(gp_stoch_grad(h, X, psi, y, R, nr, sched->probe_kind, &p, S_warm, gvec, st, stream));
        GP_HIP(hipMemcpyAsync(G + (t % sched->batch) * P, gvec, P * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        const double eps = state->frozen ? state->eps_frozen
                                         : sched->a * std::pow(sched->b + (double)t, -sched->gamma);
        eps_h.push_back(eps);
        GP_TRY(sgld_step(h, P, psi, gvec, prior, M_chol, eps, params->rng_stream, (uint64_t)t, stream));
        if (trace) GP_HIP(hipMemcpyAsync(trace + (int64_t)k * P, psi, P * sizeof(double), hipMemcpyDeviceToDevice, s));
        if ((t + 1) % sched->batch == 0) {
            GP_HIP(launch_langevin_ratio(G, sched->batch, P, M_chol, eps, ratio_dev, s));
            double r = 0.0;
            GP_HIP(hipMemcpyAsync(h->pinned_d, ratio_dev, sizeof(double), hipMemcpyDeviceToHost, s));
            GP_HIP(hipStreamSynchronize(s));
            r = *h->pinned_d;
            ratio_h.push_back(r);
            if (!state->frozen && r < sched->freeze_ratio) {
                state->frozen = 1;
                state->frozen_at = (int32_t)t;
                state->eps_frozen = eps;
            }
        }
        state->t = t + 1;
    }
    GP_HIP(hipStreamSynchronize(s));
    if (eps_trace && !eps_h.empty())
        GP_HIP(hipMemcpy(eps_trace, eps_h.data(), eps_h.size() * sizeof(double), hipMemcpyHostToDevice));
    if (ratio_trace && !ratio_h.empty())
        GP_HIP(hipMemcpy(ratio_trace, ratio_h.data(), ratio_h.size() * sizeof(double), hipMemcpyHostToDevice));
    return GP_OK;
}

}  // extern "C"

namespace {

// One FP32 covariance product of a padded n_pad x mp block (ld n_pad) into out (ld ldo).
gp_status product_padded(gp_handle* h, const KmvShape& sh, int d, const float* Z, const KParams* kp,
                         const float* Vp, int m, float* out, int64_t ldo, int64_t n, hipStream_t s) {
    float* part;
    GP_TRY(ws(h, kSlotPart, kmv_part_floats(sh), &part));
    GP_HIP(launch_kmv_partials(sh, d, Z, Vp, nullptr, nullptr, kp, part, nullptr, GP_FP32, s));
    GP_HIP(launch_kmv_reduce(sh, part, Vp, kp, n, m, out, ldo, s));
    return GP_OK;
}

gp_status check_k(int32_t k) {
    GP_CHECK(k == 16 || k == 32 || k == 64, "k must be 16, 32 or 64");
    return GP_OK;
}

gp_status check_mlp(int32_t in, int32_t hidden, int32_t out) {
    GP_CHECK(in >= 1 && in <= kMaxP && hidden >= 1 && hidden <= 1024 && out >= 1 && out <= 1024,
             "MLP sizes outside the supported range");
    return GP_OK;
}

}  // namespace

extern "C" {

gp_status precond_build_basis(gp_handle* h, gp_data X, const double* psi_ref, int32_t k,
                              float* U, int64_t ldu, double* ritz, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_TRY(check_k(k));
    GP_CHECK(X.n > k, "n must exceed k");
    GP_CHECK(U != nullptr && aligned(U, 4) && ldu >= X.n, "U null, misaligned or ldu < n");
    GP_CHECK(ritz != nullptr && aligned(ritz, 8), "ritz null or misaligned");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = X.n;
    const KmvShape sh = kmv_shape(n, X.d, k, GP_FP32);
    const int64_t np = sh.n_pad;
    float *Z, *Y0, *Y1, *Y2;
    KParams* kp;
    GP_TRY(prep(h, X, psi_ref, np, &Z, &kp, s));
    GP_TRY(ws(h, kSlotY0, (size_t)np * k, &Y0));
    GP_TRY(ws(h, kSlotY1, (size_t)np * k, &Y1));
    GP_TRY(ws(h, kSlotY2, (size_t)np * k, &Y2));
    double *gpart, *small;
    int* status;
    GP_TRY(ws(h, kSlotGpart2, (size_t)ts_blocks(n) * k * k, &gpart));
    GP_TRY(ws(h, kSlotSmall, (size_t)4 * k * k + 64, &small));
    double* G = small;
    double* M = small + k * k;
    double* Q = small + 2 * k * k;
    status = reinterpret_cast<int*>(small + 4 * k * k);
    for (float* b : {Y0, Y1, Y2}) GP_HIP(hipMemsetAsync(b, 0, (size_t)np * k * sizeof(float), s));
    GP_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
    // orthonormal columns of src into dst (tmp as scratch): a shifted CholeskyQR pass, then
    // an unshifted one
    auto orth = [&](const float* src, float* tmp, float* dst) -> gp_status {
        GP_HIP(launch_gram(src, np, k, src, np, k, n, gpart, G, s));
        GP_HIP(launch_chol_inv(G, k, 1e-5, M, status, s));
        GP_HIP(launch_right_mul(src, np, tmp, np, k, n, M, s));
        GP_HIP(launch_gram(tmp, np, k, tmp, np, k, n, gpart, G, s));
        GP_HIP(launch_chol_inv(G, k, 0.0, M, status, s));
        GP_HIP(launch_right_mul(tmp, np, dst, np, k, n, M, s));
        return GP_OK;
    };
    // subspace iteration from a Gaussian block: two products, orthonormalised after each
    GP_HIP(launch_omega(n, k, np, h->seed, 0, Y0, s));
    GP_TRY(product_padded(h, sh, X.d, Z, kp, Y0, k, Y1, np, n, s));
    GP_TRY(orth(Y1, Y0, Y2));
    GP_TRY(product_padded(h, sh, X.d, Z, kp, Y2, k, Y1, np, n, s));
    GP_TRY(orth(Y1, Y0, Y2));
    // Rayleigh-Ritz: T = U^T K U, U <- U Q
    GP_TRY(product_padded(h, sh, X.d, Z, kp, Y2, k, Y0, np, n, s));
    GP_HIP(launch_gram(Y2, np, k, Y0, np, k, n, gpart, G, s));
    GP_HIP(launch_jacobi_eig(G, k, Q, ritz, s));
    GP_HIP(launch_right_mul(Y2, np, U, ldu, k, n, Q, s));
    int st = 0;
    GP_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    GP_CHECK(st == 0, "the range-finder block was rank deficient (Cholesky of its Gram matrix failed)");
    return GP_OK;
}

gp_status precond_targets(gp_handle* h, gp_data X, const float* y, const float* U, int64_t ldu,
                          int32_t k, const double* psis, int32_t N, float* targets, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_data(X));
    GP_TRY(check_k(k));
    GP_CHECK(y && U && psis && targets && N >= 1 && ldu >= X.n && X.n > k, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = X.n;
    const int P = X.d + 2;
    const KmvShape sh = kmv_shape(n, X.d, k, GP_FP32);
    const int64_t np = sh.n_pad;
    float *Up, *KU;
    double *gpart, *small;
    GP_TRY(ws(h, kSlotY1, (size_t)np * k, &Up));
    GP_TRY(ws(h, kSlotY2, (size_t)np * k, &KU));
    GP_TRY(ws(h, kSlotGpart2, (size_t)ts_blocks(n) * k * k, &gpart));
    GP_TRY(ws(h, kSlotSmall, (size_t)4 * k * k + 64, &small));
    GP_HIP(launch_pack(U, n, k, ldu, Up, np, k, s));
    double* T = small;
    double* w = small + k * k;
    for (int i = 0; i < N; ++i) {
        float* Z;
        KParams* kp;
        GP_TRY(prep(h, X, psis + (int64_t)i * P, np, &Z, &kp, s));
        GP_TRY(product_padded(h, sh, X.d, Z, kp, Up, k, KU, np, n, s));
        GP_HIP(launch_gram(Up, np, k, KU, np, k, n, gpart, T, s));
        GP_HIP(launch_gram(Up, np, k, y, n, 1, n, gpart, w, s));
        GP_HIP(launch_targets(T, w, k, n, kp, targets + (int64_t)i * (2 * k + 1), s));
    }
    return GP_OK;
}

int64_t precond_mlp_size(int32_t in, int32_t hidden, int32_t out) {
    return mlp_layout(in, hidden, out).total;
}

gp_status precond_mlp_init(gp_handle* h, float* params, int32_t in, int32_t hidden, int32_t out,
                           const double* psis, const float* targets, int32_t N, uint64_t seed,
                           void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_mlp(in, hidden, out));
    GP_CHECK(params && psis && targets && N >= 1, "bad arguments");
    GP_HIP(launch_mlp_init(params, mlp_layout(in, hidden, out), psis, targets, N, seed, 0,
                           (hipStream_t)stream));
    return GP_OK;
}

namespace {
struct MlpWork {
    float *xs, *a1, *a2, *y, *dy, *d2, *d1, *grad;
    double* lpart;
};
gp_status mlp_work(gp_handle* h, const MlpLayout& L, int B, MlpWork* w) {
    const size_t nb = (size_t)(((int64_t)B * L.O + kWG - 1) / kWG);
    const size_t fl = (size_t)B * L.in + 4 * (size_t)B * L.H + 2 * (size_t)B * L.O + L.trainable + 2 * nb + 64;
    float* base;
    GP_TRY(ws(h, kSlotMlp, fl, &base));
    w->xs = base;
    w->a1 = w->xs + (size_t)B * L.in;
    w->a2 = w->a1 + (size_t)B * L.H;
    w->d2 = w->a2 + (size_t)B * L.H;
    w->d1 = w->d2 + (size_t)B * L.H;
    w->y = w->d1 + (size_t)B * L.H;
    w->dy = w->y + (size_t)B * L.O;
    w->grad = w->dy + (size_t)B * L.O;
    float* tail = w->grad + L.trainable;
    tail += (8 - ((uintptr_t)tail / sizeof(float)) % 8) % 8;  // 32-byte alignment for doubles
    w->lpart = reinterpret_cast<double*>(tail);
    return GP_OK;
}
}  // namespace

gp_status precond_mlp_train(gp_handle* h, float* params, float* adam, int32_t in, int32_t hidden,
                            int32_t out, const double* psis, const float* targets, int32_t N,
                            int32_t steps, int32_t first_step, float lr, float* loss_trace,
                            void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_mlp(in, hidden, out));
    GP_CHECK(params && adam && psis && targets && N >= 1 && steps >= 0 && first_step >= 0, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const MlpLayout L = mlp_layout(in, hidden, out);
    MlpWork w;
    GP_TRY(mlp_work(h, L, N, &w));
    float* loss_scratch;
    GP_TRY(ws(h, kSlotRatio, 1, &loss_scratch));
    for (int t = 0; t < steps; ++t) {
        GP_HIP(launch_mlp_forward(params, L, psis, N, w.xs, w.a1, w.a2, w.y, 0, s));
        GP_HIP(launch_mlp_backward(params, L, targets, N, w.xs, w.a1, w.a2, w.y, w.dy, w.d2, w.d1,
                                   w.grad, w.lpart, loss_trace ? loss_trace + t : loss_scratch, s));
        GP_HIP(launch_adam(params, w.grad, adam, adam + L.trainable, L.trainable, lr, first_step + t + 1, s));
    }
    return GP_OK;
}

gp_status precond_mlp_forward(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                              int32_t out, const double* psis, int32_t B, float* Y, int32_t bf16,
                              void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_mlp(in, hidden, out));
    GP_CHECK(params && psis && Y && B >= 1, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const MlpLayout L = mlp_layout(in, hidden, out);
    MlpWork w;
    GP_TRY(mlp_work(h, L, B, &w));
    GP_HIP(launch_mlp_forward(params, L, psis, B, w.xs, w.a1, w.a2, Y, bf16 ? 1 : 0, s));
    return GP_OK;
}

gp_status precond_mlp_grad(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                           int32_t out, const double* psis, const float* targets, int32_t N,
                           float* grad, float* loss, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_mlp(in, hidden, out));
    GP_CHECK(params && psis && targets && grad && loss && N >= 1, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const MlpLayout L = mlp_layout(in, hidden, out);
    MlpWork w;
    GP_TRY(mlp_work(h, L, N, &w));
    GP_HIP(launch_mlp_forward(params, L, psis, N, w.xs, w.a1, w.a2, w.y, 0, s));
    GP_HIP(launch_mlp_backward(params, L, targets, N, w.xs, w.a1, w.a2, w.y, w.dy, w.d2, w.d1, grad,
                               w.lpart, loss, s));
    return GP_OK;
}

gp_status precond_from_mlp(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                           int32_t out, const double* psi, int32_t k, double* coef, double* c,
                           void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_mlp(in, hidden, out));
    GP_TRY(check_k(k));
    GP_CHECK(out == 2 * k + 1, "the network must have 2k + 1 outputs");
    GP_CHECK(params && psi && coef, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const MlpLayout L = mlp_layout(in, hidden, out);
    MlpWork w;
    GP_TRY(mlp_work(h, L, 1, &w));
    GP_HIP(launch_mlp_forward(params, L, psi, 1, w.xs, w.a1, w.a2, w.y, 1, s));
    GP_HIP(launch_mlp_to_precond(w.y, L, k, params, coef, c, s));
    return GP_OK;
}

gp_status precond_from_targets(gp_handle* h, const float* targets, int32_t k, double* coef,
                               double* c, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_k(k));
    GP_CHECK(targets && coef && aligned(targets, 4) && aligned(coef, 8) && (c == nullptr || aligned(c, 8)),
             "bad arguments");
    GP_HIP(launch_targets_to_precond(targets, k, coef, c, (hipStream_t)stream));
    return GP_OK;
}

gp_status precond_warm_start(gp_handle* h, const float* U, int64_t ldu, int32_t k, int64_t n,
                             const double* c, double* s0, void* stream) {
    GP_TRY(check_handle(h));
    GP_TRY(check_k(k));
    GP_CHECK(U && c && s0 && ldu >= n && n >= 1, "bad arguments");
    GP_HIP(launch_warm_from_c(U, ldu, k, n, c, s0, (hipStream_t)stream));
    return GP_OK;
}

gp_status gp_autotune(gp_handle* h, int32_t enable) {
    GP_TRY(check_handle(h));
    h->autotune = enable != 0;
    return GP_OK;
}

gp_status gp_autotune_split(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec,
                            int32_t* split) {
    int32_t code = 0;
    return gp_tune_get(h, n, d, m, prec, &code, split);
}

static gp_status check_tune_args(int64_t n, int32_t d, int32_t m, gp_precision prec) {
    GP_CHECK(n >= 1 && d >= 1 && d <= kMaxD && m >= 1 && m <= kMaxSys, "bad shape (n %lld, d %d, m %d)",
             (long long)n, d, m);
    GP_CHECK(prec == GP_FP32 || prec == GP_BF16_SPLIT_V || prec == GP_BF16_SPLIT_KV, "unknown precision");
    return GP_OK;
}

gp_status gp_tune_set(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec, int32_t code) {
    GP_CHECK(h != nullptr, "null handle");
    GP_TRY(check_tune_args(n, d, m, prec));
    GP_CHECK(code >= -1 && code <= kTuneMaxCode, "shape code %d outside [-1, %d]", code, kTuneMaxCode);
    GP_CHECK(code != 0 || kmv_shape_sym(n, d, m, prec).sym,
             "the symmetric product does not apply to n = %lld, d = %d, m = %d in this precision",
             (long long)n, d, m);
    const auto key = tune_key(kmv_shape(n, d, m, prec), d, prec);
    if (code < 0)
        h->pinned_shape.erase(key);
    else
        h->pinned_shape[key] = code;
    return GP_OK;
}

gp_status gp_tune_get(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec,
                      int32_t* code, int32_t* split) {
    GP_CHECK(h != nullptr, "null handle");
    GP_TRY(check_tune_args(n, d, m, prec));
    GP_CHECK(code != nullptr && split != nullptr, "null output");
    const int c = resolved_code(h, n, d, m, prec);
    *code = c;
    *split = c < 0 ? 0 : shape_of_code(n, d, m, prec, c).split;
    return GP_OK;
}

gp_status gp_shape_query(int64_t n, int32_t d, int32_t m, gp_precision prec, int32_t code,
                         int32_t* code_out, int32_t* split_out, int32_t* mp_out,
                         int64_t* partial_floats) {
    GP_TRY(check_tune_args(n, d, m, prec));
    GP_CHECK(code_out != nullptr && split_out != nullptr && mp_out != nullptr && partial_floats != nullptr,
             "null output");
    GP_CHECK(code >= -1 && code <= kTuneMaxCode, "shape code %d outside [-1, %d]", code, kTuneMaxCode);
    GP_CHECK(code != 0 || kmv_shape_sym(n, d, m, prec).sym,
             "the symmetric product does not apply to n = %lld, d = %d, m = %d in this precision",
             (long long)n, d, m);
    const int c = code < 0 ? kmv_default_code(n, d, m, prec) : code;
    const KmvShape sh = shape_of_code(n, d, m, prec, c);
    *code_out = c;
    *split_out = sh.split;
    *mp_out = sh.mp;
    *partial_floats = (int64_t)kmv_part_floats(sh);
    return GP_OK;
}

gp_status gp_tune_save(const gp_handle* h, const char* path) {
    GP_CHECK(h != nullptr, "null handle");
    GP_CHECK(path != nullptr, "null path");
    FILE* f = std::fopen(path, "w");
    if (f == nullptr) return fail(GP_EINVAL, "cannot open %s for writing", path);
    bool ok = std::fprintf(f, "%s\n", kTuneHeader) > 0;
    for (const auto& kv : h->tuned)
        ok = ok && std::fprintf(f, "%lld %lld %lld %lld %d\n", (long long)kv.first[0], (long long)kv.first[1],
                                (long long)kv.first[2], (long long)kv.first[3], kv.second) > 0;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GP_OK : fail(GP_EINVAL, "writing %s failed", path);
}

gp_status gp_tune_load(gp_handle* h, const char* path) {
    GP_CHECK(h != nullptr, "null handle");
    GP_CHECK(path != nullptr, "null path");
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return fail(GP_EINVAL, "cannot open %s", path);
    char line[256];
    gp_status st = GP_OK;
    std::map<std::array<int64_t, 4>, int> got;
    if (std::fgets(line, sizeof line, f) == nullptr || std::strncmp(line, kTuneHeader, std::strlen(kTuneHeader)) != 0) {
        st = fail(GP_EINVAL, "%s is not a tuning cache (first line must be '%s')", path, kTuneHeader);
    } else {
        int lineno = 1;
        while (std::fgets(line, sizeof line, f) != nullptr) {
            ++lineno;
            long long np, d, mp, pr;
            int code;
            char extra;
            if (std::sscanf(line, "%lld %lld %lld %lld %d %c", &np, &d, &mp, &pr, &code, &extra) != 5 ||
                np < kRowPad || np % kRowPad != 0 || d < 1 || d > kMaxD || mp < 1 || mp > kMaxSys ||
                pr < GP_FP32 || pr > GP_BF16_SPLIT_KV || code < 0 || code > kTuneMaxCode) {
                st = fail(GP_EINVAL, "%s line %d: expected 'n_pad d mp prec code' in range", path, lineno);
                break;
            }
            got[std::array<int64_t, 4>{np, d, mp, pr}] = code;
        }
    }
    std::fclose(f);
    if (st != GP_OK) return st;
    for (const auto& kv : got) h->tuned[kv.first] = kv.second;
    return GP_OK;
}

gp_status gp_pipe_probe(gp_handle* h, int32_t iters, double* ms, double* cycles, void* stream) {
    GP_TRY(check_handle(h));
    GP_CHECK(iters >= 1 && iters <= 1000000 && ms != nullptr && cycles != nullptr, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipDeviceProp_t prop;
    GP_HIP(hipGetDeviceProperties(&prop, h->device));
    // eight waves per SIMD: 4 SIMDs per CU, 4 waves per workgroup
    const int blocks = prop.multiProcessorCount * 8;
    float* out;
    GP_TRY(ws(h, kSlotProbe, (size_t)blocks * 256, &out));
    hipEvent_t e0, e1;
    GP_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GP_EDEVICE, "event creation failed");
    }
    hipError_t e = hipSuccess;
    for (int mode = 0; mode < 6 && e == hipSuccess; ++mode) {
        float t = 0.f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = launch_pipe_probe(mode, blocks, iters, out, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        }
        ms[mode] = t;
        // clock cycles of one iteration of one wave, at the device's peak clock
        const double waves_per_simd = (double)blocks * 4 / (4.0 * prop.multiProcessorCount);
        cycles[mode] = t * 1e-3 * prop.clockRate * 1e3 / (iters * waves_per_simd);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(GP_EDEVICE, "pipe probe failed: %s", hipGetErrorString(e));
    return GP_OK;
}

gp_status gp_profile(gp_handle* h, int32_t enable) {
    GP_TRY(check_handle(h));
    if (enable) {
        for (hipEvent_t e : h->kmv_ev) h->pool.push_back(e);
        for (hipEvent_t e : h->kmv_main_ev) h->pool.push_back(e);
        for (hipEvent_t e : h->dq_ev) h->pool.push_back(e);
        h->kmv_ev.clear();
        h->kmv_main_ev.clear();
        h->dq_ev.clear();
        h->solves = h->passes = 0;
    }
    h->prof = enable != 0;
    return GP_OK;
}

gp_status gp_profile_read(gp_handle* h, gp_profile_stats* out) {
    GP_TRY(check_handle(h));
    GP_CHECK(out != nullptr, "null output");
    auto total = [&](const std::vector<hipEvent_t>& v, double* ms) -> gp_status {
        *ms = 0.0;
        for (size_t k = 0; k + 1 < v.size(); k += 2) {
            GP_HIP(hipEventSynchronize(v[k + 1]));
            float t = 0.f;
            GP_HIP(hipEventElapsedTime(&t, v[k], v[k + 1]));
            *ms += t;
        }
        return GP_OK;
    };
    gp_profile_stats r{};
    GP_TRY(total(h->kmv_ev, &r.kmv_ms));
    GP_TRY(total(h->kmv_main_ev, &r.kmv_main_ms));
    GP_TRY(total(h->dq_ev, &r.dquad_ms));
    r.kmv_launches = (int64_t)(h->kmv_ev.size() / 2);
    r.kmv_main_launches = (int64_t)(h->kmv_main_ev.size() / 2);
    r.dquad_launches = (int64_t)(h->dq_ev.size() / 2);
    r.solves = h->solves;
    r.kmv_passes = h->passes;
    *out = r;
    return GP_OK;
}

gp_status sgld_step(gp_handle* h, int32_t P, double* psi, const double* g,
                    const gp_prior* prior, const double* M_chol, double eps_t,
                    uint64_t rng_stream, uint64_t rng_counter, void* stream) {
    GP_TRY(check_handle(h));
    GP_CHECK(P >= 3 && P <= kMaxP, "P = %d outside [3, 18]", P);
    GP_CHECK(psi != nullptr && g != nullptr && aligned(psi, 8) && aligned(g, 8), "psi/g null or misaligned");
    GP_CHECK(eps_t >= 0.0, "eps_t must be >= 0");
    int kind = prior ? prior->kind : 0;
    GP_CHECK(kind >= 0 && kind <= 2, "prior kind must be 0, 1 or 2");
    const double* pa = prior ? prior->a : nullptr;
    const double* pb = prior ? prior->b : nullptr;
    GP_CHECK(kind == 0 || (pa != nullptr && pb != nullptr), "prior a/b required for kind %d", kind);
    GP_HIP(launch_sgld(P, psi, g, kind, pa, pb, M_chol, eps_t, h->seed, rng_stream, rng_counter,
                       (hipStream_t)stream));
    return GP_OK;
}

gp_status gp_draw_probes(gp_handle* h, int64_t n, int32_t n_probes, int32_t probe_kind,
                         uint64_t rng_stream, uint64_t rng_counter, float* R, int64_t ldr,
                         void* stream) {
    GP_TRY(check_handle(h));
    GP_CHECK(n >= 1 && n_probes >= 1, "n and n_probes must be >= 1");
    GP_CHECK(probe_kind == 0 || probe_kind == 1, "probe_kind must be 0 or 1");
    GP_CHECK(R != nullptr && aligned(R, 4) && ldr >= n, "R null, misaligned or ldr < n");
    GP_HIP(launch_probes(n, n_probes, probe_kind, h->seed, rng_stream, rng_counter, R, ldr,
                         (hipStream_t)stream));
    return GP_OK;
}

gp_status gp_philox(uint64_t k0, uint64_t k1, uint64_t first_block, uint64_t w1, uint64_t w2,
                    uint64_t w3, int64_t nblocks, uint64_t* out, void* stream) {
    GP_CHECK(nblocks >= 0, "nblocks must be >= 0");
    GP_CHECK(out != nullptr && aligned(out, 8), "out null or misaligned");
    if (nblocks == 0) return GP_OK;
    GP_HIP(launch_philox(k0, k1, first_block, w1, w2, w3, nblocks, out, (hipStream_t)stream));
    return GP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Batched SGLD over independent GPs with captured graphs.
// ---------------------------------------------------------------------------------------
struct gp_batch {
    int device = 0;
    int B = 0, nr = 0, kind = 0, period = 1, iters = 8;
    ulisse_params params{};
    std::vector<gp_handle*> hs;
    std::vector<gp_batch_problem> probs;
    std::vector<Grad> grads;
    std::vector<gp_precond> pcs;  // learned preconditioner of each chain (k = 0: none)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;
    hipStream_t cap = nullptr;      // capture stream
    hipEvent_t fork_ev = nullptr;
    uint64_t* dyn = nullptr;        // device: step, probe step, eps (as bits)
    uint64_t* dyn_host = nullptr;   // pinned host copy
    int max_chunks = 2;             // replays of the iteration graph a step may take
    int* active = nullptr;          // device: running systems over all chains, per replay
    int* active_host = nullptr;     // pinned copy
    int pred[2] = {1, 1};           // replays the last step needed: [0] probes kept, [1] redrawn
    // BF16 products: a chain whose solve broke down is redone in FP32 after the step
    bool rerun = false;
    std::vector<double*> bak;       // per chain, device: psi then S_warm as the step began
    int* brk = nullptr;             // device: broken-down systems per chain
    int* brk_host = nullptr;        // pinned copy
    gp_handle* rh = nullptr;        // handle of the reruns (own workspace, seed set per chain)
    const int** counts = nullptr;   // device array of the chains' running-system counters
    hipGraphExec_t pre[2] = {nullptr, nullptr};  // [0] probes kept, [1] probes redrawn
    hipGraphExec_t iter = nullptr, post = nullptr;
    bool counts_ready = false;
    gp_batch_stats st{};
};

namespace {

hipStream_t chain_stream(gp_batch* b, int i) { return b->side[i % (int)b->side.size()]; }

// Probes (when redrawn) and the start of the gradient of chain i, on its stream.
gp_status batch_pre(gp_batch* b, int i, bool redraw) {
    const gp_batch_problem& pr = b->probs[i];
    Grad& gr = b->grads[i];
    gp_handle* h = b->hs[i];
    const int64_t n = pr.X.n;
    hipStream_t s = chain_stream(b, i);
    if (redraw) {
        GP_HIP(launch_probes(n, b->nr, b->kind, h->seed, b->params.rng_stream, 0, pr.R, n, s,
                             h->dyn_probe_step));
        GP_HIP(launch_zero(pr.S_warm + n, (size_t)n * b->nr * sizeof(double), s));
    }
    if (b->rerun) {
        // the state a rerun starts from
        const int P = pr.X.d + 2;
        GP_HIP(launch_copy_f64(pr.psi, b->bak[i], P, s));
        GP_HIP(launch_copy_f64(pr.S_warm, b->bak[i] + P, n * (1 + b->nr), s));
    }
    gr = Grad{};
    gr.h = h;
    gr.X = pr.X;
    gr.psi = pr.psi;
    gr.y = pr.y;
    gr.R = pr.R;
    gr.nr = b->nr;
    gr.kind = b->kind;
    gr.p = b->params;
    gr.S_warm = pr.S_warm;
    gr.g = pr.g;
    gr.stats = pr.stats;
    gr.s = s;
    const gp_precond* pc = nullptr;
    if (pr.mlp != nullptr) {
        // the network at the chain's psi -> the preconditioner's coefficients
        const MlpLayout L = mlp_layout(pr.X.d + 2, pr.mlp_hidden, 2 * pr.k + 1);
        MlpWork w;
        GP_TRY(mlp_work(h, L, 1, &w));
        GP_HIP(launch_mlp_forward(pr.mlp, L, pr.psi, 1, w.xs, w.a1, w.a2, w.y, 1, s));
        GP_HIP(launch_mlp_to_precond(w.y, L, pr.k, pr.mlp, pr.coef, nullptr, s));
        pc = &b->pcs[i];
    }
    return gr.begin(pc, nullptr);
}

// Gradient reduction and SGLD update of chain i.
gp_status batch_post(gp_batch* b, int i) {
    const gp_batch_problem& pr = b->probs[i];
    gp_handle* h = b->hs[i];
    if (b->rerun) {
        const Solve& sv = b->grads[i].sv;
        GP_HIP(launch_count_flag(sv.a.stats, sv.m, ULISSE_BREAKDOWN, b->brk + i, chain_stream(b, i)));
    }
    GP_TRY(b->grads[i].end());
    GP_HIP(launch_sgld(pr.X.d + 2, pr.psi, pr.g, pr.prior.kind, pr.prior.a, pr.prior.b, pr.M_chol,
                       0.0, h->seed, b->params.rng_stream, 0, chain_stream(b, i), h->dyn_step,
                       reinterpret_cast<const double*>(h->dyn_eps)));
    return GP_OK;
}

// Chain i's step again in FP32, from the psi and warm starts it began with and with the
// same probes and draws (the unbatched gp_stoch_grad + sgld_step after a BF16 breakdown).
gp_status batch_rerun(gp_batch* b, int i, uint64_t t, double eps_t, hipStream_t s) {
    const gp_batch_problem& pr = b->probs[i];
    const int P = pr.X.d + 2;
    const int64_t n = pr.X.n;
    GP_HIP(launch_copy_f64(b->bak[i], pr.psi, P, s));
    GP_HIP(launch_copy_f64(b->bak[i] + P, pr.S_warm, n * (1 + b->nr), s));
    gp_handle* h = b->rh;
    h->seed = b->hs[i]->seed;
    Grad gr;
    gr.h = h;
    gr.X = pr.X;
    gr.psi = pr.psi;
    gr.y = pr.y;
    gr.R = pr.R;
    gr.nr = b->nr;
    gr.kind = b->kind;
    gr.p = b->params;
    gr.p.prec = GP_FP32;
    gr.p.refresh = 0;
    gr.p.rng_counter = t;
    gr.S_warm = pr.S_warm;
    gr.g = pr.g;
    gr.stats = pr.stats;
    gr.s = s;
    GP_TRY(gr.begin(pr.mlp != nullptr ? &b->pcs[i] : nullptr, nullptr));
    GP_TRY(gr.sv.run());
    GP_HIP(launch_or_flag(gr.sv.a.stats, gr.sv.m, ULISSE_FP32_RERUN, s));
    GP_TRY(gr.end());
    GP_HIP(launch_sgld(P, pr.psi, pr.g, pr.prior.kind, pr.prior.a, pr.prior.b, pr.M_chol, eps_t,
                       h->seed, b->params.rng_stream, t, s));
    b->st.fp32_reruns += 1;
    return GP_OK;
}

// After a step (complete on s): the chains whose BF16 solve broke down, redone.
gp_status batch_reruns(gp_batch* b, uint64_t t, double eps_t, hipStream_t s) {
    if (!b->rerun) return GP_OK;
    GP_HIP(hipMemcpyAsync(b->brk_host, b->brk, (size_t)b->B * sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int i = 0; i < b->B; ++i)
        if (b->brk_host[i] > 0) {
            GP_TRY(batch_rerun(b, i, t, eps_t, s));
            any = true;
        }
    if (any) GP_HIP(hipStreamSynchronize(s));
    return GP_OK;
}

gp_status fork(gp_batch* b, hipStream_t from) {
    GP_HIP(hipEventRecord(b->fork_ev, from));
    for (hipStream_t s : b->side) GP_HIP(hipStreamWaitEvent(s, b->fork_ev, 0));
    return GP_OK;
}

gp_status join(gp_batch* b, hipStream_t into) {
    for (size_t k = 0; k < b->side.size(); ++k) {
        GP_HIP(hipEventRecord(b->side_ev[k], b->side[k]));
        GP_HIP(hipStreamWaitEvent(into, b->side_ev[k], 0));
    }
    return GP_OK;
}

// Capture `body` (work issued on the side streams between a fork and a join) as a graph.
template <typename F>
gp_status capture(gp_batch* b, hipGraphExec_t* out, F body) {
    GP_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    gp_status st = fork(b, b->cap);
    if (st == GP_OK) st = body();
    if (st == GP_OK) st = join(b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != GP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(GP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(GP_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e2));
    b->st.captures += 1;
    return GP_OK;
}

}  // namespace

extern "C" {

void gp_batch_destroy(gp_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    for (hipGraphExec_t g : {b->pre[0], b->pre[1], b->iter, b->post})
        if (g) (void)hipGraphExecDestroy(g);
    for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->side_ev) (void)hipEventDestroy(e);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->dyn) (void)hipFree(b->dyn);
    if (b->active) (void)hipFree(b->active);
    if (b->counts) (void)hipFree(b->counts);
    if (b->dyn_host) (void)hipHostFree(b->dyn_host);
    if (b->active_host) (void)hipHostFree(b->active_host);
    for (double* p : b->bak)
        if (p) (void)hipFree(p);
    if (b->brk) (void)hipFree(b->brk);
    if (b->brk_host) (void)hipHostFree(b->brk_host);
    if (b->rh) gp_destroy(b->rh);
    for (gp_handle* h : b->hs) gp_destroy(h);
    delete b;
}

gp_status gp_batch_create(gp_batch** out, int device, uint64_t seed, int32_t B,
                          const gp_batch_problem* problems, int32_t n_probes, int32_t probe_kind,
                          int32_t probe_period, const ulisse_params* params,
                          int32_t iters_per_graph, int32_t autotune, int32_t streams) {
    GP_CHECK(out != nullptr && problems != nullptr && B >= 1, "null output, no problems or B < 1");
    GP_TRY(check_params(params));
    GP_CHECK(n_probes >= 1 && n_probes + 2 <= kMaxSys, "n_probes = %d outside [1, 62]", n_probes);
    GP_CHECK(probe_kind == 0 || probe_kind == 1, "probe_kind must be 0 or 1");
    GP_CHECK(probe_period >= 1, "probe_period must be >= 1");
    GP_CHECK(iters_per_graph >= 2 && iters_per_graph % 2 == 0, "iters_per_graph must be even and >= 2");

    GP_CHECK(streams >= 1 && streams <= 64, "streams must be in [1, 64]");
    for (int i = 0; i < B; ++i) {
        const gp_batch_problem& pr = problems[i];
        GP_TRY(check_data(pr.X));
        GP_CHECK(pr.y && pr.psi && pr.S_warm && pr.R && pr.g, "problem %d: y, psi, S_warm, R and g are required", i);
        GP_CHECK(aligned(pr.y, 4) && aligned(pr.R, 4) && aligned(pr.psi, 8) && aligned(pr.S_warm, 8) &&
                     aligned(pr.g, 8) && (pr.M_chol == nullptr || aligned(pr.M_chol, 8)),
                 "problem %d: misaligned pointer", i);
        GP_CHECK(pr.prior.kind >= 0 && pr.prior.kind <= 2 &&
                     (pr.prior.kind == 0 || (pr.prior.a != nullptr && pr.prior.b != nullptr)),
                 "problem %d: bad prior", i);
        if (pr.mlp != nullptr) {
            GP_TRY(check_k(pr.k));
            GP_TRY(check_mlp(pr.X.d + 2, pr.mlp_hidden, 2 * pr.k + 1));
            GP_CHECK(pr.U != nullptr && aligned(pr.U, 4) && pr.ldu >= pr.X.n && pr.coef != nullptr &&
                         aligned(pr.coef, 8) && aligned(pr.mlp, 4),
                     "problem %d: learned preconditioner needs U (ld >= n) and coef", i);
        }
    }
    GP_HIP(hipSetDevice(device));
    gp_batch* b = new gp_batch();
    b->device = device;
    b->B = B;
    b->nr = n_probes;
    b->kind = probe_kind;
    b->period = probe_period;
    b->iters = iters_per_graph;
    b->params = *params;
    b->probs.assign(problems, problems + B);
    b->grads.resize(B);
    b->pcs.resize(B);
    for (int i = 0; i < B; ++i)
        if (problems[i].mlp != nullptr)
            b->pcs[i] = gp_precond{problems[i].U, problems[i].ldu, problems[i].k, 0, problems[i].coef, nullptr};
    auto bail = [&](gp_status st) {
        gp_batch_destroy(b);
        return st;
    };
    b->max_chunks = params->max_iter / iters_per_graph + 2;
    if (hipMalloc((void**)&b->dyn, 3 * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void**)&b->active, (size_t)b->max_chunks * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&b->counts, (size_t)B * sizeof(int*)) != hipSuccess ||
        hipHostMalloc((void**)&b->dyn_host, 3 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->active_host, (size_t)b->max_chunks * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreate(&b->cap) != hipSuccess || hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(GP_ENOMEM, "batch set-up failed"));
    }
    const int ns = std::min(streams, B);
    for (int k = 0; k < ns; ++k) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreate(&s) != hipSuccess || hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (s) (void)hipStreamDestroy(s);
            return bail(fail(GP_EDEVICE, "stream creation failed"));
        }
        b->side.push_back(s);
        b->side_ev.push_back(e);
    }
    for (int i = 0; i < B; ++i) {
        gp_handle* h = nullptr;
        const gp_status st = gp_create(&h, device, seed + (uint64_t)i);
        if (st != GP_OK) return bail(st);
        h->autotune = autotune != 0;
        h->dyn_step = b->dyn;
        h->dyn_probe_step = b->dyn + 1;
        h->dyn_eps = reinterpret_cast<const double*>(b->dyn + 2);
        b->hs.push_back(h);
    }
    b->rerun = params->prec != GP_FP32;
    if (b->rerun) {
        if (hipMalloc((void**)&b->brk, (size_t)B * sizeof(int)) != hipSuccess ||
            hipHostMalloc((void**)&b->brk_host, (size_t)B * sizeof(int), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(GP_ENOMEM, "batch set-up failed"));
        }
        b->bak.assign(B, nullptr);
        for (int i = 0; i < B; ++i) {
            const size_t cnt = (size_t)(problems[i].X.d + 2) + (size_t)problems[i].X.n * (1 + n_probes);
            if (hipMalloc((void**)&b->bak[i], cnt * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                return bail(fail(GP_ENOMEM, "batch set-up failed (state copies)"));
            }
        }
        const gp_status st = gp_create(&b->rh, device, 0);
        if (st != GP_OK) return bail(st);
        b->rh->autotune = autotune != 0;
    }
    *out = b;
    return GP_OK;
}

gp_status gp_batch_step(gp_batch* b, uint64_t t, double eps_t, void* stream) {
    GP_CHECK(b != nullptr, "null batch");
    GP_HIP(hipSetDevice(b->device));
    hipStream_t s = (hipStream_t)stream;
    const bool redraw = t % (uint64_t)b->period == 0;
    // the step words: written to pinned memory, copied in stream order (the previous step
    // has completed: this call returns only then)
    b->dyn_host[0] = t;
    b->dyn_host[1] = t / (uint64_t)b->period;
    std::memcpy(&b->dyn_host[2], &eps_t, sizeof(double));
    GP_HIP(hipMemcpyAsync(b->dyn, b->dyn_host, 3 * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    const bool graphs = b->counts_ready;
    if (!graphs) {
        // eager step: sizes every workspace, tunes the shapes, uploads the work tables
        GP_TRY(fork(b, s));
        for (int i = 0; i < b->B; ++i) GP_TRY(batch_pre(b, i, redraw));
        for (int i = 0; i < b->B; ++i) GP_TRY(b->grads[i].sv.run());
        for (int i = 0; i < b->B; ++i) GP_TRY(batch_post(b, i));
        GP_TRY(join(b, s));
        GP_HIP(hipStreamSynchronize(s));
        GP_TRY(batch_reruns(b, t, eps_t, s));
        std::vector<const int*> cnt(b->B);
        for (int i = 0; i < b->B; ++i) cnt[i] = b->grads[i].sv.a.n_active;
        GP_HIP(hipMemcpy(b->counts, cnt.data(), (size_t)b->B * sizeof(int*), hipMemcpyHostToDevice));
        b->counts_ready = true;
        b->st.eager_steps += 1;
        return GP_OK;
    }
    hipGraphExec_t& pre = b->pre[redraw ? 1 : 0];
    if (pre == nullptr) {
        GP_TRY(capture(b, &pre, [&]() -> gp_status {
            for (int i = 0; i < b->B; ++i) GP_TRY(batch_pre(b, i, redraw));
            return GP_OK;
        }));
    }
    if (b->iter == nullptr) {
        // the chains' solver objects as left by the set-up capture (their buffers do not
        // change between steps); an even count returns each to its first state buffer
        GP_TRY(capture(b, &b->iter, [&]() -> gp_status {
            for (int k = 0; k < b->iters; ++k)
                for (int i = 0; i < b->B; ++i) GP_TRY(b->grads[i].sv.step());
            return GP_OK;
        }));
        for (int i = 0; i < b->B; ++i) b->grads[i].sv.it = 0;
    }
    if (b->post == nullptr) {
        GP_TRY(capture(b, &b->post, [&]() -> gp_status {
            for (int i = 0; i < b->B; ++i) GP_TRY(batch_post(b, i));
            return GP_OK;
        }));
    }
    GP_HIP(hipGraphLaunch(pre, s));
    // Replays of the iteration graph, each followed by the count of systems still running:
    // as many as the last step of the same kind needed are queued back to back, then the
    // host waits once; while some system still runs it goes on one replay at a time.  A
    // replay after every system has stopped changes nothing (each of its kernels returns on
    // the chain's zero count, as they do for a chain that stopped before the others), so
    // one queued too many costs only its launches.
    int& pred = b->pred[redraw ? 1 : 0];
    int c = 0, seen = 0, needed = 0;
    for (;;) {
        const int target = c == 0 ? std::min(std::max(pred, 1), b->max_chunks) : c + 1;
        for (; c < target; ++c) {
            GP_HIP(hipGraphLaunch(b->iter, s));
            GP_HIP(launch_sum_active(b->counts, b->B, b->active + c, s));
            b->st.iteration_graphs += 1;
        }
        GP_HIP(hipMemcpyAsync(b->active_host + seen, b->active + seen, (size_t)(c - seen) * sizeof(int),
                              hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        for (; seen < c; ++seen)
            if (needed == 0 && b->active_host[seen] == 0) needed = seen + 1;
        if (needed != 0 || c >= b->max_chunks) break;
    }
    pred = needed != 0 ? needed : c;
    GP_HIP(hipGraphLaunch(b->post, s));
    GP_HIP(hipStreamSynchronize(s));
    GP_TRY(batch_reruns(b, t, eps_t, s));
    b->st.graph_steps += 1;
    return GP_OK;
}

gp_status gp_batch_read_stats(const gp_batch* b, gp_batch_stats* out) {
    GP_CHECK(b != nullptr && out != nullptr, "null argument");
    *out = b->st;
    return GP_OK;
}

}  // extern "C"
