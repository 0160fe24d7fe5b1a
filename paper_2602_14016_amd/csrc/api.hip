// api.hip -- host side of the C ABI declared in include/pa.h.
//
// The context owns only constant tables (twiddles, 1/|k|^2, integrating
// factors, shell lists).  Every buffer a solve needs is carved from the
// caller's workspace by one layout routine that also answers the size query.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "kernels.hpp"

using namespace pa;

namespace {

thread_local std::string g_err;

pa_status fail(pa_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

// A failed host allocation (a schedule, a table, the context itself) becomes
// PA_ENOMEM: every entry point is a function-try-block closed by this, so no
// C++ exception unwinds through the C ABI.
pa_status fail_host_alloc() noexcept {
    try {
        g_err = "host memory allocation failed";
    } catch (...) {
    }
    return PA_ENOMEM;
}
#define PA_CATCH_HOST \
    catch (...) { return fail_host_alloc(); }

#define PA_HIP(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define PA_TRY(expr)                       \
    do {                                   \
        pa_status s_ = (expr);             \
        if (s_ != PA_OK) return s_;        \
    } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// Every pointer the kernels dereference must be device (or managed) memory: a
// host pointer would fault the device instead of returning an error.  NULL
// entries (optional arguments) pass.  A failed attribute query leaves no
// sticky error behind (it is cleared here).  Skipped while the context's
// stream is being captured into a graph.
struct NamedPtr {
    const void* p;
    const char* name;
};
pa_status require_device(hipStream_t stream, std::initializer_list<NamedPtr> ptrs) {
    // under graph capture the same call has already run eagerly with these pointers
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (stream && hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return PA_OK;
    for (const NamedPtr& q : ptrs) {
        if (!q.p) continue;
        hipPointerAttribute_t at{};
        const hipError_t e = hipPointerGetAttributes(&at, q.p);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(PA_EINVAL, std::string(q.name) + " is not device memory");
        }
        if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged && !at.isManaged)
            return fail(PA_EINVAL, std::string(q.name) + " is not device memory");
    }
    return PA_OK;
}

// One action of a checkpoint schedule over segment boundaries 0..L (segment i
// runs from boundary i to i + 1).  ADVANCE runs segments a .. b-1 without
// keeping their stage fields, starting from snapshot slot src (or from the
// live state, src = -1) and storing the state of boundary b in slot dst (if
// dst >= 0).  REVERSE recomputes segment a keeping its stage fields, from
// slot src (or the live state), and runs the adjoint steps through it.
enum { ACT_ADVANCE = 0, ACT_REVERSE = 1 };
struct PlanAct {
    int kind, a, b, src, dst;
};

}  // namespace

struct pa_ctx {
    Dims d;
    pa_physics ph;
    hipStream_t stream;
    int device;
    cd* tw;             // [N]
    double* invk2;      // [KY][KXP]
    double* ex2;        // [KXP]
    double* ey2;        // [KY]
    int* shell_start;   // [n_shell_max + 1]
    int* shell_modes;
    int n_shell_max;
    double forcing;     // curl-force spectrum value at (0, +-n_f)
    int nf;             // n_f if inside the band, else 0
    double sobolev = 0; // lambda of the Sobolev term (lambda/2) int |grad u0|^2 of the cost
    // snapshot budget of the internal checkpoints (0: one per segment boundary)
    int ckpt_slots = 0;
    const int32_t* cancel = nullptr;   // host [B]: members to stop at the next iteration boundary
    int plan_L = -1, plan_slots = -1;
    std::vector<PlanAct> plan;       // binomial schedule for plan_L segments and plan_slots slots
    std::vector<int> plan_fwd_slot;  // boundary -> slot written by the schedule's first chain (-1: none)
    // launch timing of one kernel class with HIP events on the context stream
    int prof_class = -1;
    int prof_every = 1;
    long prof_seen = 0;
    size_t prof_used = 0;
    std::vector<hipEvent_t> prof_ev;   // pairs (start, stop)
    // (kind, metric, param, power) of multiplier tables already found finite on this grid
    std::vector<std::array<double, 4>> mult_checked;
    // pinned host staging of the optimiser's status reads and mask writes
    void* pin = nullptr;
    size_t pin_bytes = 0;
};

namespace {

// ----------------------------------------------------------- workspace --

struct WS {
    cd* Y0;
    cd* Yf[4];
    cd* Yp[4];
    cd* YL[2];          // Lambda and Lambda_y (adjoint cotangent fields)
    double* P0;         // physical scratch [B][N][N]
    double* P1;         // physical scratch [B][N][N]
    cd* omega;
    cd* omega2;         // the other state buffer: stage D writes the new state there (then swapped)
    cd* acc;
    cd* lam;
    cd* omb;
    cd* seg;            // segment stage fields, (4K+1) slots x 4 fields
    cd* ckpt;           // internal checkpoints
    double* jpart;      // [B][n_obs][N]
    double* J;          // [B]
    double* J2;         // [B]
    double* mult;       // two tables of [B][KY][KXP] (member-major; one kernel per member)
    double* norm;       // [B]
    uint64_t* seeds;    // [B]
    double* partial;    // [B][DOT_BLOCKS]
    double* dots;       // [B][4]
    double* coef;       // [B][8]
    int* active;        // [B]
    // optimiser vectors [B][N*N]
    double *x, *g, *dv, *xt, *gt, *w, *gw;
    double* S;          // [m][B][N*N]
    double* Yv;         // [m][B][N*N]
    // optimiser scalars per member (ring slot p of member b at [p * B + b])
    double *oJ, *oalpha, *ogd, *ogg;   // [B] cost at the iterate, trial step, g.d, g.g
    double *orho, *ogam, *oal;         // [m][B]
    int *ook, *orun, *opend, *oreset;  // [m][B] stored-pair flags; [B] running, pending, reset
    // line-search status, copied to the host after each trial: counts[4] (pending,
    // accepted), acc[B] (accepted this iteration), Jt[B] (accepted trial cost)
    char* ostat;
    size_t total;
};

// Layout of the line-search status block of B members.
struct StatLayout {
    size_t acc, Jt, bytes;
};
StatLayout stat_layout(int B) {
    StatLayout l;
    l.acc = 16;
    l.Jt = (16 + sizeof(int) * (size_t)B + 15) & ~size_t(15);
    l.bytes = l.Jt + sizeof(double) * (size_t)B;
    return l;
}

struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int seg_len(int n_steps, int ckpt_every) { return std::max(1, std::min(ckpt_every, std::max(n_steps, 1))); }
int n_segments(int n_steps, int K) { return n_steps <= 0 ? 0 : (int)(((int64_t)n_steps + K - 1) / K); }

// The internal checkpoints follow a binomial schedule when the snapshot
// budget is set and smaller than one slot per boundary.
bool plan_mode(const pa_ctx* c, int nseg) { return c->ckpt_slots > 0 && c->ckpt_slots <= nseg; }
int ckpt_count(const pa_ctx* c, int nseg) { return plan_mode(c, nseg) ? c->ckpt_slots : nseg + 1; }

WS carve(const pa_ctx* c, int n_steps, int ckpt_every, int n_obs, int m, void* base) {
    const Dims& d = c->d;
    const size_t SY = (size_t)d.B * d.N * d.KXP;
    const size_t SC = (size_t)d.B * d.KY * d.KXP;
    const size_t SP = (size_t)d.B * d.N * d.N;
    const int K = seg_len(n_steps, ckpt_every);
    const int nseg = n_segments(n_steps, K);
    Carver cv{reinterpret_cast<char*>(base)};
    WS w{};
    w.Y0 = cv.take<cd>(SY);
    for (int i = 0; i < 4; ++i) w.Yf[i] = cv.take<cd>(SY);
    for (int i = 0; i < 4; ++i) w.Yp[i] = cv.take<cd>(SY);
    w.YL[0] = cv.take<cd>(SY);
    w.YL[1] = cv.take<cd>(SY);
    w.P0 = cv.take<double>(SP);
    w.P1 = cv.take<double>(SP);
    w.omega = cv.take<cd>(SC);
    w.omega2 = cv.take<cd>(SC);
    w.acc = cv.take<cd>(SC);
    w.lam = cv.take<cd>(SC);
    w.omb = cv.take<cd>(SC);
    w.seg = n_steps > 0 ? cv.take<cd>((size_t)(4 * K + 1) * 4 * SY) : nullptr;
    w.ckpt = cv.take<cd>((size_t)ckpt_count(c, nseg) * SC);
    w.jpart = cv.take<double>((size_t)d.B * std::max(n_obs, 1) * d.N);
    w.J = cv.take<double>(d.B);
    w.J2 = cv.take<double>(d.B);
    w.mult = cv.take<double>((size_t)2 * d.B * d.KY * d.KXP);
    w.norm = cv.take<double>(d.B);
    w.seeds = cv.take<uint64_t>(d.B);
    w.partial = cv.take<double>((size_t)d.B * DOT_BLOCKS);
    w.dots = cv.take<double>((size_t)d.B * 4);
    w.coef = cv.take<double>((size_t)d.B * 8);
    w.active = cv.take<int>(d.B);
    if (m > 0) {
        w.x = cv.take<double>(SP);
        w.g = cv.take<double>(SP);
        w.dv = cv.take<double>(SP);
        w.xt = cv.take<double>(SP);
        w.gt = cv.take<double>(SP);
        w.w = cv.take<double>(SP);
        w.gw = cv.take<double>(SP);
        w.S = cv.take<double>((size_t)m * SP);
        w.Yv = cv.take<double>((size_t)m * SP);
        w.oJ = cv.take<double>(d.B);
        w.oalpha = cv.take<double>(d.B);
        w.ogd = cv.take<double>(d.B);
        w.ogg = cv.take<double>(d.B);
        w.orho = cv.take<double>((size_t)m * d.B);
        w.ogam = cv.take<double>((size_t)m * d.B);
        w.oal = cv.take<double>((size_t)m * d.B);
        w.ook = cv.take<int>((size_t)m * d.B);
        w.orun = cv.take<int>(d.B);
        w.opend = cv.take<int>(d.B);
        w.oreset = cv.take<int>(d.B);
        w.ostat = cv.take<char>(stat_layout(d.B).bytes);
    }
    w.total = cv.off + 256;
    return w;
}

size_t ckpt_bytes(const pa_ctx* c, int n_steps, int ckpt_every) {
    const int K = seg_len(n_steps, ckpt_every);
    return (size_t)(n_segments(n_steps, K) + 1) * c->d.B * c->d.KY * c->d.KXP * sizeof(cd);
}

cd* ckpt_slot(const pa_ctx* c, cd* base, int i) {
    return base + (size_t)i * c->d.B * c->d.KY * c->d.KXP;
}

// 4 stage-field pointers of segment slot (j, s)
void seg_fields(const pa_ctx* c, const WS& w, int j, int s, cd* out[4]) {
    const size_t SY = (size_t)c->d.B * c->d.N * c->d.KXP;
    const size_t slot = (size_t)j * 4 + s;
    for (int f = 0; f < 4; ++f) out[f] = w.seg + (slot * 4 + f) * SY;
}

// ------------------------------------------------- checkpoint schedule --
// Binomial checkpointing (Griewank 1992; Griewank & Walther 2000).  With the
// state of the first boundary held and s free slots, l segments reverse in
// the fewest segment advances, t l - beta(s + 2, t - 1), where beta(a, t) =
// C(a + t, t) and t is the least integer with beta(s + 1, t) >= l; a first
// advance attaining it is min(beta(s + 1, t - 1), l - beta(s, t - 1)).

const int64_t BETA_SAT = int64_t(1) << 62;

// beta(a, t) = C(a + t, t), saturated at BETA_SAT; 0 for t < 0
int64_t beta_sat(int64_t a, int64_t t) {
    if (t < 0) return 0;
    unsigned __int128 r = 1;
    for (int64_t i = 1; i <= t; ++i) {
        r = r * (unsigned __int128)(a + i) / (unsigned __int128)i;   // C(a+i-1, i-1) (a+i) / i is exact
        if (r >= (unsigned __int128)BETA_SAT) return BETA_SAT;
    }
    return (int64_t)r;
}

// least t with beta(s + 1, t) >= l
int64_t repetitions(int64_t l, int64_t s) {
    int64_t t = 0;
    unsigned __int128 b = 1;
    while (b < (unsigned __int128)l) {
        ++t;
        b = b * (unsigned __int128)(s + 1 + t) / (unsigned __int128)t;
    }
    return t;
}

int64_t min_segment_advances(int64_t l, int64_t s) {
    if (l <= 1) return 0;
    if (s == 0) return l * (l - 1) / 2;
    const int64_t t = repetitions(l, s);
    return t * l - beta_sat(s + 2, t - 1);
}

int64_t first_advance(int64_t l, int64_t s) {
    const int64_t t = repetitions(l, s);
    return std::min(beta_sat(s + 1, t - 1), l - beta_sat(s, t - 1));
}

// Schedule reversing L segments with `slots` snapshot slots, slot 0 holding
// boundary 0.  The actions up to the first REVERSE (of segment L-1, from the
// live state) form the forward sweep; the rest run in the backward sweep.
void build_plan(int L, int slots, std::vector<PlanAct>& out) {
    out.clear();
    struct Task {
        int a, b, src, live, free_slot;   // free_slot >= 0: return that slot to the pool
    };
    std::vector<int> pool;
    for (int i = slots - 1; i >= 1; --i) pool.push_back(i);
    std::vector<Task> stack{{0, L, 0, 1, -1}};
    while (!stack.empty()) {
        const Task t = stack.back();
        stack.pop_back();
        if (t.free_slot >= 0) {
            pool.push_back(t.free_slot);
            continue;
        }
        const int l = t.b - t.a;
        const int from = t.live ? -1 : t.src;
        if (l == 1) {
            out.push_back({ACT_REVERSE, t.a, t.a + 1, from, -1});
            continue;
        }
        if (pool.empty()) {
            // no free slot: every segment from the held state
            for (int i = t.b - 1; i > t.a; --i) {
                out.push_back({ACT_ADVANCE, t.a, i, i == t.b - 1 ? from : t.src, -1});
                out.push_back({ACT_REVERSE, i, i + 1, -1, -1});
            }
            out.push_back({ACT_REVERSE, t.a, t.a + 1, t.src, -1});
            continue;
        }
        const int m = t.a + (int)first_advance(l, (int64_t)pool.size());
        const int dst = pool.back();
        pool.pop_back();
        out.push_back({ACT_ADVANCE, t.a, m, from, dst});
        stack.push_back({t.a, m, t.src, 0, -1});
        stack.push_back({0, 0, 0, 0, dst});
        stack.push_back({m, t.b, dst, 1, -1});
    }
}

// the context's schedule for nseg segments, or nullptr for one checkpoint per boundary
const std::vector<PlanAct>* plan_for(pa_ctx* c, int nseg) {
    if (!plan_mode(c, nseg)) return nullptr;
    if (c->plan_L != nseg || c->plan_slots != c->ckpt_slots) {
        build_plan(nseg, c->ckpt_slots, c->plan);
        c->plan_fwd_slot.assign((size_t)nseg + 1, -1);
        for (const PlanAct& a : c->plan) {
            if (a.kind == ACT_REVERSE) break;
            if (a.dst >= 0) c->plan_fwd_slot[(size_t)a.b] = a.dst;
        }
        c->plan_L = nseg;
        c->plan_slots = c->ckpt_slots;
    }
    return &c->plan;
}

// --------------------------------------------------------- validation --

// Observations of a solve as ranges of members [b0, b0 + nb) that share one
// observation set (stride, steps, values): one range when every member has
// the same set (a pa_obs), one per member for per-member sets.  Observation
// work at a step is launched range by range on the members' slices of the
// buffers, so a shared set costs exactly one launch per observed step.
struct ObsRange {
    int b0 = 0, nb = 0;
    int stride = 1, M = 1, n_times = 0;
    const int32_t* steps = nullptr;     // host, strictly increasing
    const double* values = nullptr;     // device [nb][n_times][2][M][M], or null
    size_t jrow0 = 0;                   // first cost-partial row of the range ([nb][n_times][M] rows)
    // index of step n among the observation steps, or -1 (binary search; allocates nothing)
    int slot(int n) const {
        int lo = 0, hi = n_times;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (steps[mid] < n) lo = mid + 1;
            else hi = mid;
        }
        return (lo < n_times && steps[lo] == n) ? lo : -1;
    }
};

struct ObsPlan {
    ObsRange one;                       // storage of a set shared by every member
    const ObsRange* r = nullptr;        // the ranges (n = 0: no observations)
    int n = 0;
    int B = 0;
    bool values = false;                // every range has values: the cost is formed
    int max_times = 0;                  // most observation times of a range
    // active[n]: the members [0, active[n]) advance through step n (n < n_steps); null: all of
    // them at every step.  A member whose last observation is at step L needs steps 0 .. L-1
    // only; members past their horizon keep their buffers untouched.
    const int* active = nullptr;
    int act(int step) const { return active ? active[step] : B; }
};

pa_status check_obs_set(const pa_ctx* c, const pa_obs* obs, int n_steps, bool need_values) {
    if (obs->stride < 1 || obs->stride > c->d.N || c->d.N % obs->stride)
        return fail(PA_EINVAL, "obs stride must divide N");
    if (obs->n_times < 0 || obs->n_times > n_steps + 1) return fail(PA_EINVAL, "bad n_times");
    if (obs->n_times > 0 && !obs->steps) return fail(PA_EINVAL, "obs steps is NULL");
    if (need_values && !obs->values) return fail(PA_EINVAL, "obs values required");
    int prev = -1;
    for (int i = 0; i < obs->n_times; ++i) {
        const int s = obs->steps[i];
        if (s <= prev || s > n_steps) return fail(PA_EINVAL, "obs steps must increase within [0, n_steps]");
        prev = s;
    }
    return PA_OK;
}

void fill_range(const pa_ctx* c, const pa_obs* obs, int b0, int nb, size_t jrow0, ObsRange* r) {
    r->b0 = b0;
    r->nb = nb;
    r->stride = obs->stride;
    r->M = c->d.N / obs->stride;
    r->n_times = obs->n_times;
    r->steps = obs->steps;
    r->values = obs->values;
    r->jrow0 = jrow0;
}

// One observation set for every member (obs may be NULL: no observations).
pa_status make_obs_plan(const pa_ctx* c, const pa_obs* obs, int n_steps, bool need_values, ObsPlan* p) {
    p->B = c->d.B;
    p->n = 0;
    p->r = nullptr;
    p->active = nullptr;
    p->values = false;
    p->max_times = 0;
    if (!obs) {
        if (need_values) return fail(PA_EINVAL, "observations required");
        return PA_OK;
    }
    PA_TRY(check_obs_set(c, obs, n_steps, need_values));
    fill_range(c, obs, 0, c->d.B, 0, &p->one);
    p->r = &p->one;
    p->n = obs->n_times > 0 ? 1 : 0;
    p->values = obs->values != nullptr;
    p->max_times = obs->n_times;
    return PA_OK;
}

// One observation set per member (obs: host array of B, each with values for its own member
// only, [1][n_times][2][M][M]).  n_steps must be the latest observation step of all members.
// Member b advances only through its own last observation step; ranges and active counts live
// in the caller's vectors.
pa_status make_member_plan(const pa_ctx* c, const pa_obs* obs, int n_steps, std::vector<ObsRange>& ranges,
                           std::vector<int>& active, ObsPlan* p) {
    const int B = c->d.B;
    p->B = B;
    ranges.assign((size_t)B, ObsRange());
    std::vector<int> top((size_t)n_steps + 1, 0);   // top[t]: 1 + last member whose horizon is t
    size_t jrow = 0;
    int latest = -1, most = 0;
    for (int b = 0; b < B; ++b) {
        PA_TRY(check_obs_set(c, &obs[b], n_steps, true));
        if (obs[b].n_times < 1) return fail(PA_EINVAL, "every member needs at least one observation time");
        fill_range(c, &obs[b], b, 1, jrow, &ranges[(size_t)b]);
        jrow += (size_t)obs[b].n_times * (size_t)(c->d.N / obs[b].stride);
        const int last = obs[b].steps[obs[b].n_times - 1];
        top[(size_t)last] = b + 1;
        latest = std::max(latest, last);
        most = std::max(most, (int)obs[b].n_times);
    }
    if (latest != n_steps) return fail(PA_EINVAL, "n_steps must equal the latest observation step of the members");
    // active[n] = 1 + last member whose horizon exceeds n (a suffix maximum of top)
    active.assign((size_t)n_steps + 1, 0);
    int run = 0;
    for (int t = n_steps; t >= 0; --t) {
        active[(size_t)t] = run;          // members with horizon > t
        run = std::max(run, top[(size_t)t]);
    }
    p->r = ranges.data();
    p->n = B;
    p->values = true;
    p->max_times = most;
    p->active = active.data();
    return PA_OK;
}

// `scheduled`: the solve reverses its segments by the context's schedule
// (plan_for), whose size is checked here, before anything is enqueued
pa_status check_ws(const pa_ctx* c, void* ws, size_t bytes, int n_steps, int K, int n_obs, int m, WS* out,
                   bool scheduled = false) {
    if (!ws) return fail(PA_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PA_EINVAL, "workspace must be 256-byte aligned");
    if (scheduled && plan_mode(c, n_segments(n_steps, K)) && n_segments(n_steps, K) > PA_MAX_SCHEDULE_SEGMENTS)
        return fail(PA_EINVAL, "binomial schedule over more than PA_MAX_SCHEDULE_SEGMENTS segments: "
                               "raise ckpt_every");
    WS w = carve(c, n_steps, K, n_obs, m, ws);
    if (w.total > bytes)
        return fail(PA_ENOMEM, "workspace too small: need " + std::to_string(w.total) + " bytes");
    *out = w;
    return PA_OK;
}

// ------------------------------------------------------------- timing --
// Kernel classes that pa_profile_start can time.
enum { PROF_ROW_NL = 0, PROF_COL_FWD = 1, PROF_ROW_ADJ = 2, PROF_COL_ADJ = 3 };

template <class F>
hipError_t timed(pa_ctx* c, int cls, F&& launch) {
    if (c->prof_class != cls) return launch();
    const bool take = (c->prof_seen++ % c->prof_every) == 0;
    if (!take) return launch();
    if (c->prof_used + 2 > c->prof_ev.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            c->prof_ev.push_back(e);
        }
    }
    // the kernel's dispatch records the pair (see launch_kernel)
    DispatchEvents& de = dispatch_events();
    de.start = c->prof_ev[c->prof_used];
    de.stop = c->prof_ev[c->prof_used + 1];
    de.used = false;
    const hipError_t r = launch();
    const bool used = de.used;
    de = DispatchEvents();
    if (r != hipSuccess) return r;
    if (used) c->prof_used += 2;
    return hipSuccess;
}

// -------------------------------------------------------------- sweeps --

RowObs row_obs_args(const ObsRange* r, int slot, double* obs_out, double* jpart) {
    RowObs o{};
    o.slot = slot;
    if (r) {
        o.stride = r->stride;
        o.M = r->M;
        o.n_times = r->n_times;
        o.values = r->values;
    } else {
        o.stride = o.M = 1;
    }
    o.obs_out = obs_out;
    o.jpart = jpart;
    o.imp_x = o.imp_y = -1;
    return o;
}

// Per-member sizes of the buffer kinds, for launches on a slice of members.
size_t per_y(const pa_ctx* c) { return (size_t)c->d.N * c->d.KXP; }
size_t per_c(const pa_ctx* c) { return (size_t)c->d.KY * c->d.KXP; }

// Members [lo, hi) of a context's batch as a launch of their own.
Dims slice_dims(const pa_ctx* c, int lo, int hi) {
    Dims d = c->d;
    d.B = hi - lo;
    (void)lo;
    return d;
}

// Observation of range r at its slot (velocity probes and cost partials) from the
// stage-a fields (the packed pairs (u, w_x), (v, w_y)) of the state at that step.
pa_status observe_range(pa_ctx* c, WS& w, const ObsRange& r, int slot, cd* const fields[4], double* obs_out) {
    RowArgs ra{};
    for (int i = 0; i < 4; ++i) ra.yin[i] = fields[i] + (size_t)r.b0 * per_y(c);
    ra.tw = c->tw;
    ra.obs = row_obs_args(&r, slot, obs_out, w.jpart + r.jrow0);
    PA_HIP(launch_row_obs(slice_dims(c, r.b0, r.b0 + r.nb), ra, c->stream));
    return PA_OK;
}

// Every range observed at step n.
pa_status observe_step(pa_ctx* c, WS& w, const ObsPlan& op, int n, cd* const fields[4], double* obs_out) {
    for (int i = 0; i < op.n; ++i) {
        const int slot = op.r[i].slot(n);
        if (slot >= 0) PA_TRY(observe_range(c, w, op.r[i], slot, fields, obs_out));
    }
    return PA_OK;
}

// Residual source rows (-S^T r_u, -S^T r_v, row-transformed) of the members [lo, hi) of
// range r at its slot, into out[0..1] (full-batch buffers; the slice is written).
pa_status source_rows(pa_ctx* c, const ObsRange& r, int slot, int lo, int hi, cd* const fields[4],
                      cd* const out[2]) {
    const size_t off = (size_t)lo * per_y(c);
    RowArgs rs{};
    for (int i = 0; i < 4; ++i) rs.yin[i] = fields[i] + off;
    rs.yout[0] = out[0] + off;
    rs.yout[1] = out[1] + off;
    rs.tw = c->tw;
    rs.obs = row_obs_args(&r, slot, nullptr, nullptr);
    if (r.values) rs.obs.values = r.values + (size_t)(lo - r.b0) * r.n_times * 2 * r.M * r.M;
    PA_HIP(launch_row_src(slice_dims(c, lo, hi), rs, 0, c->stream));
    return PA_OK;
}

// Source rows at step n for the members [lo, hi): the observing ranges write their
// members' rows; the rest of the slice is zeroed unless the ranges cover it.  Returns
// (in *any) whether some member of the slice observes at n.
pa_status sources_at(pa_ctx* c, WS& w, const ObsPlan& op, int n, int lo, int hi, cd* const fields[4],
                     cd* const out[2], bool* any) {
    *any = false;
    int covered = 0;
    for (int i = 0; i < op.n; ++i) {
        const ObsRange& r = op.r[i];
        const int a = std::max(lo, r.b0), b = std::min(hi, r.b0 + r.nb);
        if (a < b && r.slot(n) >= 0) covered += b - a;
    }
    if (covered == 0) return PA_OK;
    *any = true;
    if (covered < hi - lo) {
        const size_t off = (size_t)lo * per_y(c), cnt = 2 * (size_t)(hi - lo) * per_y(c);
        PA_HIP(launch_fill(reinterpret_cast<double*>(out[0] + off), 0.0, cnt, c->stream));
        PA_HIP(launch_fill(reinterpret_cast<double*>(out[1] + off), 0.0, cnt, c->stream));
    }
    for (int i = 0; i < op.n; ++i) {
        const ObsRange& r = op.r[i];
        const int a = std::max(lo, r.b0), b = std::min(hi, r.b0 + r.nb);
        const int slot = r.slot(n);
        if (a < b && slot >= 0) PA_TRY(source_rows(c, r, slot, a, b, fields, out));
    }
    return PA_OK;
}

// Cost per member from the partial rows of every range (fixed order within a member).
pa_status reduce_cost(pa_ctx* c, WS& w, const ObsPlan& op) {
    for (int i = 0; i < op.n; ++i) {
        const ObsRange& r = op.r[i];
        PA_HIP(launch_reduce_j(r.nb, r.n_times * r.M, w.jpart + r.jrow0, w.J + r.b0, c->stream));
    }
    return PA_OK;
}

ColArgs col_base(const pa_ctx* c) {
    ColArgs a{};
    a.invk2 = c->invk2;
    a.ex2 = c->ex2;
    a.ey2 = c->ey2;
    a.tw = c->tw;
    a.h = c->ph.dt;
    a.forcing = c->forcing;
    a.nf = c->nf;
    return a;
}

void set_stage_fields(ColArgs& a, cd* const f[4]) {
    a.nout = 4;
    a.fields[0] = F_UP;
    a.fields[1] = F_UQ;
    a.fields[2] = F_VP;
    a.fields[3] = F_VQ;
    for (int i = 0; i < 4; ++i) a.yout[i] = f[i];
}

// Transform physical omega0 to the band-limited state (P omega0), write
// checkpoint slot 0 if given, and the stage-a fields to `fields`.
pa_status start_state(pa_ctx* c, WS& w, const double* omega0, cd* ck0, cd* const fields[4]) {
    PA_HIP(launch_row_r2c(c->d, omega0, w.Y0, c->tw, c->stream));
    ColArgs a = col_base(c);
    a.yin[0] = w.Y0;
    a.omega = w.omega;
    a.ckpt = ck0;
    set_stage_fields(a, fields);
    PA_HIP(launch_col(c->d, COL_INIT, a, c->stream));
    return PA_OK;
}

// Where run_steps writes checkpoints: boundary i (step i K, or n_total for
// the last) goes to slot map[i] of base (none if -1), or to slot i without a map.
struct CkptTarget {
    cd* base = nullptr;
    const std::vector<int>* map = nullptr;
};

// Steps n0 .. n1-1 from the state in w.omega whose stage-a fields are in
// `start` (which must equal the segment slot (0,0) when store).  With store
// the fields of every stage are kept in the segment slots; otherwise they
// live in w.Yf.  Checkpoints are written to ckpt (if it has a base) at the
// boundaries, multiples of K and the final step n_total.  With op, the
// ranges observed at a step are observed from its stage-a fields before the
// step (cost partials, model observations) when `observe`, and only the
// members [0, op->act(n)) advance through step n.
pa_status run_steps(pa_ctx* c, WS& w, int n0, int n1, int n_total, int K, bool store, const ObsPlan* op,
                    bool observe, double* obs_out, CkptTarget ckpt, bool final_fields) {
    const int nseg = n_segments(n_total, K);
    for (int n = n0; n < n1; ++n) {
        const int j = n - n0;
        Dims dn = c->d;
        if (op) dn.B = op->act(n);
        for (int s = 0; s < 4; ++s) {
            cd* fin[4];
            cd* fout[4];
            if (store) {
                seg_fields(c, w, j, s, fin);
                if (s < 3) seg_fields(c, w, j, s + 1, fout);
                else seg_fields(c, w, j + 1, 0, fout);
            } else {
                for (int i = 0; i < 4; ++i) fin[i] = fout[i] = w.Yf[i];
            }
            if (s == 0 && op && observe) PA_TRY(observe_step(c, w, *op, n, fin, obs_out));
            if (dn.B < 1) continue;
            RowArgs ra{};
            for (int i = 0; i < 4; ++i) ra.yin[i] = fin[i];
            ra.yout[0] = w.Yp[0];
            ra.tw = c->tw;
            ra.obs = row_obs_args(nullptr, -1, nullptr, nullptr);
            PA_HIP(timed(c, PROF_ROW_NL, [&] { return launch_row_nl(dn, ra, c->stream); }));
            ColArgs a = col_base(c);
            a.yin[0] = w.Yp[0];
            a.omega = w.omega;
            a.acc = w.acc;
            set_stage_fields(a, fout);
            if (s == 3) {
                const int nn = n + 1;
                if (ckpt.base && (nn % K == 0 || nn == n_total)) {
                    const int bi = nn == n_total ? nseg : nn / K;
                    const int slot = ckpt.map ? (*ckpt.map)[(size_t)bi] : bi;
                    if (slot >= 0) a.ckpt = ckpt_slot(c, ckpt.base, slot);
                }
                if (nn == n1 && !final_fields) a.nout = 0;
                // the new state goes to the other buffer, so that no workgroup of the launch
                // overwrites a state another one still reads
                a.omega_out = w.omega2;
            }
            PA_HIP(timed(c, PROF_COL_FWD, [&] { return launch_col(dn, COL_A + s, a, c->stream); }));
            if (s == 3) std::swap(w.omega, w.omega2);
        }
    }
    return PA_OK;
}

// Physical field from a compact state.
pa_status state_to_phys(pa_ctx* c, WS& w, const cd* state, double* out) {
    ColArgs a = col_base(c);
    a.state_in = state;
    a.nout = 1;
    a.fields[0] = F_OMEGA;
    a.yout[0] = w.Y0;
    PA_HIP(launch_col(c->d, COL_FROM_STATE, a, c->stream));
    PA_HIP(launch_row_c2r(c->d, w.Y0, out, c->tw, c->stream));
    return PA_OK;
}

// Forward sweep with checkpoints into `ckpt` and J into w.J (if values).
// With store_last (and a segment buffer), the last checkpoint segment runs in
// store mode: its stage fields go straight to the segment slots, so a
// backward sweep that follows (last_ready) starts that segment without
// recomputing it.  With ckpt_every >= n_steps the whole trajectory is kept
// and the gradient needs no recomputation at all.  The stage fields are the
// same either way (same kernels, only their output addresses differ).  With
// a schedule (plan_for) the checkpoints are those of its first chain, in its
// slots, and the last segment is always stored.
pa_status forward_sweep(pa_ctx* c, WS& w, const double* omega0, int n_steps, const ObsPlan& op,
                        double* obs_out, cd* ckpt, int K, bool store_last,
                        const std::vector<PlanAct>* plan = nullptr) {
    if (plan && !(store_last && w.seg && n_steps > 0)) return fail(PA_EINVAL, "schedule needs the segment store");
    const CkptTarget tgt{ckpt, plan ? &c->plan_fwd_slot : nullptr};
    const bool store = store_last && w.seg && n_steps > 0;
    const int n_last = store ? (n_segments(n_steps, K) - 1) * K : n_steps;   // first step of the stored segment
    bool final_obs = false;
    for (int i = 0; i < op.n; ++i) final_obs = final_obs || op.r[i].slot(n_steps) >= 0;
    cd* f0[4] = {w.Yf[0], w.Yf[1], w.Yf[2], w.Yf[3]};
    if (store && n_last == 0) seg_fields(c, w, 0, 0, f0);
    PA_TRY(start_state(c, w, omega0, ckpt ? ckpt_slot(c, ckpt, 0) : nullptr, f0));
    // Sobolev term (lambda/2) int |grad u0|^2 = (lambda/2) int omega0^2 (periodic, divergence-free),
    // exact on the grid for the band-limited P omega0: 4 pi^2 lambda * (1/2) sum |omega_hat|^2 / N^4
    const bool reg = c->sobolev > 0.0 && op.values && op.n > 0;
    if (reg) PA_HIP(launch_state_energy(c->d, w.omega, 4.0 * M_PI * M_PI * c->sobolev, w.J2, c->stream));
    if (n_last > 0) {
        PA_TRY(run_steps(c, w, 0, n_last, n_steps, K, false, &op, true, obs_out, tgt, !store && final_obs));
        if (store) {
            // stage-a fields of the state at n_last (in w.omega) into segment slot (0, 0), for
            // every member: a member whose horizon is n_last is observed from them
            cd* s0[4];
            seg_fields(c, w, 0, 0, s0);
            ColArgs a = col_base(c);
            a.state_in = w.omega;
            set_stage_fields(a, s0);
            PA_HIP(launch_col(c->d, COL_FROM_STATE, a, c->stream));
        }
    }
    cd* fH[4] = {w.Yf[0], w.Yf[1], w.Yf[2], w.Yf[3]};
    if (store) {
        PA_TRY(run_steps(c, w, n_last, n_steps, n_steps, K, true, &op, true, obs_out, tgt, true));
        seg_fields(c, w, n_steps - n_last, 0, fH);
    }
    if (final_obs) PA_TRY(observe_step(c, w, op, n_steps, fH, obs_out));
    if (op.values && op.n > 0) PA_TRY(reduce_cost(c, w, op));
    if (reg) PA_HIP(launch_axpy(c->d.B, 1, nullptr, 1.0, w.J2, w.J, nullptr, c->stream));
    return PA_OK;
}

// Adjoint stage of step n: row products + column transposes for stage
// `mode`, for the members [0, op->act(n)) (all members without op).  At
// stage n of a step that members observe, their residual source rows are
// formed from the same stage fields and enter the column pass as two extra
// inputs (zero for the other members of the launch).
pa_status adj_stage(pa_ctx* c, WS& w, cd* const fields[4], int mode, const ObsPlan* op, int n, int final_out,
                    const double* scale) {
    Dims dn = c->d;
    if (op) dn.B = op->act(n);
    RowArgs ra{};
    for (int i = 0; i < 4; ++i) ra.yin[i] = fields[i];
    ra.yin[4] = w.YL[0];
    ra.yin[5] = w.YL[1];
    ra.yout[0] = w.Yp[0];
    ra.yout[1] = w.Yp[1];
    ra.tw = c->tw;
    ra.obs = row_obs_args(nullptr, -1, nullptr, nullptr);
    PA_HIP(timed(c, PROF_ROW_ADJ, [&] { return launch_row_adj(dn, ra, c->stream); }));
    ColArgs a = col_base(c);
    a.yin[0] = w.Yp[0];
    a.yin[1] = w.Yp[1];
    a.nin = 2;
    a.inmul[0] = IN_PAIRP;
    a.inmul[1] = IN_PAIRQ;
    if (mode == COL_ADJ_N && op && op->values) {
        bool any = false;
        cd* const out[2] = {w.Yp[2], w.Yp[3]};
        PA_TRY(sources_at(c, w, *op, n, 0, dn.B, fields, out, &any));
        if (any) {
            a.yin[2] = w.Yp[2];
            a.yin[3] = w.Yp[3];
            a.nin = 4;
            a.inmul[2] = IN_IKY_INVK2;
            a.inmul[3] = IN_MIKX_INVK2;
        }
    }
    a.lam = w.lam;
    a.omb = w.omb;
    a.final_out = final_out;
    a.scale = scale;
    a.yout[0] = w.YL[0];
    a.fields[0] = F_OMEGA;
    if (final_out) {
        a.nout = 1;
    } else {
        a.nout = 2;
        a.fields[0] = F_LP;
        a.yout[1] = w.YL[1];
        a.fields[1] = F_LQ;
    }
    const int cmode = (mode == COL_ADJ_N && a.nin > 2) ? COL_ADJ_NSRC : mode;
    PA_HIP(timed(c, PROF_COL_ADJ, [&] { return launch_col(dn, cmode, a, c->stream); }));
    return PA_OK;
}

struct Shells {
    double* out = nullptr;
    int n = 0;
    size_t stride = 0;
    pa_ensemble_acc* acc = nullptr;   // ensemble sums to add each row to
};

pa_status record_shells(pa_ctx* c, WS& w, const Shells& sh, int row) {
    if (!sh.out) return PA_OK;
    PA_HIP(launch_shells(c->d, w.lam, c->shell_start, c->shell_modes, sh.n, sh.out + (size_t)row * sh.n,
                         sh.stride, c->stream));
    if (sh.acc) {
        const size_t SC = (size_t)c->d.KY * c->d.KXP;
        PA_HIP(launch_ens_accumulate(c->d, w.lam, static_cast<cd*>(sh.acc->lambda_sum) + (size_t)row * SC,
                                     sh.out + (size_t)row * sh.n, sh.stride, sh.n,
                                     sh.acc->shell_sum + (size_t)row * sh.n, w.dots, sh.acc->energy_sum + row,
                                     c->stream));
    }
    return PA_OK;
}

// Terminal adjoint state of the members [lo, hi) at step `step` (their last
// step, or the first one at which they take part in the backward sweep):
// lambda = the residual sources of the members observed there, or a unit
// u-impulse at (ix, iy) (impulse), else zero.  Writes lambda and the Lambda
// fields of the slice (with final_out the gradient field, times scale).
pa_status terminal(pa_ctx* c, WS& w, const ObsPlan* op, int step, cd* const fields[4], int impulse, int ix,
                   int iy, bool final_out, const double* scale, int lo, int hi) {
    const size_t offY = (size_t)lo * per_y(c), offC = (size_t)lo * per_c(c);
    const size_t nY = (size_t)(hi - lo) * per_y(c), nC = (size_t)(hi - lo) * per_c(c);
    const Dims ds = slice_dims(c, lo, hi);
    cd* const src[2] = {w.Yp[0], w.Yp[1]};
    bool any = false;
    if (impulse) {
        RowArgs ra{};
        ra.yout[0] = src[0] + offY;
        ra.yout[1] = src[1] + offY;
        ra.tw = c->tw;
        ra.obs = row_obs_args(nullptr, -1, nullptr, nullptr);
        ra.obs.imp_x = ix;
        ra.obs.imp_y = iy;
        PA_HIP(launch_row_src(ds, ra, 1, c->stream));
        any = true;
    } else if (op && op->values) {
        PA_TRY(sources_at(c, w, *op, step, lo, hi, fields, src, &any));
    }
    if (!any) {
        PA_HIP(launch_fill(reinterpret_cast<double*>(w.lam + offC), 0.0, 2 * nC, c->stream));
        PA_HIP(launch_fill(reinterpret_cast<double*>(w.YL[0] + offY), 0.0, 2 * nY, c->stream));
        PA_HIP(launch_fill(reinterpret_cast<double*>(w.YL[1] + offY), 0.0, 2 * nY, c->stream));
        return PA_OK;
    }
    ColArgs a = col_base(c);
    a.yin[0] = src[0] + offY;
    a.yin[1] = src[1] + offY;
    a.nin = 2;
    a.inmul[0] = IN_IKY_INVK2;
    a.inmul[1] = IN_MIKX_INVK2;
    a.lam = w.lam + offC;
    a.final_out = final_out ? 1 : 0;
    a.scale = scale ? scale + lo : nullptr;
    a.yout[0] = w.YL[0] + offY;
    a.fields[0] = F_OMEGA;
    if (final_out) {
        a.nout = 1;
    } else {
        a.nout = 2;
        a.fields[0] = F_LP;
        a.yout[1] = w.YL[1] + offY;
        a.fields[1] = F_LQ;
    }
    PA_HIP(launch_col(ds, COL_ADJ_SRC, a, c->stream));
    return PA_OK;
}

// Gradient of the Sobolev term, lambda (2 pi / N)^2 P omega0 (times the
// member's scale), added to grad_out; P omega0 is checkpoint 0.  Cost
// gradients only (observations given, not the impulse response).
pa_status add_sobolev_gradient(pa_ctx* c, WS& w, const cd* ckpt, const ObsPlan* op, int impulse,
                               const double* scale, double* grad_out) {
    if (!(c->sobolev > 0.0) || impulse || !op || !op->values || op->n == 0) return PA_OK;
    const size_t n = (size_t)c->d.N * c->d.N;
    PA_TRY(state_to_phys(c, w, ckpt_slot(c, const_cast<cd*>(ckpt), 0), w.P0));
    const double coef = c->sobolev * 4.0 * M_PI * M_PI / (double)n;
    PA_HIP(launch_axpy(c->d.B, n, scale, coef, w.P0, grad_out, nullptr, c->stream));
    return PA_OK;
}

// Backward sweep from checkpoints: recompute each segment storing every
// stage's fields, then run the adjoint steps of the segment in reverse.  With
// last_ready the last segment's fields are already in the segment slots (a
// forward sweep with store_last just ran in this workspace).  The final
// field (P lambda_0 times scale) is written to grad_out (physical).  With a
// schedule (plan_for; needs last_ready) the segments are reversed in its
// order, re-advancing from its snapshot slots in ckpt.
pa_status backward_sweep(pa_ctx* c, WS& w, const cd* ckpt, int n_steps, int K, const ObsPlan* op, int impulse,
                         int ix, int iy, const double* scale, double* grad_out, const Shells& sh,
                         bool last_ready, const std::vector<PlanAct>* plan = nullptr) {
    const int nseg = n_segments(n_steps, K);
    const int B = c->d.B;
    auto act = [&](int n) { return op ? op->act(n) : B; };
    cd* const ck = const_cast<cd*>(ckpt);
    // members that take part in no step (their only observation is at step 0) start and
    // end at step 0: the gradient field straight from their sources, from the state in slot 0
    auto finish_idle = [&](int lo) -> pa_status {
        if (lo >= B) return PA_OK;
        cd* f0[4] = {w.Yf[0], w.Yf[1], w.Yf[2], w.Yf[3]};
        const size_t offY = (size_t)lo * per_y(c);
        ColArgs a = col_base(c);
        a.state_in = ckpt_slot(c, ck, 0) + (size_t)lo * per_c(c);
        a.nout = 4;
        a.fields[0] = F_UP;
        a.fields[1] = F_UQ;
        a.fields[2] = F_VP;
        a.fields[3] = F_VQ;
        for (int i = 0; i < 4; ++i) a.yout[i] = f0[i] + offY;
        PA_HIP(launch_col(slice_dims(c, lo, B), COL_FROM_STATE, a, c->stream));
        return terminal(c, w, op, 0, f0, impulse, ix, iy, true, scale, lo, B);
    };
    if (n_steps == 0) {
        bool obs0 = impulse != 0;
        for (int i = 0; op && op->values && i < op->n; ++i) obs0 = obs0 || op->r[i].slot(0) >= 0;
        if (!obs0) {
            if (grad_out) PA_HIP(launch_fill(grad_out, 0.0, (size_t)B * c->d.N * c->d.N, c->stream));
            if (grad_out) PA_TRY(add_sobolev_gradient(c, w, ckpt, op, impulse, scale, grad_out));
            return PA_OK;
        }
        PA_TRY(finish_idle(0));
        PA_TRY(record_shells(c, w, sh, 0));
        if (grad_out) PA_HIP(launch_row_c2r(c->d, w.YL[0], grad_out, c->tw, c->stream));
        if (grad_out) PA_TRY(add_sobolev_gradient(c, w, ckpt, op, impulse, scale, grad_out));
        return PA_OK;
    }
    if (!w.seg) return fail(PA_EINVAL, "workspace carved without a segment buffer");
    if (plan && !last_ready) return fail(PA_EINVAL, "a schedule's backward sweep follows its forward sweep");
    // Recompute segment `seg` keeping its stage fields (from state src; src ==
    // w.omega is the live state), unless its fields are already stored, then
    // run the adjoint steps through it.  Members join the sweep at the step
    // after their last: their terminal state is formed there, from the stage-a
    // fields of their final state.
    auto reverse_segment = [&](int seg, const cd* src, bool recompute) -> pa_status {
        const int n0 = seg * K, n1 = std::min(n_steps, n0 + K), L = n1 - n0;
        const bool last = seg == nseg - 1;
        if (recompute) {
            cd* f0[4];
            seg_fields(c, w, 0, 0, f0);
            ColArgs a = col_base(c);
            a.state_in = src;
            a.omega = src == w.omega ? nullptr : w.omega;
            set_stage_fields(a, f0);
            PA_HIP(launch_col(slice_dims(c, 0, act(n0)), COL_FROM_STATE, a, c->stream));
            // the fields of the segment's end state are needed when members join at its last step
            const bool joins = !last && act(n1 - 1) > act(n1);
            PA_TRY(run_steps(c, w, n0, n1, n_steps, K, true, op, false, nullptr, CkptTarget(), last || joins));
        }
        for (int j = L - 1; j >= 0; --j) {
            const int n = n0 + j;
            const int hi = act(n), lo = (n + 1 >= n_steps) ? 0 : act(n + 1);
            if (hi > lo) {
                cd* fm[4];
                seg_fields(c, w, j + 1, 0, fm);
                PA_TRY(terminal(c, w, op, n + 1, fm, impulse, ix, iy, false, scale, lo, hi));
                if (n + 1 == n_steps) PA_TRY(record_shells(c, w, sh, 0));
            }
            cd* fs[4];
            seg_fields(c, w, j, 3, fs);
            PA_TRY(adj_stage(c, w, fs, COL_ADJ_C, op, n, 0, nullptr));
            seg_fields(c, w, j, 2, fs);
            PA_TRY(adj_stage(c, w, fs, COL_ADJ_B, op, n, 0, nullptr));
            seg_fields(c, w, j, 1, fs);
            PA_TRY(adj_stage(c, w, fs, COL_ADJ_A, op, n, 0, nullptr));
            seg_fields(c, w, j, 0, fs);
            PA_TRY(adj_stage(c, w, fs, COL_ADJ_N, impulse ? nullptr : op, n, n == 0 ? 1 : 0, scale));
            PA_TRY(record_shells(c, w, sh, n_steps - n));
        }
        return PA_OK;
    };
    if (!plan) {
        for (int seg = nseg - 1; seg >= 0; --seg)
            PA_TRY(reverse_segment(seg, ckpt_slot(c, ck, seg), !(seg == nseg - 1 && last_ready)));
    } else {
        // the forward sweep ran the schedule up to its first REVERSE (segment nseg-1, stored)
        size_t i = 0;
        while (i < plan->size() && (*plan)[i].kind != ACT_REVERSE) ++i;
        if (i == plan->size() || (*plan)[i].a != nseg - 1) return fail(PA_EINVAL, "internal: malformed checkpoint schedule");
        PA_TRY(reverse_segment(nseg - 1, nullptr, false));
        std::vector<int> end_slot((size_t)nseg + 1, -1);
        for (++i; i < plan->size(); ++i) {
            const PlanAct& act_ = (*plan)[i];
            const cd* src = act_.src >= 0 ? ckpt_slot(c, ck, act_.src) : w.omega;
            if (act_.kind == ACT_REVERSE) {
                PA_TRY(reverse_segment(act_.a, src, true));
                continue;
            }
            // advance: the stage-a fields of the start state into w.Yf (a live start has them there)
            cd* f0[4] = {w.Yf[0], w.Yf[1], w.Yf[2], w.Yf[3]};
            if (act_.src >= 0) {
                ColArgs a = col_base(c);
                a.state_in = src;
                a.omega = w.omega;
                set_stage_fields(a, f0);
                PA_HIP(launch_col(c->d, COL_FROM_STATE, a, c->stream));
            }
            if (act_.dst >= 0) end_slot[(size_t)act_.b] = act_.dst;
            PA_TRY(run_steps(c, w, act_.a * K, std::min(n_steps, act_.b * K), n_steps, K, false, nullptr, false,
                             nullptr, CkptTarget{ck, &end_slot}, true));
            end_slot[(size_t)act_.b] = -1;
        }
    }
    PA_TRY(finish_idle(act(0)));
    if (grad_out) PA_HIP(launch_row_c2r(c->d, w.YL[0], grad_out, c->tw, c->stream));
    if (grad_out) PA_TRY(add_sobolev_gradient(c, w, ckpt, op, impulse, scale, grad_out));
    return PA_OK;
}

// precondition with the multiplier table mult (computed before): one table
// for every member, or with per_member one table per member ([B][KY][KXP])
pa_status apply_filter(pa_ctx* c, WS& w, const double* mult, const double* in, double* out,
                       bool per_member = false) {
    PA_HIP(launch_row_r2c(c->d, in, w.Y0, c->tw, c->stream));
    ColArgs a = col_base(c);
    a.yin[0] = w.Y0;
    a.mult = mult;
    a.mult_per_member = per_member ? 1 : 0;
    a.nout = 1;
    a.fields[0] = F_OMEGA;
    a.yout[0] = w.Yf[0];
    PA_HIP(launch_col(c->d, COL_FILTER, a, c->stream));
    PA_HIP(launch_row_c2r(c->d, w.Yf[0], out, c->tw, c->stream));
    return PA_OK;
}

pa_status valid_kernel(const pa_kernel* k) {
    if (!k) return fail(PA_EINVAL, "kernel is NULL");
    if (k->kind < 0 || k->kind > 3) return fail(PA_EINVAL, "kernel kind must be 0..3");
    if (k->metric < 0 || k->metric > 2) return fail(PA_EINVAL, "kernel metric must be 0, 1 or 2");
    if (!std::isfinite(k->param)) return fail(PA_EINVAL, "kernel parameter must be finite");
    return PA_OK;
}

// The multiplier (m^2 W)^power must be finite on the whole band of the
// context's grid.  It is evaluated here with the operations of
// make_mult_kernel (W, then m^2 W, then the power), before anything is
// enqueued: a kernel whose W underflows to zero where it is inverted, or whose
// power leaves the double range, has no finite latent map on this grid and is
// refused rather than turned into infinite fields.  The multiplier depends on
// kx^2 + ky^2 only, so 0 <= kx <= ky <= Kc covers the band.  Tables found
// finite are remembered per context.
pa_status check_multiplier(pa_ctx* c, const pa_kernel* k, double power) {
    const std::array<double, 4> key{(double)k->kind, (double)k->metric, k->param, power};
    for (const auto& q : c->mult_checked)
        if (q == key) return PA_OK;
    const int K = c->d.K;
    for (int ky = 1; ky <= K; ++ky) {
        for (int kx = 0; kx <= ky; ++kx) {
            const double k2 = (double)kx * kx + (double)ky * ky;
            const double kap = std::sqrt(k2);
            double W = 1.0;
            if (k->kind == 1) W = std::exp(-k->param * kap);
            else if (k->kind == 2) W = std::pow(kap, -2.0 * k->param);
            else if (k->kind == 3) W = std::exp(-k->param * k2);
            const double base = (k->metric == 0 ? k2 : k->metric == 2 ? k2 * k2 : 1.0) * W;
            const double v = std::pow(base, power);
            if (!std::isfinite(v)) {
                char msg[256];
                std::snprintf(msg, sizeof msg,
                              "kernel (kind %d, metric %d, param %.17g) to the power %.17g is not finite at "
                              "|k| = %.6g of the %d^2 grid's band: no finite preconditioner there",
                              k->kind, k->metric, k->param, power, kap, c->d.N);
                return fail(PA_EINVAL, msg);
            }
        }
    }
    c->mult_checked.push_back(key);
    return PA_OK;
}

// host twiddle exp(-2 pi i m/N) from the first octant with exact symmetries
void host_twiddles(int N, std::vector<cd>& tw) {
    tw.resize(N);
    const long double pi2 = 1.57079632679489661923132169163975144L;   // pi / 2
    for (int m = 0; m < N; ++m) {
        const long q = (4L * m) / N, r = (4L * m) % N;     // angle = (pi/2)(q + r/N)
        const bool flip = 2 * r > N;
        const long rr = flip ? N - r : r;
        const long double ang = pi2 * (long double)rr / (long double)N;
        long double cphi = cosl(ang), sphi = sinl(ang);
        if (flip) std::swap(cphi, sphi);
        long double cs, sn;
        switch (q & 3) {
            case 0: cs = cphi; sn = sphi; break;
            case 1: cs = -sphi; sn = cphi; break;
            case 2: cs = -cphi; sn = -sphi; break;
            default: cs = sphi; sn = -cphi; break;
        }
        tw[m].x = (double)cs;
        tw[m].y = -(double)sn;
    }
}

}  // namespace

// ------------------------------------------------ allocation-free calls --
// Scratch of pa_adjoint_gradient_noalloc: a file-scope device array, one copy
// on every device the library runs on, held until the process ends.  In host
// code `scratch` is only a stand-in for the symbol, not a device address: the
// address of each device's copy is looked up once, with that device current,
// when the first context is created on it (bind_scratch), and only that
// address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[PA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 256;
std::once_flag g_scratch_once[SCRATCH_DEVICES];
void* g_scratch_ptr[SCRATCH_DEVICES];
hipError_t g_scratch_err[SCRATCH_DEVICES];

// Device address of the current device `dev`'s copy of scratch (once per device).
void bind_scratch(int dev) {
    if (dev < 0 || dev >= SCRATCH_DEVICES) return;
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        g_scratch_err[dev] = e;
        g_scratch_ptr[dev] = p;
    });
}

}  // namespace

// ================================================================= ABI ==

extern "C" {

const char* pa_last_error(void) { return g_err.c_str(); }

pa_status pa_create(const pa_physics* phys, int32_t N, int32_t B, void* hip_stream, pa_ctx** out) try {
    g_err.clear();
    if (!out) return fail(PA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!phys) return fail(PA_EINVAL, "physics is NULL");
    if (!is_pow2(N) || N < 8 || N > 1024) return fail(PA_EINVAL, "N must be a power of two in [8, 1024]");
    // members run along the second grid dimension of the column and batched kernels
    if (B < 1 || B > PA_MAX_MEMBERS) return fail(PA_EINVAL, "B must be in [1, 65535]");
    if (!finite_nonneg(phys->nu) || !finite_nonneg(phys->mu)) return fail(PA_EINVAL, "nu, mu must be finite, >= 0");
    if (!std::isfinite(phys->dt) || phys->dt <= 0) return fail(PA_EINVAL, "dt must be finite and > 0");
    if (!std::isfinite(phys->forcing_amp)) return fail(PA_EINVAL, "forcing amplitude must be finite");
    if (phys->forcing_amp != 0.0 && (phys->forcing_k < 1 || phys->forcing_k >= N / 2))
        return fail(PA_EINVAL, "forcing wavenumber must be in [1, N/2)");
    if (phys->reserved != 0) return fail(PA_EINVAL, "reserved must be 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PA_EDEVICE, "no HIP device");

    int dev = 0;
    PA_HIP(hipGetDevice(&dev));
    bind_scratch(dev);   // the allocation-free calls' scratch on this device
    // owned until it is handed out: every early return (or a failed host
    // allocation below) frees it and whatever device tables it already holds
    std::unique_ptr<pa_ctx, pa_status (*)(pa_ctx*)> owner(new pa_ctx(), pa_destroy);
    pa_ctx* c = owner.get();
    c->ph = *phys;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->device = dev;
    Dims& d = c->d;
    d.N = N;
    d.B = B;
    d.K = (N - 1) / 3;
    d.KX = d.K + 1;
    d.KXP = (d.KX + 7) / 8 * 8;
    d.KY = 2 * d.K + 1;
    d.cus = 0;
    if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || d.cus < 1)
        d.cus = 1;
    d.lds_max = 0;
    if (hipDeviceGetAttribute(&d.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        d.lds_max < 65536)
        d.lds_max = 65536;
    d.var = 0;
    d.tpb = 4;
    d.avar = 0;
    d.atpb = 4;
    d.cvar = 0;
    d.cb = 8;
    d.csplit = 0;
    while (d.cb > 1 && (d.cb * fft_threads(N, d.cvar) > 512 ||
                        ((size_t)d.cb * (N + N / 16 + 1) + N) * sizeof(cd) > 65536)) d.cb >>= 1;

    std::vector<cd> tw;
    host_twiddles(N, tw);
    std::vector<double> invk2((size_t)d.KY * d.KXP, 0.0), ex2(d.KXP, 0.0), ey2(d.KY, 0.0);
    const double h2 = 0.5 * phys->dt;
    for (int r = 0; r < d.KY; ++r) {
        const int ky = (r <= d.K) ? r : r - d.KY;
        ey2[r] = std::exp(-phys->nu * h2 * (double)ky * ky);
        for (int kx = 0; kx <= d.K; ++kx) {
            const double k2 = (double)kx * kx + (double)ky * ky;
            if (k2 > 0) invk2[(size_t)r * d.KXP + kx] = 1.0 / k2;
        }
    }
    for (int kx = 0; kx < d.KXP; ++kx) ex2[kx] = std::exp(-(phys->nu * (double)kx * kx + phys->mu) * h2);
    // shells: compact indices grouped by floor(|k|), k = 1..floor(sqrt(2) K)
    const int smax = (int)std::floor(std::sqrt(2.0) * d.K);
    std::vector<std::vector<int>> lists(smax + 1);
    for (int r = 0; r < d.KY; ++r) {
        const int ky = (r <= d.K) ? r : r - d.KY;
        for (int kx = 0; kx <= d.K; ++kx) {
            const long m2 = (long)kx * kx + (long)ky * ky;
            long s = (long)std::sqrt((double)m2);
            while (s * s > m2) --s;
            while ((s + 1) * (s + 1) <= m2) ++s;
            if (s >= 1 && s <= smax) lists[s].push_back(r * d.KXP + kx);
        }
    }
    std::vector<int> start(smax + 1, 0), modes;
    for (int k = 1; k <= smax; ++k) {
        start[k - 1] = (int)modes.size();
        modes.insert(modes.end(), lists[k].begin(), lists[k].end());
    }
    start[smax] = (int)modes.size();
    c->n_shell_max = smax;
    c->nf = (phys->forcing_amp != 0.0 && phys->forcing_k <= d.K) ? phys->forcing_k : 0;
    c->forcing = -phys->forcing_amp * phys->forcing_k * 0.5 * (double)N * (double)N;

    if (hipMalloc(&c->tw, sizeof(cd) * N) != hipSuccess) return fail(PA_ENOMEM, "hipMalloc tables");
    if (hipMalloc(&c->invk2, sizeof(double) * invk2.size()) != hipSuccess) return fail(PA_ENOMEM, "hipMalloc tables");
    if (hipMalloc(&c->ex2, sizeof(double) * ex2.size()) != hipSuccess) return fail(PA_ENOMEM, "hipMalloc tables");
    if (hipMalloc(&c->ey2, sizeof(double) * ey2.size()) != hipSuccess) return fail(PA_ENOMEM, "hipMalloc tables");
    if (hipMalloc(&c->shell_start, sizeof(int) * start.size()) != hipSuccess) return fail(PA_ENOMEM, "hipMalloc tables");
    if (hipMalloc(&c->shell_modes, sizeof(int) * std::max<size_t>(modes.size(), 1)) != hipSuccess)
        return fail(PA_ENOMEM, "hipMalloc tables");
    bool ok = hipMemcpy(c->tw, tw.data(), sizeof(cd) * N, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->invk2, invk2.data(), sizeof(double) * invk2.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->ex2, ex2.data(), sizeof(double) * ex2.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->ey2, ey2.data(), sizeof(double) * ey2.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->shell_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice) == hipSuccess &&
              (modes.empty() || hipMemcpy(c->shell_modes, modes.data(), sizeof(int) * modes.size(),
                                          hipMemcpyHostToDevice) == hipSuccess);
    if (!ok) return fail(PA_EDEVICE, "copying constant tables failed");
    *out = owner.release();
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_destroy(pa_ctx* c) try {
    if (!c) return PA_OK;
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    if (c->pin) (void)hipHostFree(c->pin);
    (void)hipFree(c->tw);
    (void)hipFree(c->invk2);
    (void)hipFree(c->ex2);
    (void)hipFree(c->ey2);
    (void)hipFree(c->shell_start);
    (void)hipFree(c->shell_modes);
    delete c;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_set_stream(pa_ctx* c, void* s) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    c->stream = reinterpret_cast<hipStream_t>(s);
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_get_shape(const pa_ctx* c, int32_t* N, int32_t* B, int32_t* Kc) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    if (N) *N = c->d.N;
    if (B) *B = c->d.B;
    if (Kc) *Kc = c->d.K;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_set_tiles(pa_ctx* c, const pa_tiles* t) try {
    if (!c || !t) return fail(PA_EINVAL, "NULL argument");
    auto variant_ok = [](int v) { return v < 0 || v <= 2; };
    auto row_variant_ok = [](int v) { return v < 0 || v <= 3; };
    auto block_ok = [](int b) { return b < 0 || b == 1 || b == 2 || b == 4 || b == 8; };
    if (!row_variant_ok(t->row_variant) || !row_variant_ok(t->adj_variant) || !variant_ok(t->col_variant))
        return fail(PA_EINVAL, "row FFT variants must be 0..3, column variants 0..2 (negative keeps)");
    if (!block_ok(t->row_teams) || !block_ok(t->adj_teams) || !block_ok(t->col_block))
        return fail(PA_EINVAL, "row teams and col_block must be 1, 2, 4 or 8 (negative keeps)");
    if (!(t->col_split < 0 || t->col_split == 0 || t->col_split == 1 || t->col_split == 2 || t->col_split == 4))
        return fail(PA_EINVAL, "col_split must be 0 (automatic), 1, 2 or 4 (negative keeps)");
    Dims d = c->d;
    if (t->row_variant >= 0) d.var = t->row_variant;
    if (t->row_teams > 0) d.tpb = t->row_teams;
    if (t->adj_variant >= 0) d.avar = t->adj_variant;
    if (t->adj_teams > 0) d.atpb = t->adj_teams;
    if (t->col_variant >= 0) d.cvar = t->col_variant;
    if (t->col_split >= 0) d.csplit = t->col_split;
    const int T = fft_threads(d.N, d.cvar);
    auto col_fits = [&](int cb) {
        return cb * T <= 512 && ((size_t)cb * (d.N + d.N / 16 + 1) + d.N) * sizeof(cd) <= (size_t)d.lds_max;
    };
    if (t->col_block > 0) {
        if (!col_fits(t->col_block)) return fail(PA_EINVAL, "col_block too large for this N and column FFT variant");
        d.cb = t->col_block;
    } else {
        while (d.cb > 1 && !col_fits(d.cb)) d.cb >>= 1;
    }
    c->d = d;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_set_sobolev(pa_ctx* c, double lambda) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    if (!std::isfinite(lambda) || lambda < 0.0) return fail(PA_EINVAL, "lambda must be finite and >= 0");
    c->sobolev = lambda;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_set_cancel_flags(pa_ctx* c, const int32_t* flags) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    c->cancel = flags;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_set_checkpoint_slots(pa_ctx* c, int32_t slots) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    if (slots < 0) return fail(PA_EINVAL, "slots must be >= 0");
    c->ckpt_slots = slots;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_get_checkpoint_slots(const pa_ctx* c, int32_t* slots) try {
    if (!c || !slots) return fail(PA_EINVAL, "NULL argument");
    *slots = c->ckpt_slots;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_checkpoint_advances(int32_t n_segments, int32_t slots, int64_t* advances) try {
    if (!advances) return fail(PA_EINVAL, "NULL argument");
    if (n_segments < 1 || slots < 1) return fail(PA_EINVAL, "need n_segments >= 1 and slots >= 1");
    *advances = min_segment_advances(n_segments, slots - 1);
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_checkpoint_schedule(int32_t n_segments, int32_t slots, int32_t* actions, int64_t capacity,
                                 int64_t* n_actions) try {
    if (!n_actions) return fail(PA_EINVAL, "n_actions is NULL");
    if (n_segments < 1 || slots < 1) return fail(PA_EINVAL, "need n_segments >= 1 and slots >= 1");
    if (n_segments > PA_MAX_SCHEDULE_SEGMENTS)
        return fail(PA_EINVAL, "n_segments exceeds PA_MAX_SCHEDULE_SEGMENTS");
    std::vector<PlanAct> plan;
    build_plan(n_segments, std::min(slots, n_segments), plan);
    *n_actions = (int64_t)plan.size();
    if (!actions) return PA_OK;
    if (capacity < (int64_t)plan.size()) return fail(PA_EINVAL, "actions buffer too small");
    for (size_t i = 0; i < plan.size(); ++i) {
        const PlanAct& a = plan[i];
        int32_t* o = actions + 5 * i;
        o[0] = a.kind;
        o[1] = a.a;
        o[2] = a.b;
        o[3] = a.src;
        o[4] = a.dst;
    }
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_is_device_memory(const void* ptr, int32_t* is_device) try {
    if (!is_device) return fail(PA_EINVAL, "NULL argument");
    const pa_status st = require_device(nullptr, {{ptr, "pointer"}});
    *is_device = (ptr && st == PA_OK) ? 1 : 0;
    g_err.clear();
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_get_tiles(const pa_ctx* c, pa_tiles* t) try {
    if (!c || !t) return fail(PA_EINVAL, "NULL argument");
    t->row_variant = c->d.var;
    t->row_teams = c->d.tpb;
    t->adj_variant = c->d.avar;
    t->adj_teams = c->d.atpb;
    t->col_variant = c->d.cvar;
    t->col_block = c->d.cb;
    t->col_split = c->d.csplit;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_profile_start(pa_ctx* c, int32_t kernel_class, int32_t sample_every) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    if (kernel_class < 0 || kernel_class > 3) return fail(PA_EINVAL, "kernel_class must be 0..3");
    if (sample_every < 1) return fail(PA_EINVAL, "sample_every must be >= 1");
    c->prof_class = kernel_class;
    c->prof_every = sample_every;
    c->prof_seen = 0;
    c->prof_used = 0;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_profile_stop(pa_ctx* c, int64_t* timed_launches, int64_t* seen_launches, double* total_ms) try {
    if (!c) return fail(PA_EINVAL, "ctx is NULL");
    PA_HIP(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->prof_used; i += 2) {
        float ms = 0.f;
        PA_HIP(hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]));
        tot += ms;
    }
    if (timed_launches) *timed_launches = (int64_t)(c->prof_used / 2);
    if (seen_launches) *seen_launches = c->prof_seen;
    if (total_ms) *total_ms = tot;
    c->prof_class = -1;
    c->prof_used = 0;
    c->prof_seen = 0;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_workspace_bytes(const pa_ctx* c, int32_t n_steps, int32_t ckpt_every, int32_t n_obs_times,
                             int32_t lbfgs_m, size_t* bytes) try {
    if (!c || !bytes) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || ckpt_every < 1 || n_obs_times < 0 || lbfgs_m < 0) return fail(PA_EINVAL, "bad sizes");
    *bytes = carve(c, n_steps, ckpt_every, n_obs_times, lbfgs_m, nullptr).total;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_checkpoint_bytes(const pa_ctx* c, int32_t n_steps, int32_t ckpt_every, size_t* bytes) try {
    if (!c || !bytes) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    *bytes = ckpt_bytes(c, n_steps, ckpt_every);
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_init_field(pa_ctx* c, const uint64_t* seeds, int32_t kind, double k0, double target,
                        double* omega_out, void* workspace, size_t wbytes) try {
    g_err.clear();
    if (!c || !seeds || !omega_out) return fail(PA_EINVAL, "NULL argument");
    if (kind < 0 || kind > 2) return fail(PA_EINVAL, "kind must be 0, 1 or 2");
    if (!(std::isfinite(target) && target > 0)) return fail(PA_EINVAL, "target must be > 0");
    if (kind != 2 && !(std::isfinite(k0) && k0 > 0)) return fail(PA_EINVAL, "k0 must be > 0");
    PA_TRY(require_device(c->stream, {{omega_out, "omega_out"}, {workspace, "workspace"}}));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, 0, 1, 0, 0, &w));
    PA_HIP(hipMemcpyAsync(w.seeds, seeds, sizeof(uint64_t) * c->d.B, hipMemcpyHostToDevice, c->stream));
    PA_HIP(hipStreamSynchronize(c->stream));   // seeds is pageable host memory owned by the caller
    PA_HIP(launch_init_spectrum(c->d, w.seeds, kind, k0, w.omega, c->stream));
    PA_HIP(launch_state_norm(c->d, w.omega, kind, w.norm, c->stream));
    PA_HIP(launch_state_scale(c->d, w.omega, kind, target, w.norm, c->stream));
    return state_to_phys(c, w, w.omega, omega_out);
} PA_CATCH_HOST

pa_status pa_forward(pa_ctx* c, const double* omega0, int32_t n_steps, const pa_obs* obs, double* J_out,
                     double* obs_out, double* omega_T, int32_t ckpt_every, void* ckpt, void* workspace,
                     size_t wbytes) try {
    g_err.clear();
    if (!c || !omega0) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0) return fail(PA_EINVAL, "n_steps must be >= 0");
    if (ckpt_every < 1) return fail(PA_EINVAL, "ckpt_every must be >= 1");
    if (reinterpret_cast<uintptr_t>(ckpt) % 16) return fail(PA_EINVAL, "checkpoint buffer must be 16-byte aligned");
    if (J_out && (!obs || !obs->values)) return fail(PA_EINVAL, "J_out needs observation values");
    if (obs_out && !obs) return fail(PA_EINVAL, "obs_out needs observations");
    PA_TRY(require_device(c->stream, {{omega0, "omega0"}, {J_out, "J_out"}, {obs_out, "obs_out"}, {omega_T, "omega_T"},
                           {ckpt, "ckpt"}, {workspace, "workspace"}, {obs ? obs->values : nullptr, "obs values"}}));
    ObsPlan op;
    PA_TRY(make_obs_plan(c, obs, n_steps, false, &op));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, 0, ckpt_every, op.max_times, 0, &w));
    const int K = seg_len(n_steps, ckpt_every);
    PA_TRY(forward_sweep(c, w, omega0, n_steps, op, obs_out, reinterpret_cast<cd*>(ckpt), K, false));
    if (J_out) {
        if (op.n > 0) PA_HIP(launch_copy(J_out, w.J, c->d.B, c->stream));
        else PA_HIP(launch_fill(J_out, 0.0, c->d.B, c->stream));
    }
    if (omega_T) PA_TRY(state_to_phys(c, w, w.omega, omega_T));
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_adjoint_from_checkpoints(pa_ctx* c, const void* ckpt, int32_t n_steps, const pa_obs* obs,
                                      const double* scale, double* grad_out, int32_t ckpt_every, void* workspace,
                                      size_t wbytes) try {
    g_err.clear();
    if (!c || !ckpt || !grad_out) return fail(PA_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ckpt) % 16) return fail(PA_EINVAL, "checkpoint buffer must be 16-byte aligned");
    if (n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    PA_TRY(require_device(c->stream, {{ckpt, "ckpt"}, {scale, "scale"}, {grad_out, "grad_out"}, {workspace, "workspace"},
                           {obs ? obs->values : nullptr, "obs values"}}));
    ObsPlan op;
    PA_TRY(make_obs_plan(c, obs, n_steps, true, &op));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, n_steps, ckpt_every, op.max_times, 0, &w));
    const int K = seg_len(n_steps, ckpt_every);
    return backward_sweep(c, w, reinterpret_cast<const cd*>(ckpt), n_steps, K, &op, 0, -1, -1, scale, grad_out,
                          Shells(), false);
} PA_CATCH_HOST

pa_status pa_adjoint_gradient(pa_ctx* c, const double* omega0, int32_t n_steps, const pa_obs* obs, double* J_out,
                              double* grad_out, int32_t ckpt_every, void* workspace, size_t wbytes) try {
    g_err.clear();
    if (!c || !omega0 || !grad_out) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    PA_TRY(require_device(c->stream, {{omega0, "omega0"}, {J_out, "J_out"}, {grad_out, "grad_out"}, {workspace, "workspace"},
                           {obs ? obs->values : nullptr, "obs values"}}));
    ObsPlan op;
    PA_TRY(make_obs_plan(c, obs, n_steps, true, &op));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, n_steps, ckpt_every, op.max_times, 0, &w, true));
    const int K = seg_len(n_steps, ckpt_every);
    const std::vector<PlanAct>* plan = plan_for(c, n_segments(n_steps, K));
    PA_TRY(forward_sweep(c, w, omega0, n_steps, op, nullptr, w.ckpt, K, true, plan));
    if (J_out) {
        if (op.n > 0) PA_HIP(launch_copy(J_out, w.J, c->d.B, c->stream));
        else PA_HIP(launch_fill(J_out, 0.0, c->d.B, c->stream));
    }
    return backward_sweep(c, w, w.ckpt, n_steps, K, &op, 0, -1, -1, nullptr, grad_out, Shells(), true, plan);
} PA_CATCH_HOST

// pa_adjoint_gradient with the workspace carved from this device's scratch.
// Allocates nothing: no device memory, and on its success path no host memory
// (the observation plan is a binary search over the caller's steps).
pa_status pa_adjoint_gradient_noalloc(pa_ctx* c, const double* omega0, int32_t n_steps, const pa_obs* obs,
                                      double* J_out, double* grad_out, int32_t ckpt_every) try {
    g_err.clear();
    if (!c || !omega0 || !grad_out) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    const int K = seg_len(n_steps, ckpt_every);
    if (plan_mode(c, n_segments(n_steps, K)))
        return fail(PA_EINVAL, "pa_adjoint_gradient_noalloc keeps one state per segment boundary: "
                               "set the snapshot budget to 0");
    PA_TRY(require_device(c->stream, {{omega0, "omega0"}, {J_out, "J_out"}, {grad_out, "grad_out"},
                           {obs ? obs->values : nullptr, "obs values"}}));
    ObsPlan op;
    PA_TRY(make_obs_plan(c, obs, n_steps, true, &op));
    const size_t need = carve(c, n_steps, ckpt_every, op.max_times, 0, nullptr).total;
    if (need > PA_NOALLOC_SCRATCH_BYTES)
        return fail(PA_EINVAL, "this gradient needs " + std::to_string(need) +
                                   " bytes of scratch, more than the PA_NOALLOC_SCRATCH_BYTES the library holds "
                                   "per device: lower ckpt_every, or call pa_adjoint_gradient with a workspace");
    void* ws = (c->device >= 0 && c->device < SCRATCH_DEVICES) ? g_scratch_ptr[c->device] : nullptr;
    if (!ws)
        return fail(PA_EDEVICE, std::string("no scratch address on this device: ") +
                                    ((c->device >= 0 && c->device < SCRATCH_DEVICES)
                                         ? hipGetErrorString(g_scratch_err[c->device])
                                         : "device index out of range"));
    WS w;
    PA_TRY(check_ws(c, ws, PA_NOALLOC_SCRATCH_BYTES, n_steps, ckpt_every, op.max_times, 0, &w, true));
    PA_TRY(forward_sweep(c, w, omega0, n_steps, op, nullptr, w.ckpt, K, true, nullptr));
    if (J_out) {
        if (op.n > 0) PA_HIP(launch_copy(J_out, w.J, c->d.B, c->stream));
        else PA_HIP(launch_fill(J_out, 0.0, c->d.B, c->stream));
    }
    return backward_sweep(c, w, w.ckpt, n_steps, K, &op, 0, -1, -1, nullptr, grad_out, Shells(), true, nullptr);
} PA_CATCH_HOST

pa_status pa_ensemble_acc_bytes(const pa_ctx* c, int32_t n_steps, int32_t n_shells, size_t* lambda_bytes,
                                size_t* energy_bytes, size_t* shell_bytes) try {
    if (!c || !lambda_bytes || !energy_bytes || !shell_bytes) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || n_shells < 1) return fail(PA_EINVAL, "bad sizes");
    const size_t rows = (size_t)n_steps + 1;
    *lambda_bytes = rows * c->d.KY * c->d.KXP * sizeof(cd);
    *energy_bytes = rows * sizeof(double);
    *shell_bytes = rows * n_shells * sizeof(double);
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_adjoint_impulse(pa_ctx* c, const double* omega0, int32_t n_steps, int32_t ix, int32_t iy,
                             int32_t n_shells, double* shells_out, double* field_out, pa_ensemble_acc* acc,
                             int32_t ckpt_every, void* workspace, size_t wbytes) try {
    g_err.clear();
    if (!c || !omega0 || !shells_out) return fail(PA_EINVAL, "NULL argument");
    if (n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    if (ix < 0 || iy < 0 || ix >= c->d.N || iy >= c->d.N) return fail(PA_EINVAL, "impulse point outside the grid");
    if (n_shells < 1 || n_shells > c->n_shell_max)
        return fail(PA_EINVAL, "n_shells must be in [1, floor(sqrt(2) Kc)]");
    if (acc && (!acc->lambda_sum || !acc->energy_sum || !acc->shell_sum || acc->count < 0))
        return fail(PA_EINVAL, "ensemble accumulator has a NULL buffer or a negative count");
    if (acc && reinterpret_cast<uintptr_t>(acc->lambda_sum) % 16)
        return fail(PA_EINVAL, "lambda_sum must be 16-byte aligned");
    PA_TRY(require_device(c->stream, {{omega0, "omega0"}, {shells_out, "shells_out"}, {field_out, "field_out"},
                           {workspace, "workspace"}, {acc ? acc->lambda_sum : nullptr, "lambda_sum"},
                           {acc ? acc->energy_sum : nullptr, "energy_sum"}, {acc ? acc->shell_sum : nullptr, "shell_sum"}}));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, n_steps, ckpt_every, 0, 0, &w, true));
    const int K = seg_len(n_steps, ckpt_every);
    ObsPlan none;
    PA_TRY(make_obs_plan(c, nullptr, n_steps, false, &none));
    const std::vector<PlanAct>* plan = plan_for(c, n_segments(n_steps, K));
    PA_TRY(forward_sweep(c, w, omega0, n_steps, none, nullptr, w.ckpt, K, true, plan));
    Shells sh;
    sh.out = shells_out;
    sh.n = n_shells;
    sh.stride = (size_t)(n_steps + 1) * n_shells;
    sh.acc = acc;
    PA_TRY(backward_sweep(c, w, w.ckpt, n_steps, K, nullptr, 1, ix, iy, nullptr, field_out, sh, true, plan));
    if (acc) acc->count += c->d.B;
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_ensemble_stats(pa_ctx* c, const pa_ensemble_acc* acc, int32_t rows, int32_t n_shells,
                            double* mean_energy, double* energy_of_mean, double* total_mean, double* total_of_mean,
                            double* snr) try {
    g_err.clear();
    if (!c || !acc || !acc->lambda_sum || !acc->energy_sum || !acc->shell_sum || !mean_energy || !energy_of_mean ||
        !total_mean || !total_of_mean || !snr)
        return fail(PA_EINVAL, "NULL argument");
    if (acc->count < 1) return fail(PA_EINVAL, "no members accumulated");
    if (rows < 1 || n_shells < 1 || n_shells > c->n_shell_max) return fail(PA_EINVAL, "bad sizes");
    PA_TRY(require_device(c->stream, {{acc->lambda_sum, "lambda_sum"}, {acc->energy_sum, "energy_sum"},
                           {acc->shell_sum, "shell_sum"}, {mean_energy, "mean_energy"},
                           {energy_of_mean, "energy_of_mean"}, {total_mean, "total_mean"},
                           {total_of_mean, "total_of_mean"}, {snr, "snr"}}));
    PA_HIP(launch_ens_stats(c->d, rows, n_shells, 1.0 / (double)acc->count, static_cast<const cd*>(acc->lambda_sum),
                            acc->shell_sum, acc->energy_sum, c->shell_start, c->shell_modes, mean_energy,
                            energy_of_mean, total_mean, total_of_mean, snr, c->stream));
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_first_guess(pa_ctx* c, int32_t stride, const double* probes, double* omega_out, void* workspace,
                         size_t wbytes) try {
    g_err.clear();
    if (!c || !probes || !omega_out) return fail(PA_EINVAL, "NULL argument");
    if (stride < 1 || stride > c->d.N || c->d.N % stride) return fail(PA_EINVAL, "stride must divide N");
    PA_TRY(require_device(c->stream, {{probes, "probes"}, {omega_out, "omega_out"}, {workspace, "workspace"}}));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, 0, 1, 0, 0, &w));
    double* gu = w.P0;
    double* gv = w.P1;
    const int M = c->d.N / stride;
    PA_HIP(launch_scatter_probes(c->d.B, c->d.N, stride, probes, gu, gv, c->stream));
    PA_HIP(launch_row_r2c(c->d, gu, w.Yf[0], c->tw, c->stream));
    PA_HIP(launch_row_r2c(c->d, gv, w.Yf[1], c->tw, c->stream));
    ColArgs a = col_base(c);
    a.yin[0] = w.Yf[0];
    a.yin[1] = w.Yf[1];
    a.lowpass = (M % 2 == 0) ? M / 2 - 1 : (M - 1) / 2;
    a.nout = 1;
    a.fields[0] = F_OMEGA;
    a.yout[0] = w.Y0;
    PA_HIP(launch_col(c->d, COL_FIRST_GUESS, a, c->stream));
    PA_HIP(launch_row_c2r(c->d, w.Y0, omega_out, c->tw, c->stream));
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_shell_growth(pa_ctx* c, const double* shells, int32_t rows, int32_t n_shells, double tau_min,
                          double tau_max, double* mean_out, double* rate_out) try {
    g_err.clear();
    if (!c || !shells || !rate_out) return fail(PA_EINVAL, "NULL argument");
    if (rows < 1 || n_shells < 1) return fail(PA_EINVAL, "bad sizes");
    if (!std::isfinite(tau_min) || !std::isfinite(tau_max) || tau_max < tau_min)
        return fail(PA_EINVAL, "bad growth window");
    PA_TRY(require_device(c->stream, {{shells, "shells"}, {mean_out, "mean_out"}, {rate_out, "rate_out"}}));
    PA_HIP(launch_shell_growth(c->d.B, rows, n_shells, shells, c->ph.dt, tau_min, tau_max, mean_out, rate_out,
                               c->stream));
    return PA_OK;
} PA_CATCH_HOST

pa_status pa_precondition(pa_ctx* c, const pa_kernel* k, double power, const double* in, double* out,
                          void* workspace, size_t wbytes) try {
    g_err.clear();
    if (!c || !in || !out) return fail(PA_EINVAL, "NULL argument");
    PA_TRY(valid_kernel(k));
    if (!std::isfinite(power)) return fail(PA_EINVAL, "power must be finite");
    PA_TRY(check_multiplier(c, k, power));
    PA_TRY(require_device(c->stream, {{in, "in"}, {out, "out"}, {workspace, "workspace"}}));
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, 0, 1, 0, 0, &w));
    PA_HIP(launch_make_mult(c->d, k->kind, k->metric, k->param, power, w.mult, c->stream));
    return apply_filter(c, w, w.mult, in, out);
} PA_CATCH_HOST

}  // extern "C"

namespace {

// Host side of the batched optimiser.  Every O(N^2) operation and every
// per-member scalar decision of the recursion runs on the device (misc.hip:
// lbfgs_*); the host keeps only the loop control (which members still run,
// how many iterations each has completed) and reads one status block per
// line-search trial.  Transfers go through the context's pinned buffer.
struct Opt {
    pa_ctx* c;
    WS& w;
    size_t n;        // N*N
    int B;

    pa_status pinned(size_t bytes) {
        if (c->pin_bytes >= bytes) return PA_OK;
        if (c->pin) (void)hipHostFree(c->pin);
        c->pin = nullptr;
        c->pin_bytes = 0;
        PA_HIP(hipHostMalloc(&c->pin, bytes, hipHostMallocDefault));
        c->pin_bytes = bytes;
        return PA_OK;
    }
    // device -> host (through the pinned buffer), then wait for it
    pa_status read(const void* dev, size_t bytes, void* host) {
        PA_TRY(pinned(bytes));
        PA_HIP(hipMemcpyAsync(c->pin, dev, bytes, hipMemcpyDeviceToHost, c->stream));
        PA_HIP(hipStreamSynchronize(c->stream));
        std::memcpy(host, c->pin, bytes);
        return PA_OK;
    }
    // host -> device (through the pinned buffer, which is free again on return)
    pa_status write(void* dev, const void* host, size_t bytes) {
        PA_TRY(pinned(bytes));
        std::memcpy(c->pin, host, bytes);
        PA_HIP(hipMemcpyAsync(dev, c->pin, bytes, hipMemcpyHostToDevice, c->stream));
        PA_HIP(hipStreamSynchronize(c->stream));
        return PA_OK;
    }
    pa_status sync() {
        PA_HIP(hipStreamSynchronize(c->stream));
        return PA_OK;
    }
};

}  // namespace

namespace {

// Optimiser state of a batched solve (pa_assimilate_ex), caller-owned device
// memory: a header and the O(B m) scalars, then the latent iterate x, its
// gradient g and the m-slot pair ring (S, Y), each B N^2 doubles.
const uint64_t OPT_MAGIC = 0x3154534f5054504fULL;   // "OPTPOST1"
struct OptHeader {
    uint64_t magic;
    int32_t N, B, m, method, per_member, n_steps, n_times, stride, head, iters;
};
struct OptLayout {
    size_t J, running, done, ok, rho, gam, kern, x, g, S, Y, total;
};
OptLayout opt_layout(int N, int B, int m, int nk) {
    auto up = [](size_t v, size_t a) { return (v + a - 1) / a * a; };
    const size_t SP = (size_t)B * N * N * sizeof(double);
    OptLayout l;
    size_t o = up(sizeof(OptHeader), 16);
    l.J = o;        o = up(o + sizeof(double) * B, 16);
    l.running = o;  o = up(o + sizeof(int32_t) * B, 16);
    l.done = o;     o = up(o + sizeof(int32_t) * B, 16);
    l.ok = o;       o = up(o + sizeof(int32_t) * (size_t)m * B, 16);
    l.rho = o;      o = up(o + sizeof(double) * (size_t)m * B, 16);
    l.gam = o;      o = up(o + sizeof(double) * (size_t)m * B, 16);
    l.kern = o;     o = up(o + sizeof(pa_kernel) * nk, 256);
    l.x = o;        o += SP;
    l.g = o;        o += SP;
    l.S = o;        o += SP * m;
    l.Y = o;        o += SP * m;
    l.total = o;
    return l;
}

}  // namespace

// kernels: host array of B kernels (one per member) when per_member, else one kernel for all.
// state_in: resume from a state a previous call wrote (omega_inout is then output only);
// state_out: write the state after the last iteration (which then also takes the gradient
// and stores the pair, as a longer run would).
static pa_status assimilate_impl(pa_ctx* c, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                 const pa_kernel* kernels, bool per_member, int32_t method, int32_t max_iter,
                                 int32_t lbfgs_m, int32_t ckpt_every, double* J_hist, int32_t* iters_done,
                                 void* workspace, size_t wbytes, const void* state_in = nullptr,
                                 void* state_out = nullptr, size_t state_bytes = 0, bool member_obs = false) {
    g_err.clear();
    if (!c || !omega_inout || !J_hist || !iters_done) return fail(PA_EINVAL, "NULL argument");
    if (member_obs && (state_in || state_out)) return fail(PA_EINVAL, "per-member observations keep no optimiser state");
    if (member_obs && !obs) return fail(PA_EINVAL, "obs is NULL");
    if (!kernels) return fail(PA_EINVAL, "kernel is NULL");
    for (int b = 0; b < (per_member ? c->d.B : 1); ++b) {
        PA_TRY(valid_kernel(&kernels[b]));
        PA_TRY(check_multiplier(c, &kernels[b], 0.5));
        PA_TRY(check_multiplier(c, &kernels[b], -0.5));
    }
    if (method != 0 && method != 1) return fail(PA_EINVAL, "method must be 0 (L-BFGS) or 1 (steepest descent)");
    if (max_iter < 0 || n_steps < 0 || ckpt_every < 1) return fail(PA_EINVAL, "bad sizes");
    if (method == 0 && lbfgs_m < 1) return fail(PA_EINVAL, "lbfgs_m must be >= 1");
    PA_TRY(require_device(c->stream, {{omega_inout, "omega_inout"}, {workspace, "workspace"},
                           {obs ? obs->values : nullptr, "obs values"}, {state_in, "state_in"},
                           {state_out, "state_out"}}));
    ObsPlan op;
    std::vector<ObsRange> ranges;
    std::vector<int> active;
    if (member_obs) {
        for (int b = 0; b < c->d.B; ++b)
            if (obs[b].values) PA_TRY(require_device(c->stream, {{obs[b].values, "obs values"}}));
        PA_TRY(make_member_plan(c, obs, n_steps, ranges, active, &op));
        if (plan_mode(c, n_segments(n_steps, seg_len(n_steps, ckpt_every))))
            return fail(PA_EINVAL, "per-member observations keep one state per segment boundary: "
                                   "set the snapshot budget to 0");
    } else {
        PA_TRY(make_obs_plan(c, obs, n_steps, true, &op));
    }
    if (op.n == 0) return fail(PA_EINVAL, "assimilation needs at least one observation time");
    const int m = std::max(1, (int)lbfgs_m);
    const int nk = per_member ? c->d.B : 1;
    const OptLayout sl_ = opt_layout(c->d.N, c->d.B, m, nk);
    if ((state_in && reinterpret_cast<uintptr_t>(state_in) % 256) ||
        (state_out && reinterpret_cast<uintptr_t>(state_out) % 256))
        return fail(PA_EINVAL, "optimiser state must be 256-byte aligned");
    if ((state_in || state_out) && state_bytes < sl_.total)
        return fail(PA_EINVAL, "optimiser state too small: need " + std::to_string(sl_.total) + " bytes");
    OptHeader want{OPT_MAGIC, c->d.N, c->d.B, m, method, per_member ? 1 : 0, n_steps, op.max_times,
                   obs ? obs->stride : 0, 0, 0};
    // a resumed state: header and scalars read (and checked) before anything is enqueued
    std::vector<unsigned char> hs;
    OptHeader got{};
    if (state_in) {
        hs.resize(sl_.x);
        PA_HIP(hipMemcpyAsync(hs.data(), state_in, sl_.x, hipMemcpyDeviceToHost, c->stream));
        PA_HIP(hipStreamSynchronize(c->stream));
        std::memcpy(&got, hs.data(), sizeof(got));
        const bool same = got.magic == want.magic && got.N == want.N && got.B == want.B && got.m == want.m &&
                          got.method == want.method && got.per_member == want.per_member &&
                          got.n_steps == want.n_steps && got.n_times == want.n_times && got.stride == want.stride &&
                          got.head >= 0 && got.iters >= 0 &&
                          std::memcmp(hs.data() + sl_.kern, kernels, sizeof(pa_kernel) * nk) == 0;
        if (!same)
            return fail(PA_EINVAL, "optimiser state does not match this call (sizes, method, memory, window, "
                                   "observation layout or kernels)");
    }
    WS w;
    PA_TRY(check_ws(c, workspace, wbytes, n_steps, ckpt_every, op.max_times, m, &w, true));
    const int B = c->d.B;
    const int K = seg_len(n_steps, ckpt_every);
    const size_t n = (size_t)c->d.N * c->d.N;
    const size_t SP = (size_t)B * n;
    const size_t MT = (size_t)c->d.KY * c->d.KXP;
    const size_t MTB = per_member ? (size_t)B * MT : MT;
    double* mult_p = w.mult;         // (m^2 W)^(+1/2), one table per member when per_member
    double* mult_m = w.mult + MTB;   // (m^2 W)^(-1/2)
    for (int b = 0; b < (per_member ? B : 1); ++b) {
        const pa_kernel* k = &kernels[b];
        PA_HIP(launch_make_mult(c->d, k->kind, k->metric, k->param, 0.5, mult_p + b * MT, c->stream));
        PA_HIP(launch_make_mult(c->d, k->kind, k->metric, k->param, -0.5, mult_m + b * MT, c->stream));
    }
    Opt o{c, w, n, B};
    const StatLayout stl = stat_layout(B);
    int* counts = reinterpret_cast<int*>(w.ostat);
    int* acc_d = reinterpret_cast<int*>(w.ostat + stl.acc);
    double* Jt_d = reinterpret_cast<double*>(w.ostat + stl.Jt);
    const std::vector<PlanAct>* plan = plan_for(c, n_segments(n_steps, K));

    auto eval_J = [&](const double* x) -> pa_status {
        PA_TRY(apply_filter(c, w, mult_p, x, w.w, per_member));
        return forward_sweep(c, w, w.w, n_steps, op, nullptr, w.ckpt, K, true, plan);
    };
    // gradient at the point whose forward sweep last filled w.ckpt
    auto eval_grad = [&](double* gout) -> pa_status {
        PA_TRY(backward_sweep(c, w, w.ckpt, n_steps, K, &op, 0, -1, -1, nullptr, w.gw, Shells(), true, plan));
        return apply_filter(c, w, mult_p, w.gw, gout, per_member);
    };
    auto dev_copy = [&](void* dst, const void* src, size_t bytes) -> pa_status {
        PA_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
        return PA_OK;
    };

    for (int i = 0; i < B * (max_iter + 1); ++i) J_hist[i] = NAN;
    // host loop control: members still iterating, iterations completed, members paused by a cancel flag
    std::vector<int> running(B, 1), done(B, 0), paused(B, 0);
    std::vector<double> Jh(B);
    int head = 0;   // pushes into the pair ring so far: push p lives in slot p % m
    int it0 = 0;    // iterations completed before this call (the most any member has done)

    if (state_in) {
        const unsigned char* h = hs.data();
        auto rd = [&](size_t off, size_t i, auto* v) { std::memcpy(v, h + off + i * sizeof(*v), sizeof(*v)); };
        head = got.head;
        it0 = got.iters;
        for (int b = 0; b < B; ++b) {
            int32_t r, d;
            rd(sl_.J, b, &Jh[b]);
            rd(sl_.running, b, &r);
            rd(sl_.done, b, &d);
            running[b] = r;
            done[b] = d;
            if (!running[b]) iters_done[b] = -(done[b] + 1);
        }
        const unsigned char* d = static_cast<const unsigned char*>(state_in);
        PA_TRY(dev_copy(w.oJ, d + sl_.J, sizeof(double) * B));
        PA_TRY(dev_copy(w.orun, d + sl_.running, sizeof(int32_t) * B));
        PA_TRY(dev_copy(w.ook, d + sl_.ok, sizeof(int32_t) * (size_t)m * B));
        PA_TRY(dev_copy(w.orho, d + sl_.rho, sizeof(double) * (size_t)m * B));
        PA_TRY(dev_copy(w.ogam, d + sl_.gam, sizeof(double) * (size_t)m * B));
        PA_HIP(launch_copy(w.x, reinterpret_cast<const double*>(d + sl_.x), SP, c->stream));
        PA_HIP(launch_copy(w.g, reinterpret_cast<const double*>(d + sl_.g), SP, c->stream));
        for (int q = 0; q < m; ++q) {
            PA_HIP(launch_copy(w.S + q * SP, reinterpret_cast<const double*>(d + sl_.S) + q * SP, SP, c->stream));
            PA_HIP(launch_copy(w.Yv + q * SP, reinterpret_cast<const double*>(d + sl_.Y) + q * SP, SP, c->stream));
        }
    } else {
        PA_HIP(launch_fill_int(w.ook, 0, (size_t)m * B, c->stream));
        PA_HIP(launch_fill(w.orho, 0.0, (size_t)m * B, c->stream));
        PA_HIP(launch_fill(w.ogam, 1.0, (size_t)m * B, c->stream));
        PA_HIP(launch_fill_int(w.orun, 1, B, c->stream));
        PA_TRY(apply_filter(c, w, mult_m, omega_inout, w.x, per_member));
        PA_TRY(eval_J(w.x));
        PA_TRY(eval_grad(w.g));
        PA_HIP(launch_copy(w.oJ, w.J, B, c->stream));
        PA_TRY(o.read(w.J, sizeof(double) * B, Jh.data()));
    }
    for (int b = 0; b < B; ++b) J_hist[(size_t)b * (max_iter + 1)] = Jh[b];

    std::vector<unsigned char> st(stl.bytes);   // the last trial's status block
    for (int it = 0; it < max_iter; ++it) {
        // members cancelled by the caller (another thread may set their flags at any time) stop here,
        // after their last completed iteration
        if (c->cancel) {
            bool changed = false;
            for (int b = 0; b < B; ++b)
                if (running[b] && __atomic_load_n(c->cancel + b, __ATOMIC_ACQUIRE)) {
                    running[b] = 0;
                    paused[b] = 1;
                    iters_done[b] = done[b];
                    changed = true;
                }
            if (changed) PA_TRY(o.write(w.orun, running.data(), sizeof(int) * B));
        }
        bool any = false;
        for (int b = 0; b < B; ++b) any = any || running[b];
        if (!any) break;
        // ---- search direction d = -H g (two-loop recursion over the ring window [lo, hi)); members
        // without pairs in it get zero coefficients and gamma = 1, i.e. d = -g
        const int lo = std::max(0, head - m), hi = head;
        if (method == 0) {
            PA_HIP(launch_copy(w.dv, w.g, SP, c->stream));
            for (int p = hi - 1; p >= lo; --p) {
                const int sl = p % m;
                PA_HIP(launch_dot(B, n, w.S + sl * SP, w.dv, w.dots, w.partial, c->stream));
                PA_HIP(launch_lbfgs_first(B, sl, w.dots, w.ook, w.orho, w.oal, w.coef, c->stream));
                PA_HIP(launch_axpy(B, n, w.coef, 1.0, w.Yv + sl * SP, w.dv, nullptr, c->stream));
            }
            PA_HIP(launch_lbfgs_gamma(B, m, lo, hi, w.ook, w.ogam, w.coef, c->stream));
            PA_HIP(launch_scal_copy(B, n, w.coef, w.dv, w.dv, c->stream));
            for (int p = lo; p < hi; ++p) {
                const int sl = p % m;
                PA_HIP(launch_dot(B, n, w.Yv + sl * SP, w.dv, w.dots, w.partial, c->stream));
                PA_HIP(launch_lbfgs_second(B, sl, w.dots, w.ook, w.orho, w.oal, w.coef, c->stream));
                PA_HIP(launch_axpy(B, n, w.coef, 1.0, w.S + sl * SP, w.dv, nullptr, c->stream));
            }
            PA_HIP(launch_fill(w.coef, -1.0, B, c->stream));
            PA_HIP(launch_scal_copy(B, n, w.coef, w.dv, w.dv, c->stream));
        } else {
            PA_HIP(launch_fill(w.coef, -1.0, B, c->stream));
            PA_HIP(launch_scal_copy(B, n, w.coef, w.g, w.dv, c->stream));
        }
        PA_HIP(launch_dot(B, n, w.g, w.dv, w.ogd, w.partial, c->stream));
        PA_HIP(launch_dot(B, n, w.g, w.g, w.ogg, w.partial, c->stream));
        // a member whose d is not a descent direction drops its pairs and takes d = -g
        PA_HIP(launch_lbfgs_direction(B, m, lo, hi, method == 0, w.ogd, w.ogg, w.oJ, w.ook, w.oreset, w.oalpha,
                                      w.orun, w.opend, acc_d, c->stream));
        PA_HIP(launch_fill(w.coef, -1.0, B, c->stream));
        PA_HIP(launch_axpby(B, n, w.coef, 1.0, w.g, nullptr, 0.0, w.g, w.dv, w.oreset, c->stream));
        // ---- backtracking Armijo line search, per member; one status read per trial
        PA_HIP(launch_copy(w.xt, w.x, SP, c->stream));
        for (int trial = 0; trial < 30; ++trial) {
            PA_HIP(launch_axpby(B, n, nullptr, 1.0, w.x, w.oalpha, 1.0, w.dv, w.xt, w.opend, c->stream));
            PA_TRY(eval_J(w.xt));
            PA_HIP(launch_lbfgs_armijo(B, w.J, w.oJ, w.oalpha, w.ogd, w.opend, acc_d, Jt_d, counts, c->stream));
            PA_TRY(o.read(w.ostat, stl.bytes, st.data()));
            int pending;
            std::memcpy(&pending, st.data(), sizeof(int));
            if (pending == 0) break;
        }
        // members still pending failed (step size collapsed); the accepted ones take their trial cost
        PA_HIP(launch_lbfgs_close(B, w.opend, acc_d, Jt_d, w.orun, w.oJ, c->stream));
        const int* acc_h = reinterpret_cast<const int*>(st.data() + stl.acc);
        const double* Jt_h = reinterpret_cast<const double*>(st.data() + stl.Jt);
        bool any_acc = false;
        for (int b = 0; b < B; ++b) {
            if (running[b] && !acc_h[b]) {
                running[b] = 0;
                iters_done[b] = -(done[b] + 1);
            }
            any_acc = any_acc || acc_h[b];
        }
        if (!any_acc) break;
        // the last iteration skips the gradient at the new point, unless a state is kept for a resume
        const bool last = it == max_iter - 1 && !state_out;
        if (!last) {
            // the last trial's forward sweep holds valid checkpoints for every accepted member
            PA_TRY(eval_grad(w.gt));
            if (method == 0) {
                const int sl = head % m;
                PA_HIP(launch_axpby(B, n, nullptr, 1.0, w.xt, nullptr, -1.0, w.x, w.S + sl * SP, nullptr, c->stream));
                PA_HIP(launch_axpby(B, n, nullptr, 1.0, w.gt, nullptr, -1.0, w.g, w.Yv + sl * SP, nullptr, c->stream));
                double* sy = w.dots;
                double* ss = w.dots + B;
                double* yy = w.dots + 2 * B;
                PA_HIP(launch_dot(B, n, w.S + sl * SP, w.Yv + sl * SP, sy, w.partial, c->stream));
                PA_HIP(launch_dot(B, n, w.S + sl * SP, w.S + sl * SP, ss, w.partial, c->stream));
                PA_HIP(launch_dot(B, n, w.Yv + sl * SP, w.Yv + sl * SP, yy, w.partial, c->stream));
                PA_HIP(launch_lbfgs_pair(B, sl, sy, ss, yy, acc_d, w.ook, w.orho, w.ogam, c->stream));
                ++head;
            }
            PA_HIP(launch_axpby(B, n, nullptr, 1.0, w.gt, nullptr, 0.0, w.gt, w.g, acc_d, c->stream));
        }
        PA_HIP(launch_axpby(B, n, nullptr, 1.0, w.xt, nullptr, 0.0, w.xt, w.x, acc_d, c->stream));
        for (int b = 0; b < B; ++b) {
            if (!acc_h[b]) continue;
            Jh[b] = Jt_h[b];
            ++done[b];
            J_hist[(size_t)b * (max_iter + 1) + it + 1] = Jh[b];
        }
        if (last) break;
    }
    for (int b = 0; b < B; ++b)
        if (running[b]) iters_done[b] = done[b];
    PA_TRY(apply_filter(c, w, mult_p, w.x, omega_inout, per_member));
    if (state_out) {
        int iters = it0;
        for (int b = 0; b < B; ++b) iters = std::max(iters, done[b]);
        OptHeader hd = want;
        hd.head = head;
        hd.iters = iters;
        // header, running and done flags and kernels from the host; the scalars of the
        // recursion, the iterate, its gradient and the pairs from the device
        std::vector<unsigned char> out(sl_.x, 0);
        std::memcpy(out.data(), &hd, sizeof(hd));
        auto wr = [&](size_t off, size_t i, auto v) { std::memcpy(out.data() + off + i * sizeof(v), &v, sizeof(v)); };
        for (int b = 0; b < B; ++b) {
            wr(sl_.running, b, (int32_t)(running[b] || paused[b]));   // a cancelled member resumes
            wr(sl_.done, b, (int32_t)done[b]);
        }
        std::memcpy(out.data() + sl_.kern, kernels, sizeof(pa_kernel) * nk);
        unsigned char* d = static_cast<unsigned char*>(state_out);
        PA_TRY(o.write(d, out.data(), out.size()));
        PA_TRY(dev_copy(d + sl_.J, w.oJ, sizeof(double) * B));
        PA_TRY(dev_copy(d + sl_.ok, w.ook, sizeof(int32_t) * (size_t)m * B));
        PA_TRY(dev_copy(d + sl_.rho, w.orho, sizeof(double) * (size_t)m * B));
        PA_TRY(dev_copy(d + sl_.gam, w.ogam, sizeof(double) * (size_t)m * B));
        PA_HIP(launch_copy(reinterpret_cast<double*>(d + sl_.x), w.x, SP, c->stream));
        PA_HIP(launch_copy(reinterpret_cast<double*>(d + sl_.g), w.g, SP, c->stream));
        for (int q = 0; q < m; ++q) {
            PA_HIP(launch_copy(reinterpret_cast<double*>(d + sl_.S) + q * SP, w.S + q * SP, SP, c->stream));
            PA_HIP(launch_copy(reinterpret_cast<double*>(d + sl_.Y) + q * SP, w.Yv + q * SP, SP, c->stream));
        }
    }
    PA_TRY(o.sync());
    return PA_OK;
}


extern "C" pa_status pa_assimilate(pa_ctx* c, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                   const pa_kernel* kernel, int32_t method, int32_t max_iter, int32_t lbfgs_m,
                                   int32_t ckpt_every, double* J_hist, int32_t* iters_done, void* workspace,
                                   size_t wbytes) try {
    return assimilate_impl(c, omega_inout, n_steps, obs, kernel, false, method, max_iter, lbfgs_m, ckpt_every,
                           J_hist, iters_done, workspace, wbytes);
} PA_CATCH_HOST

extern "C" pa_status pa_assimilate_state_bytes(const pa_ctx* c, int32_t lbfgs_m, int32_t per_member,
                                               size_t* bytes) try {
    if (!c || !bytes) return fail(PA_EINVAL, "NULL argument");
    if (lbfgs_m < 0) return fail(PA_EINVAL, "lbfgs_m must be >= 0");
    *bytes = opt_layout(c->d.N, c->d.B, std::max(1, (int)lbfgs_m), per_member ? c->d.B : 1).total;
    return PA_OK;
} PA_CATCH_HOST

extern "C" pa_status pa_assimilate_ex(pa_ctx* c, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                      const pa_kernel* kernels, int32_t per_member, int32_t method,
                                      int32_t max_iter, int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                                      int32_t* iters_done, const void* state_in, void* state_out,
                                      size_t state_bytes, void* workspace, size_t wbytes) try {
    return assimilate_impl(c, omega_inout, n_steps, obs, kernels, per_member != 0, method, max_iter, lbfgs_m,
                           ckpt_every, J_hist, iters_done, workspace, wbytes, state_in, state_out, state_bytes);
} PA_CATCH_HOST

extern "C" pa_status pa_assimilate_members(pa_ctx* c, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                           const pa_kernel* kernels, int32_t method, int32_t max_iter,
                                           int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                                           int32_t* iters_done, void* workspace, size_t wbytes) try {
    return assimilate_impl(c, omega_inout, n_steps, obs, kernels, true, method, max_iter, lbfgs_m, ckpt_every,
                           J_hist, iters_done, workspace, wbytes, nullptr, nullptr, 0, true);
} PA_CATCH_HOST

extern "C" pa_status pa_assimilate_kernels(pa_ctx* c, double* omega_inout, int32_t n_steps, const pa_obs* obs,
                                           const pa_kernel* kernels, int32_t method, int32_t max_iter,
                                           int32_t lbfgs_m, int32_t ckpt_every, double* J_hist,
                                           int32_t* iters_done, void* workspace, size_t wbytes) try {
    return assimilate_impl(c, omega_inout, n_steps, obs, kernels, true, method, max_iter, lbfgs_m, ckpt_every,
                           J_hist, iters_done, workspace, wbytes);
} PA_CATCH_HOST
