// C ABI of the dSDC library: argument validation, device memory, setup and the orchestration of
// Algorithm 2 (diagonal IMEX SDC step) on one HIP stream.
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <roctracer/roctx.h>

#include "common.h"

// Device scratch of the allocation-free IMEX-o2 step (imex2_step_noalloc): the intermediate state
// u* and the two tendencies k1, k2 of every member, kScratchBytes at most.  Each device that loads
// the library holds its own copy until the process ends; in host code the array's name is only a
// stand-in, so kernels get its device address (resolved once per device by hipGetSymbolAddress
// in sdc_init, with that device current) and never the name itself.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(SDC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on the first call per device);
// nullptr with *err set when it cannot be resolved.
double* scratch_address(int dev, hipError_t* err) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = e;
        g_scratch_ptr[dev] = e == hipSuccess ? static_cast<double*>(p) : nullptr;
        if (e != hipSuccess) (void)hipGetLastError();
        g_scratch_done[dev] = true;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

// FFT plan for nlon = 2^p or 3*2^p: an optional radix-3 stage, then the power of two split into
// radices 16, 8, 4, 2.  A pass advances fchunk of a workgroup's up to 5 signals together, every
// stage within the per-thread task budget fft_task_cap; the plan minimises the number of
// stage passes ceil(5 / fchunk) * stages.
constexpr int kFFTSignals = 5;

int fft_chunk_for(int n, const std::vector<int>& radices) {
    int best = 0;
    for (int F = 1; F <= kFFTSignals; ++F) {
        bool ok = true;
        for (int R : radices) ok = ok && (F * (n / R) + kBlock - 1) / kBlock <= fft_task_cap(R);
        if (ok) best = F;
    }
    return best;
}

void search_pow2(int n, int p_left, std::vector<int>& cur, const std::vector<int>& head,
                 std::vector<int>& best, int& best_cost) {
    if (p_left == 0) {
        std::vector<int> all(head);
        all.insert(all.end(), cur.begin(), cur.end());
        const int fc = fft_chunk_for(n, all);
        if (fc == 0) return;
        const int cost = (kFFTSignals + fc - 1) / fc * (int)all.size();
        if (best.empty() || cost < best_cost) {
            best = all;
            best_cost = cost;
        }
        return;
    }
    const int last = cur.empty() ? 4 : 31 - __builtin_clz(cur.back());
    for (int part = last; part >= 1; --part) {       // non-increasing radices
        if (part > p_left) continue;
        cur.push_back(1 << part);
        search_pow2(n, p_left - part, cur, head, best, best_cost);
        cur.pop_back();
    }
}

bool make_fft_plan(int n, FFTPlan& pl) {
    pl.n = n;
    pl.nst = 0;
    pl.fchunk = 0;
    int rest = n;
    std::vector<int> head;
    if (rest % 3 == 0) {
        rest /= 3;
        head.push_back(3);
    }
    int p = 0;
    while (rest > 1 && rest % 2 == 0) {
        rest /= 2;
        ++p;
    }
    if (rest != 1) return false;
    std::vector<int> cur, best;
    int best_cost = 0;
    if (p > 0) {
        search_pow2(n, p, cur, head, best, best_cost);
    } else {
        best = head;
    }
    if (best.empty() || (int)best.size() > kMaxFFTStages) return false;
    pl.fchunk = fft_chunk_for(n, best);
    if (pl.fchunk == 0) return false;
    for (int R : best) pl.radix[pl.nst++] = R;
    return true;
}

// Order workgroup tasks for round-robin dispatch over the 8 XCDs (workgroup b runs on XCD b % 8):
// every task of one group lands on the same XCD (its operands stay in that XCD's L2), groups are
// spread over the XCDs by work (largest first, onto the least-loaded XCD), and each XCD receives
// its tasks in decreasing work.  Empty slots are filled with `pad`.
template <class Task>
std::vector<Task> xcd_order(const std::vector<Task>& tasks, const std::vector<int>& group,
                            const std::vector<double>& work, Task pad) {
    constexpr int kXcd = 8;
    int ngroups = 0;
    for (int gidx : group) ngroups = gidx + 1 > ngroups ? gidx + 1 : ngroups;
    std::vector<double> gwork(ngroups, 0.0);
    for (size_t t = 0; t < tasks.size(); ++t) gwork[group[t]] += work[t];
    std::vector<int> order(ngroups);
    for (int gi = 0; gi < ngroups; ++gi) order[gi] = gi;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gwork[a] > gwork[b]; });
    std::vector<int> xcd_of(ngroups, 0);
    double load[kXcd] = {0};
    for (int gi : order) {
        int best = 0;
        for (int x = 1; x < kXcd; ++x)
            if (load[x] < load[best]) best = x;
        xcd_of[gi] = best;
        load[best] += gwork[gi];
    }
    std::vector<std::vector<size_t>> lists(kXcd);
    for (size_t t = 0; t < tasks.size(); ++t) lists[xcd_of[group[t]]].push_back(t);
    size_t longest = 0;
    for (auto& l : lists) {
        std::stable_sort(l.begin(), l.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
        longest = l.size() > longest ? l.size() : longest;
    }
    std::vector<Task> out(longest * kXcd, pad);
    for (int x = 0; x < kXcd; ++x)
        for (size_t r = 0; r < lists[x].size(); ++r) out[r * kXcd + x] = tasks[lists[x][r]];
    return out;
}

}  // namespace

// One launch group of a step as enqueue_step issues it, recorded instead of launched when a
// group merges its members' launches: an f_E evaluation (synthesis, grid, analysis with an
// optional fused node update) or a separate node-update launch.
struct StepOp {
    int kind;                         // 0: f_E of S states, 1: node update
    int S;
    const double* states;             // f_E: the states read in place (or nullptr: synthesis layout)
    double* out;
    double2* save;
    UpdateArgs upd;                   // f_E: the fused update (fuse_mode > 0); kind 1: the update
    int fuse_mode;
};

struct sdc_ctx {
    std::vector<StepOp>* rec = nullptr;   // when set, f_E and update launches are recorded here
    bool roctx = false;                   // SDC_ROCTX set at sdc_init: roctx ranges around the phases
    bool debug_poison = false;            // sdc_debug_poison: NaN-fill workspaces before their writers
    bool poison_now = false;              // inside enqueue_step with debug_poison on
    sdc_config cfg{};
    hipStream_t st = nullptr;
    Geom g{};
    FFTPlan plan{};
    double phibar = 0, inv_a2 = 0, two_omega = 0;
    double two_omega_explicit = 0;    // f in the explicit products (0 when L_c is implicit)
    double2* lc = nullptr;            // implicit_coriolis: (e-_k, e+_k) per coefficient
    double2* lc_scratch = nullptr;    // implicit_coriolis: elimination coefficients of the chains
    double* lc_beta = nullptr;        // implicit_coriolis: right-hand sides of the node updates
    std::vector<void*> allocs;
    long long bytes = 0, table_bytes = 0;
    double *mu = nullptr, *w = nullptr, *P = nullptr, *H = nullptr, *tau = nullptr, *Q = nullptr;
    double *rc = nullptr, *sect = nullptr;  // Legendre recurrence coefficients, sectoral values
    float *P32 = nullptr, *H32 = nullptr;   // FP32 copies of the tables (FP32 and BF16x3 modes)
    double *inv_lap = nullptr, *neg_lap = nullptr;
    long long* toff = nullptr;
    int* rowoff = nullptr;
    int* n_of = nullptr;
    int* m_of = nullptr;
    double2* tw = nullptr;
    // the same for 1, 2, 3, 4, 6 latitude tiles per workgroup
    static constexpr int kTileCounts[5] = {1, 2, 3, 4, 6};
    int2* syn_tasks_t[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int n_syn_t[5] = {0, 0, 0, 0, 0};
    // Legendre launch variants (defaults or sdc_autotune), per launch shape: lplan for launches
    // over the node states of a sweep (batch x M states), lplan1 for launches over one state per
    // member (a step's first f_E, eval_explicit, the comparison integrators, the adjoint's first
    // stage).  fuse_update and node_launch belong to the step and are read from lplan only.
    LegPlan lplan{};
    LegPlan lplan1{};
    int4* ana_tasks = nullptr;        // SWE analysis: 4 wave tasks per workgroup (XCD-ordered)
    int n_ana_wg = 0;
    int2* ssyn_tasks = nullptr;       // scalar synthesis (m, latitude group)
    int n_ssyn = 0;
    int4* sana_tasks = nullptr;       // scalar analysis wave tasks
    int n_sana = 0;
    double *ua = nullptr, *ub = nullptr, *E = nullptr, *E0 = nullptr;
    // captured steps: (state, dt, M, K) -> executable graph, replayed on st
    struct GraphEntry {
        int kind;                     // 0: dSDC step, 1: IMEX-o2 step, 2: sequential IMEX SDC
        const double* state;
        double dt;
        int M, K;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    hipStream_t cap = nullptr;        // private stream used only for capture
    std::vector<GraphEntry> graphs;
    // adjoint workspaces (allocated by the first sdc_step_adjoint call)
    bool adj_ready = false;
    double2* adj_save = nullptr;      // stage grid fields [stage states][4][nh][nlon] (N, S)
    double2* adj_four5 = nullptr;     // adjoint Fourier fields [S][5][nlat][m]
    double* adj_ubar = nullptr;       // node adjoints of the current sweep [B][M][3][ncoef]
    double* adj_ebar = nullptr;       // tendency adjoints [B][M][3][ncoef]
    double* adj_un = nullptr;         // u_n adjoint [B][3][ncoef]
    double* adj_x = nullptr;          // copy of u_n for the recomputation
    // IMEX-o2 workspaces (allocated by the first imex2_step call): u*, k1, k2 per member
    double *i2_ustar = nullptr, *i2_k1 = nullptr, *i2_k2 = nullptr;
    // device address of the library's scratch array on this handle's device (imex2_step_noalloc)
    int dev = -1;
    double* scratch_dev = nullptr;
    hipError_t scratch_err = hipSuccess;
    // sequential IMEX SDC workspaces (first sdc_step_sequential call): nodes and tendencies of
    // two sweeps, node-major [M][B][3][ncoef]
    double* seq_u[2] = {nullptr, nullptr};
    double* seq_e[2] = {nullptr, nullptr};
    double* cml = nullptr;            // synthesis input, coefficient-major
    double* G = nullptr;              // analysis input (also the scalar analysis input)
    double2* four = nullptr;
    int* flag = nullptr;
    int smax = 0;
    std::vector<long long> h_toff;
    // benchmark timing: event pairs per kernel class (pool reused between enables)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<size_t, size_t>> ev_marks[SDC_KERNEL_CLASSES];

    hipEvent_t next_event() {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    // record a start event before a launch of class k; returns the pool index (or -1)
    long begin(int k) {
        if (!timing) return -1;
        hipEvent_t e = next_event();
        if (!e) return -1;
        (void)hipEventRecord(e, st);
        (void)k;
        return (long)(ev_used - 1);
    }
    void end(int k, long start) {
        if (start < 0) return;
        hipEvent_t e = next_event();
        if (!e) return;
        (void)hipEventRecord(e, st);
        ev_marks[k].push_back({(size_t)start, ev_used - 1});
    }
    // SWE synthesis workgroups (XCD-ordered) for the plan's latitude tiles per workgroup
    static int tiles_index(int jt) {
        for (int k = 0; k < 5; ++k)
            if (kTileCounts[k] == jt) return k;
        return 0;
    }
    const LegPlan& plan_for(int S) const { return (cfg.M > 1 && S <= cfg.batch) ? lplan1 : lplan; }
    const int2* syn_list(const LegPlan& lp) const { return syn_tasks_t[tiles_index(lp.syn_tiles)]; }
    int syn_count(const LegPlan& lp) const { return n_syn_t[tiles_index(lp.syn_tiles)]; }
    void drop_graphs() {
        for (auto& ge : graphs) {
            (void)hipGraphExecDestroy(ge.exec);
            (void)hipGraphDestroy(ge.graph);
        }
        graphs.clear();
    }
    void reset_timing() {
        ev_used = 0;
        for (auto& v : ev_marks) v.clear();
    }

    Tables tables() const {
        return Tables{P, H, P32, H32, cfg.precision == SDC_BF16X3_MFMA ? 1 : 0, rc, sect, mu, inv_lap};
    }
    // the Legendre operand type of the handle's kernels (kTabF64, kTabF32, kTabBf3)
    int table_type() const {
        return cfg.precision == SDC_BF16X3_MFMA ? kTabBf3 : (cfg.precision == SDC_FP32_MFMA ? kTabF32 : kTabF64);
    }

    template <typename T>
    int alloc(T*& p, size_t count, bool table = false) {
        void* q = nullptr;
        const size_t nb = count * sizeof(T);
        if (hipMalloc(&q, nb) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SDC_ENOMEM, "device allocation of %zu bytes failed", nb);
        }
        allocs.push_back(q);
        bytes += (long long)nb;
        if (table) table_bytes += (long long)nb;
        if (hipMemset(q, 0, nb) != hipSuccess) return fail(SDC_EHIP, "hipMemset failed");
        p = static_cast<T*>(q);
        return SDC_OK;
    }
    ~sdc_ctx() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (void* p : allocs) (void)hipFree(p);
    }
};

namespace {

int validate_config(const sdc_config* c) {
    if (!c) return fail(SDC_EINVAL, "cfg is NULL");
    if (c->T < 1 || c->T > 1023) return fail(SDC_EINVAL, "T=%d out of range 1..1023", c->T);
    if (c->nlat < c->T + 1) return fail(SDC_EINVAL, "nlat=%d < T+1", c->nlat);
    if (c->nlat % 2 != 0) return fail(SDC_EINVAL, "nlat=%d must be even", c->nlat);
    if (c->nlon < 2 * c->T + 1) return fail(SDC_EINVAL, "nlon=%d < 2T+1", c->nlon);
    if (!(c->radius > 0) || !std::isfinite(c->radius)) return fail(SDC_EINVAL, "radius must be > 0");
    if (!(c->gravity > 0) || !std::isfinite(c->gravity)) return fail(SDC_EINVAL, "gravity must be > 0");
    if (!std::isfinite(c->omega)) return fail(SDC_EINVAL, "omega must be finite");
    if (!(c->mean_depth > 0) || !std::isfinite(c->mean_depth)) return fail(SDC_EINVAL, "mean_depth must be > 0");
    if (c->M < 1 || c->M > kMaxNodes) return fail(SDC_EINVAL, "M=%d out of range 1..%d", c->M, kMaxNodes);
    if (c->K < 1 || c->K > kMaxSweeps) return fail(SDC_EINVAL, "K=%d out of range 1..%d", c->K, kMaxSweeps);
    if (c->nodes != 0) return fail(SDC_EINVAL, "nodes=%d: only Radau-right (0) is defined", c->nodes);
    if (c->qdelta < 0 || c->qdelta > 2)
        return fail(SDC_EINVAL, "qdelta=%d: MIN-SR-FLEX (0), MIN-SR-NS (1) or parallel implicit Euler (2)",
                    c->qdelta);
    if (c->precision < SDC_FP64 || c->precision > SDC_BF16X3_MFMA)
        return fail(SDC_EINVAL, "precision=%d unknown", c->precision);
    if (c->batch < 1 || c->batch > 4096) return fail(SDC_EINVAL, "batch=%d out of range 1..4096", c->batch);
    if (c->implicit_coriolis != 0 && c->implicit_coriolis != 1)
        return fail(SDC_EINVAL, "implicit_coriolis=%d: 0 or 1", c->implicit_coriolis);
    if (c->nlon > 2048) return fail(SDC_EUNSUPPORTED, "nlon=%d > 2048 is not supported", c->nlon);
    FFTPlan pl;
    if (!make_fft_plan(c->nlon, pl) || !fft_length_supported(c->nlon))
        return fail(SDC_EUNSUPPORTED, "nlon=%d is not one of 16..2048 = 2^p or 24..1536 = 3*2^p", c->nlon);
    return SDC_OK;
}

int setup(sdc_ctx* c) {
    const sdc_config& cf = c->cfg;
    Geom& g = c->g;
    g.T = cf.T;
    g.nlat = cf.nlat;
    g.nlon = cf.nlon;
    g.nh = cf.nlat / 2;
    g.nhp = (g.nh + 15) / 16 * 16;
    g.ms = cf.T + 1;
    g.ncoef = (cf.T + 1) * (cf.T + 2) / 2;
    g.radius = cf.radius;
    make_fft_plan(cf.nlon, c->plan);
    c->phibar = cf.gravity * cf.mean_depth;
    c->inv_a2 = 1.0 / (cf.radius * cf.radius);
    c->two_omega = 2.0 * cf.omega;
    c->two_omega_explicit = cf.implicit_coriolis ? 0.0 : c->two_omega;
    c->smax = cf.batch * cf.M;
    int rc;

    // packed Legendre layout
    c->h_toff.assign(2 * (g.T + 1), 0);
    std::vector<int> h_rowoff(2 * (g.T + 1), 0);
    long long tot = 0;
    int rows = 0;
    for (int m = 0; m <= g.T; ++m)
        for (int p = 0; p < 2; ++p) {
            c->h_toff[2 * m + p] = tot;
            h_rowoff[2 * m + p] = rows;
            const int np4 = (npk_of(g.T, m, p) + 3) & ~3;
            tot += (long long)np4 * g.nhp;
            rows += np4;
        }
    g.nrows = rows;
    if ((rc = c->alloc(c->mu, g.nlat))) return rc;
    if ((rc = c->alloc(c->w, g.nlat))) return rc;
    if ((rc = c->alloc(c->P, tot, true))) return rc;
    if ((rc = c->alloc(c->H, tot, true))) return rc;
    if ((rc = c->alloc(c->rc, (size_t)4 * (g.T + 1) * (g.T + kRecPad)))) return rc;
    if ((rc = c->alloc(c->sect, (size_t)(g.T + 1) * g.nhp))) return rc;
    if ((rc = c->alloc(c->toff, c->h_toff.size()))) return rc;
    if ((rc = c->alloc(c->rowoff, h_rowoff.size()))) return rc;
    if ((rc = c->alloc(c->n_of, g.ncoef))) return rc;
    if ((rc = c->alloc(c->m_of, g.ncoef))) return rc;
    if ((rc = c->alloc(c->inv_lap, g.T + 1))) return rc;
    if ((rc = c->alloc(c->neg_lap, g.T + 1))) return rc;
    if ((rc = c->alloc(c->tau, (kMaxNodes + 1) * kMaxNodes))) return rc;
    if ((rc = c->alloc(c->Q, (kMaxNodes + 1) * kMaxNodes * kMaxNodes))) return rc;
    if ((rc = c->alloc(c->tw, cf.nlon))) return rc;
    if ((rc = c->alloc(c->flag, 4))) return rc;

    // task lists.  SWE synthesis: (m, 16-latitude tile) per workgroup of two waves (one per
    // parity).  SWE analysis: (m, parity, first of four 16-row tiles) per workgroup.  Both are
    // grouped per block of 8 orders on one XCD (the partial output lines of neighbouring orders
    // meet in that L2) and issued longest first.
    const int ntj = g.nhp / 16, njg = (ntj + 3) / 4;
    for (int jt_per : sdc_ctx::kTileCounts) {
        std::vector<int2> t;
        std::vector<int> grp;
        std::vector<double> wk;
        for (int m = 0; m <= g.T; ++m)
            for (int jt = 0; jt < ntj; jt += jt_per) {
                t.push_back(make_int2(m, jt));
                grp.push_back(m / 8);
                const int tiles = ntj - jt < jt_per ? ntj - jt : jt_per;
                wk.push_back((double)((npk_of(g.T, m, 0) + 3) / 4) * tiles + 4.0);
            }
        std::vector<int2> ord = xcd_order(t, grp, wk, make_int2(-1, 0));
        int2*& dst = c->syn_tasks_t[sdc_ctx::tiles_index(jt_per)];
        c->n_syn_t[sdc_ctx::tiles_index(jt_per)] = (int)ord.size();
        if ((rc = c->alloc(dst, ord.size()))) return rc;
        HIP_TRY(hipMemcpy(dst, ord.data(), ord.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    {
        std::vector<int4> t, sw;
        std::vector<int> grp;
        std::vector<double> wk;
        for (int m = 0; m <= g.T; ++m)
            for (int p = 0; p < 2; ++p) {
                const int np = npk_of(g.T, m, p);
                for (int kk = 0; kk < np; kk += 64) {
                    t.push_back(make_int4(m, p, kk, 1));
                    grp.push_back(m / 8);
                    wk.push_back((double)((np - kk < 64 ? np - kk : 64) + 15) / 16.0 + 0.5);
                }
                for (int kk = 0; kk < np; kk += 16) sw.push_back(make_int4(m, p, kk, 0));
            }
        std::vector<int4> ord = xcd_order(t, grp, wk, make_int4(0, 0, 0, 0));
        c->n_ana_wg = (int)ord.size();
        if ((rc = c->alloc(c->ana_tasks, ord.size()))) return rc;
        HIP_TRY(hipMemcpy(c->ana_tasks, ord.data(), ord.size() * sizeof(int4), hipMemcpyHostToDevice));
        c->n_sana = (int)sw.size();
        if ((rc = c->alloc(c->sana_tasks, sw.size()))) return rc;
        HIP_TRY(hipMemcpy(c->sana_tasks, sw.data(), sw.size() * sizeof(int4), hipMemcpyHostToDevice));
    }
    {
        std::vector<int2> ss;
        for (int m = 0; m <= g.T; ++m)
            for (int jg = 0; jg < njg; ++jg) ss.push_back(make_int2(m, jg));
        c->n_ssyn = (int)ss.size();
        if ((rc = c->alloc(c->ssyn_tasks, ss.size()))) return rc;
        HIP_TRY(hipMemcpy(c->ssyn_tasks, ss.data(), ss.size() * sizeof(int2), hipMemcpyHostToDevice));
    }

    // workspaces
    const size_t st_d = (size_t)3 * g.ncoef * 2;
    if ((rc = c->alloc(c->ua, st_d * c->smax))) return rc;
    if ((rc = c->alloc(c->ub, st_d * c->smax))) return rc;
    if ((rc = c->alloc(c->E, st_d * c->smax))) return rc;
    if ((rc = c->alloc(c->E0, st_d * cf.batch))) return rc;
    if ((rc = c->alloc(c->cml, (size_t)g.nrows * c->smax * kCmlVals))) return rc;
    if ((rc = c->alloc(c->four, (size_t)c->smax * kSynFields * g.nlat * g.ms))) return rc;
    if ((rc = c->alloc(c->G, (size_t)(g.T + 1) * 2 * g.nhp * c->smax * kAnaStride))) return rc;

    // host-computed index data and twiddles e^{-2 pi i k/nlon} (long double, rounded once)
    std::vector<double2> tw(cf.nlon);
    for (int k = 0; k < cf.nlon; ++k) {
        const long double ang = -2.0L * 3.141592653589793238462643383279502884L * k / cf.nlon;
        tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    HIP_TRY(hipMemcpy(c->tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->toff, c->h_toff.data(), c->h_toff.size() * sizeof(long long), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->rowoff, h_rowoff.data(), h_rowoff.size() * sizeof(int), hipMemcpyHostToDevice));

    // FP64 setup kernels
    launch_gauss(c->mu, c->w, g.nlat, c->st);
    launch_rec_coefs(c->rc, g, c->st);
    launch_legendre_tables(c->mu, c->rc, c->P, c->H, c->sect, c->toff, g, c->st);
    if (cf.precision != SDC_FP64) {
        // FP32 copies of the FP64 tables for the Legendre contractions (FP32 and BF16x3 modes)
        if ((rc = c->alloc(c->P32, tot, true))) return rc;
        if ((rc = c->alloc(c->H32, tot, true))) return rc;
        launch_round_tables(c->P, c->H, c->P32, c->H32, tot, c->st);
    }
    launch_collocation(c->tau, c->Q, cf.M, c->st);
    launch_degree_tables(c->n_of, c->m_of, c->inv_lap, c->neg_lap, g.T, g.radius, c->st);
    if (cf.implicit_coriolis) {
        if ((rc = c->alloc(c->lc, g.ncoef))) return rc;
        if ((rc = c->alloc(c->lc_scratch, (size_t)c->smax * 2 * 3 * g.ncoef))) return rc;
        if ((rc = c->alloc(c->lc_beta, (size_t)c->smax * 3 * g.ncoef * 2))) return rc;
        launch_lc_coefs(c->lc, c->n_of, c->m_of, g.ncoef, c->st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->st));

    const size_t lds = (size_t)4 * cf.nlon * sizeof(double2);      // four signals per grid workgroup
    if (lds > 65536) HIP_TRY(grid_set_lds_limit(cf.nlon, lds));
    return SDC_OK;
}

// Host-side roctx range (rocprofv3 --marker-trace) around the enqueue of one phase when the
// handle was created with SDC_ROCTX set; under graph capture it marks the capture.
struct PhaseRange {
    bool on;
    PhaseRange(const sdc_ctx* c, const char* name) : on(c->roctx && !c->rec) {
        if (on) roctxRangePushA(name);
    }
    ~PhaseRange() {
        if (on) roctxRangePop();
    }
};

// f_E of S states whose synthesis input is already in c->cml (written by the update kernels), or,
// with states != null, read by the synthesis from the state layout.
void run_explicit_cml(sdc_ctx* c, int S, double* out, double2* save = nullptr,
                      const UpdateArgs* fuse = nullptr, int fuse_mode = 0, const double* states = nullptr) {
    if (c->rec) {
        c->rec->push_back(StepOp{0, S, states, out, save, fuse ? *fuse : UpdateArgs{}, fuse ? fuse_mode : 0});
        return;
    }
    const PhaseRange range(c, fuse ? "sdc.f_E+update" : "sdc.f_E");
    const LegPlan& lp = c->plan_for(S);
    const size_t tb = c->P32 ? sizeof(float) : sizeof(double);
    if (c->poison_now)
        launch_poison(c->four, (size_t)S * kSynFields * c->g.nlat * c->g.ms * sizeof(double2), c->st);
    long t = c->begin(SDC_KERNEL_SYNTHESIS);
    launch_synthesis_swe(c->tables(), lp, c->toff, c->rowoff, c->syn_list(lp), c->syn_count(lp),
                         c->cml, S, c->four, c->g, c->st, states);
    c->end(SDC_KERNEL_SYNTHESIS, t);
    if (c->poison_now)
        launch_poison(c->G, (size_t)c->g.nh * (c->g.T + 1) * S * 2 * kFwdVals * tb, c->st);
    t = c->begin(SDC_KERNEL_GRID);
    launch_grid_swe(c->four, c->G, c->P32 != nullptr, c->mu, c->w, c->tw, c->plan, S, c->two_omega_explicit, save,
                    c->g, c->st);
    c->end(SDC_KERNEL_GRID, t);
    if (c->poison_now) {
        const size_t st_b = (size_t)3 * c->g.ncoef * 2 * sizeof(double);
        if (!fuse) launch_poison(out, (size_t)S * st_b, c->st);          // the tendencies
        if (fuse && !fuse->last_only)                                     // the updated nodes
            launch_poison(fuse->uout, (size_t)fuse->batch * fuse->M * st_b, c->st);
    }
    t = c->begin(SDC_KERNEL_ANALYSIS);
    launch_analysis_swe(c->tables(), lp, c->toff, c->ana_tasks, c->n_ana_wg, c->G, S, c->neg_lap,
                        out, c->g, c->st, fuse, fuse_mode);
    c->end(SDC_KERNEL_ANALYSIS, t);
}

// f_E of S states in the state layout (every synthesis variant reads them in place).
void run_explicit(sdc_ctx* c, const double* states, int S, double* out, double2* save = nullptr,
                  const UpdateArgs* fuse = nullptr, int fuse_mode = 0) {
    run_explicit_cml(c, S, out, save, fuse, fuse_mode, states);
}

// out_acc += J_E(u)^T ebar for S states whose stage grid fields are in `save`.
// Transposed tendency of S states: ebar -> synthesis-adjoint layout (skipped when an earlier fused
// epilogue wrote that layout already), then synthesis^T, products'^T, analysis^T accumulated into
// out_acc (or, with fuse, consumed by the analysis epilogue).
void run_explicit_adj(sdc_ctx* c, const double* ebar, int S, const double2* save, double* out_acc,
                      const AdjFuse* fuse = nullptr, bool cml_ready = false) {
    if (!cml_ready)
        launch_prep_cml_adj(ebar, S, c->cml, c->P32 != nullptr, c->n_of, c->m_of, c->rowoff, c->neg_lap, c->g.ncoef,
                            c->g.T, c->st);
    const LegPlan& lp = c->plan_for(S);
    launch_synthesis_adj(c->tables(), lp, c->toff, c->rowoff, c->syn_list(lp), c->syn_count(lp),
                         c->cml, S, c->adj_four5, c->g, c->st);
    launch_grid_adj(c->adj_four5, save, c->G, c->P32 != nullptr, c->mu, c->w, c->tw, c->plan, S, c->two_omega, c->g, c->st);
    launch_analysis_adjoint(c->tables(), lp, c->toff, c->ana_tasks, c->n_ana_wg, c->G, S,
                            c->inv_lap, out_acc, c->g, c->st, fuse);
}

size_t stage_states(const sdc_ctx* c, int s, int M) {     // states stored before stage s
    return s == 0 ? 0 : (size_t)c->cfg.batch + (size_t)(s - 1) * c->cfg.batch * M;
}

// Adjoint workspaces (first adjoint call); the stage grid fields of the recomputing adjoint only
// when `with_save` (the taped adjoint reads them from the caller's tape).
int alloc_adjoint(sdc_ctx* c, bool with_save) {
    const Geom& g = c->g;
    const size_t B = c->cfg.batch;
    const size_t st_d = (size_t)3 * g.ncoef * 2;
    int rc;
    if (!c->adj_ready) {
        if ((rc = c->alloc(c->adj_four5, (size_t)c->smax * 5 * g.nlat * g.ms))) return rc;
        if ((rc = c->alloc(c->adj_ubar, st_d * c->smax))) return rc;
        if ((rc = c->alloc(c->adj_ebar, st_d * c->smax))) return rc;
        if ((rc = c->alloc(c->adj_un, st_d * B))) return rc;
        if ((rc = c->alloc(c->adj_x, st_d * B))) return rc;
        c->adj_ready = true;
    }
    if (with_save && !c->adj_save) {
        const size_t nst = B + (size_t)(c->cfg.K > 1 ? c->cfg.K - 1 : 0) * B * c->cfg.M;
        if ((rc = c->alloc(c->adj_save, nst * kSynFields * g.nh * g.nlon))) return rc;
    }
    return SDC_OK;
}

// Stage grid fields per state in a tape: zeta, Phi', U, V as (north, south) pairs.
size_t tape_per_state(const sdc_ctx* c) { return (size_t)kSynFields * c->g.nh * c->g.nlon; }

void run_update(sdc_ctx* c, const UpdateArgs& a) {
    if (c->rec) {
        c->rec->push_back(StepOp{1, 0, nullptr, nullptr, nullptr, a, 0});
        return;
    }
    const PhaseRange range(c, "sdc.update");
    if (c->poison_now && !a.last_only) {
        const size_t st_b = (size_t)3 * c->g.ncoef * 2 * sizeof(double);
        launch_poison(a.uout, (size_t)a.batch * a.M * st_b, c->st);
    }
    const long t = c->begin(SDC_KERNEL_UPDATE);
    launch_update(a, c->st);
    c->end(SDC_KERNEL_UPDATE, t);
}

int check_handle(sdc_handle h) {
    if (!h) return fail(SDC_EINVAL, "handle is NULL");
    return SDC_OK;
}

}  // namespace

extern "C" {

const char* sdc_last_error(void) { return g_last_error.c_str(); }

int sdc_init(const sdc_config* cfg, void* hip_stream, sdc_handle* out) {
    g_last_error.clear();
    if (!out) return fail(SDC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc) return rc;
    sdc_ctx* c = new (std::nothrow) sdc_ctx();
    if (!c) return fail(SDC_ENOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->st = static_cast<hipStream_t>(hip_stream);
    rc = setup(c);
    if (rc) {
        (void)hipStreamSynchronize(c->st);
        delete c;
        return rc;
    }
    if (const char* e = std::getenv("SDC_ROCTX")) c->roctx = e[0] != '\0' && std::strcmp(e, "0") != 0;
    // the scratch array's address on this device (the device current at init owns the handle)
    if (hipGetDevice(&c->dev) == hipSuccess) {
        c->scratch_dev = scratch_address(c->dev, &c->scratch_err);
    } else {
        (void)hipGetLastError();
        c->scratch_err = hipErrorInvalidDevice;
    }
    *out = c;
    return SDC_OK;
}

int sdc_free(sdc_handle h) {
    if (!h) return SDC_OK;
    (void)hipStreamSynchronize(h->st);
    delete h;
    return SDC_OK;
}

int sdc_get_info(sdc_handle h, sdc_info* info) {
    if (int rc = check_handle(h)) return rc;
    if (!info) return fail(SDC_EINVAL, "info is NULL");
    info->T = h->g.T;
    info->nlat = h->g.nlat;
    info->nlon = h->g.nlon;
    info->ncoef = h->g.ncoef;
    info->M = h->cfg.M;
    info->K = h->cfg.K;
    info->batch = h->cfg.batch;
    info->precision = h->cfg.precision;
    info->device_bytes = h->bytes;
    info->table_bytes = h->table_bytes;
    return SDC_OK;
}

}  // extern "C"

namespace {

void plan_out(const LegPlan& lp, const LegPlan& step, sdc_plan* plan) {
    plan->syn_lat_tiles = lp.syn_tiles;
    plan->syn_depth = lp.syn_depth;
    plan->ana_depth = lp.ana_depth;
    plan->ana_interleave = lp.ana_interleave;
    plan->syn_recur = lp.syn_recur;
    plan->ana_recur = lp.ana_recur;
    plan->fuse_update = step.fuse_update;
    plan->node_launch = step.node_launch;
}

int check_plan(sdc_handle h, const sdc_plan* plan) {
    if (!plan) return fail(SDC_EINVAL, "plan is NULL");
    if (plan->fuse_update != 0 && plan->fuse_update != 1)
        return fail(SDC_EINVAL, "fuse_update=%d: 0 or 1", plan->fuse_update);
    if (plan->syn_recur != 0 && plan->syn_recur != 1)
        return fail(SDC_EINVAL, "syn_recur=%d: 0 or 1", plan->syn_recur);
    if (plan->ana_recur != 0 && plan->ana_recur != 1)
        return fail(SDC_EINVAL, "ana_recur=%d: 0 or 1", plan->ana_recur);
    if (plan->node_launch != 0 && plan->node_launch != 1)
        return fail(SDC_EINVAL, "node_launch=%d: 0 or 1", plan->node_launch);
    if (plan->node_launch && h->cfg.batch != 1)
        return fail(SDC_EINVAL, "node_launch=1 is defined for handles of one member (batch=%d)", h->cfg.batch);
    if (plan->node_launch && h->cfg.implicit_coriolis)
        return fail(SDC_EUNSUPPORTED, "node_launch=1 is built for the split with f_I = L_g");
    const int jt = plan->syn_lat_tiles, d = plan->syn_depth;
    const bool syn_ok = (jt == 1 && (d == 8 || d == 4)) || (jt == 2 && (d == 4 || d == 2)) ||
                        (jt == 3 && d == 2) || (jt == 4 && (d == 2 || d == 1)) || (jt == 6 && d == 1);
    if (!syn_ok)
        return fail(SDC_EINVAL, "synthesis variant (%d tiles, depth %d) not built: use (1, 8), (1, 4), (2, 4), "
                    "(2, 2), (3, 2), (4, 2), (4, 1) or (6, 1)", jt, d);
    if (plan->syn_recur && (jt == 3 || jt == 6))
        return fail(SDC_EINVAL, "the regenerating synthesis (syn_recur) is built for 1, 2 or 4 latitude tiles");
    if ((plan->ana_depth != 2 && plan->ana_depth != 4) || (plan->ana_interleave != 0 && plan->ana_interleave != 1))
        return fail(SDC_EINVAL, "analysis variant (depth %d, interleave %d) not built: depth 2 or 4, interleave 0 or 1",
                    plan->ana_depth, plan->ana_interleave);
    return SDC_OK;
}

void plan_in(const sdc_plan* plan, LegPlan& lp) {
    lp.syn_tiles = plan->syn_lat_tiles;
    lp.syn_depth = plan->syn_depth;
    lp.ana_depth = plan->ana_depth;
    lp.ana_interleave = plan->ana_interleave;
    lp.syn_recur = plan->syn_recur;
    lp.ana_recur = plan->ana_recur;
    lp.fuse_update = plan->fuse_update;
    lp.node_launch = plan->node_launch;
}

// the plan of launches over `states` states per member: 1 or the configured M
LegPlan* plan_of(sdc_handle h, int states) {
    if (states == h->cfg.M) return &h->lplan;
    if (states == 1) return &h->lplan1;
    return nullptr;
}

}  // namespace

extern "C" {

int sdc_get_plan(sdc_handle h, sdc_plan* plan) {
    if (int rc = check_handle(h)) return rc;
    if (!plan) return fail(SDC_EINVAL, "plan is NULL");
    plan_out(h->lplan, h->lplan, plan);
    return SDC_OK;
}

int sdc_set_plan(sdc_handle h, const sdc_plan* plan) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = check_plan(h, plan)) return rc;
    plan_in(plan, h->lplan);
    plan_in(plan, h->lplan1);
    h->drop_graphs();                 // recaptured with the new variants on their next replay
    return SDC_OK;
}

int sdc_get_plan_for(sdc_handle h, int states, sdc_plan* plan) {
    if (int rc = check_handle(h)) return rc;
    if (!plan) return fail(SDC_EINVAL, "plan is NULL");
    const LegPlan* lp = plan_of(h, states);
    if (!lp) return fail(SDC_EINVAL, "states=%d: 1 or the configured M=%d", states, h->cfg.M);
    plan_out(h->cfg.M > 1 ? *lp : h->lplan, h->lplan, plan);
    return SDC_OK;
}

int sdc_set_plan_for(sdc_handle h, int states, const sdc_plan* plan) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = check_plan(h, plan)) return rc;
    LegPlan* lp = plan_of(h, states);
    if (!lp) return fail(SDC_EINVAL, "states=%d: 1 or the configured M=%d", states, h->cfg.M);
    if (h->cfg.M == 1) {              // one launch shape: both plans are the same
        plan_in(plan, h->lplan);
        plan_in(plan, h->lplan1);
    } else {
        plan_in(plan, *lp);
        // the step's fields live in lplan
        h->lplan.fuse_update = plan->fuse_update;
        h->lplan.node_launch = plan->node_launch;
        h->lplan1.fuse_update = plan->fuse_update;
        h->lplan1.node_launch = plan->node_launch;
    }
    h->drop_graphs();
    return SDC_OK;
}

int sdc_autotune(sdc_handle h, int reps, sdc_plan* chosen) {
    if (int rc = check_handle(h)) return rc;
    if (reps < 1 || reps > 1000) return fail(SDC_EINVAL, "reps = %d outside [1, 1000]", reps);
    sdc_ctx* c = h;
    // the launch shape that dominates a step: every node state of every member at once
    const int S = c->cfg.batch * c->cfg.M;
    // finite operands for every candidate (the buffers are workspaces every step rewrites)
    HIP_TRY(hipMemsetAsync(c->ua, 0, (size_t)c->smax * 3 * c->g.ncoef * 2 * sizeof(double), c->st));
    HIP_TRY(hipMemsetAsync(c->cml, 0, (size_t)c->g.nrows * c->smax * kCmlVals * sizeof(double), c->st));
    HIP_TRY(hipMemsetAsync(c->G, 0, (size_t)(c->g.T + 1) * 2 * c->g.nhp * c->smax * kAnaStride * sizeof(double),
                           c->st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SDC_EHIP, "hipEventCreate failed");
    }
    auto time_it = [&](auto&& launch, float& ms) -> hipError_t {
        launch();                                        // warm-up (code objects, caches)
        hipError_t e = hipEventRecord(e0, c->st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, c->st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipGetLastError();
        return e;
    };
    // a candidate replaces the current variant only when it is at least 5 % faster (timing noise
    // and near-ties do not flip the choice)
    constexpr float kMargin = 0.95f;
    constexpr int kSyn = 14;
    const int shapes[kSyn][3] = {{1, 8, 0}, {1, 4, 0}, {2, 4, 0}, {2, 2, 0}, {3, 2, 0},
                                 {4, 2, 0}, {4, 1, 0}, {6, 1, 0}, {1, 8, 1}, {1, 4, 1},
                                 {2, 4, 1}, {2, 2, 1}, {4, 2, 1}, {4, 1, 1}};
    constexpr int kAna = 8;                 // depth 4 / 2 x interleave 1 / 0 x read / regenerate
    hipError_t err = hipSuccess;
    // Times every synthesis and analysis variant at S states and returns `cur` with the fastest
    // of each (the synthesis reads the states in place, as every f_E of a step does).
    auto tune = [&](const LegPlan& cur, int S, const double* state_in) {
        LegPlan syn_cands[kSyn], ana_cands[kAna];
        for (int k = 0; k < kSyn; ++k) {
            syn_cands[k] = cur;
            syn_cands[k].syn_tiles = shapes[k][0];
            syn_cands[k].syn_depth = shapes[k][1];
            syn_cands[k].syn_recur = shapes[k][2];
        }
        for (int k = 0; k < kAna; ++k) {
            ana_cands[k] = cur;
            ana_cands[k].ana_depth = (k & 2) ? 2 : 4;
            ana_cands[k].ana_interleave = (k & 1) ? 0 : 1;
            ana_cands[k].ana_recur = k >> 2;
        }
        float syn_ms[kSyn] = {0.f}, ana_ms[kAna] = {0.f};
        for (int k = 0; k < kSyn && err == hipSuccess; ++k) {
            const LegPlan& lp = syn_cands[k];
            err = time_it([&] {
                launch_synthesis_swe(c->tables(), lp, c->toff, c->rowoff, c->syn_list(lp), c->syn_count(lp),
                                     c->cml, S, c->four, c->g, c->st, state_in);
            }, syn_ms[k]);
        }
        for (int k = 0; k < kAna && err == hipSuccess; ++k) {
            const LegPlan& lp = ana_cands[k];
            err = time_it([&] {
                launch_analysis_swe(c->tables(), lp, c->toff, c->ana_tasks, c->n_ana_wg, c->G, S, c->neg_lap,
                                    c->E, c->g, c->st);
            }, ana_ms[k]);
        }
        LegPlan best = cur;
        if (err != hipSuccess) return best;
        int now = 0, fast = 0;
        for (int k = 0; k < kSyn; ++k) {
            if (syn_cands[k].syn_tiles == cur.syn_tiles && syn_cands[k].syn_depth == cur.syn_depth &&
                syn_cands[k].syn_recur == cur.syn_recur)
                now = k;
            if (syn_ms[k] < syn_ms[fast]) fast = k;
        }
        if (syn_ms[fast] < kMargin * syn_ms[now]) {
            best.syn_tiles = syn_cands[fast].syn_tiles;
            best.syn_depth = syn_cands[fast].syn_depth;
            best.syn_recur = syn_cands[fast].syn_recur;
        }
        now = 0;
        fast = 0;
        for (int k = 0; k < kAna; ++k) {
            if (ana_cands[k].ana_depth == cur.ana_depth && ana_cands[k].ana_interleave == cur.ana_interleave &&
                ana_cands[k].ana_recur == cur.ana_recur)
                now = k;
            if (ana_ms[k] < ana_ms[fast]) fast = k;
        }
        if (ana_ms[fast] < kMargin * ana_ms[now]) {
            best.ana_depth = ana_cands[fast].ana_depth;
            best.ana_interleave = ana_cands[fast].ana_interleave;
            best.ana_recur = ana_cands[fast].ana_recur;
        }
        return best;
    };
    const LegPlan saved = c->lplan, saved1 = c->lplan1;
    LegPlan best = tune(saved, S, c->ua);
    // launches over one state per member (handles with more than one node): their own variants
    LegPlan best1 = c->cfg.M > 1 ? tune(saved1, c->cfg.batch, c->ua) : best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) {
        c->lplan = saved;
        c->lplan1 = saved1;
        return fail(SDC_EHIP, "autotune launch failed: %s", hipGetErrorString(err));
    }
    c->lplan = best;
    c->lplan1 = best1;
    c->lplan1.fuse_update = best.fuse_update;
    c->lplan1.node_launch = best.node_launch;
    c->drop_graphs();
    if (chosen) plan_out(best, best, chosen);
    return SDC_OK;
}

}  // extern "C"

namespace {

int check_step_args(sdc_handle h, const double* state, double dt, int M, int K) {
    if (int rc = check_handle(h)) return rc;
    if (!state) return fail(SDC_EINVAL, "state is NULL");
    if (M < 1 || M > h->cfg.M) return fail(SDC_EINVAL, "M=%d out of range 1..%d", M, h->cfg.M);
    if (K < 1 || K > h->cfg.K) return fail(SDC_EINVAL, "K=%d out of range 1..%d", K, h->cfg.K);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(SDC_EINVAL, "dt must be positive and finite");
    return SDC_OK;
}

// The update kernels form the diagonal coefficient of sweep s as tau_m / min(s, M)
// (MIN-SR-FLEX); MIN-SR-NS uses tau_m / M in every sweep, i.e. the kernels' s = M.
// The kernels take q_mm = tau_m / min(sweep, M): MIN-SR-FLEX passes the sweep, MIN-SR-NS M and
// parallel implicit Euler 1.
int qd_sweep(const sdc_ctx* c, int s, int M) { return c->cfg.qdelta == 1 ? M : (c->cfg.qdelta == 2 ? 1 : s); }

// Algorithm 2 for all members of the handle, enqueued on c->st (arguments already checked).
// With `tape`, the grid fields of every f_E evaluation are kept there (stage s at
// tape + stage_states(s) * tape_per_state); without `last_update` the final last-node update is
// skipped (the adjoint's recomputation needs only the stages).
void enqueue_step_impl(sdc_ctx* c, double* state, double dt, int M, int K, double2* tape,
                       bool last_update);

void enqueue_step(sdc_ctx* c, double* state, double dt, int M, int K, double2* tape = nullptr,
                  bool last_update = true) {
    c->poison_now = c->debug_poison && !c->rec;
    const PhaseRange range(c, "sdc.step");
    enqueue_step_impl(c, state, dt, M, K, tape, last_update);
    c->poison_now = false;
}

void enqueue_step_impl(sdc_ctx* c, double* state, double dt, int M, int K, double2* tape,
                       bool last_update) {
    const int B = c->cfg.batch;
    const long long fs = 3LL * c->g.ncoef * 2;
    auto tape_at = [&](int s) -> double2* {
        return tape ? tape + stage_states(c, s, M) * tape_per_state(c) : nullptr;
    };
    UpdateArgs a{};
    a.un = state;
    a.tau = c->tau + M * kMaxNodes;
    a.Q = c->Q + M * kMaxNodes * kMaxNodes;
    a.n_of = c->n_of;
    a.m_of = c->m_of;
    a.rowoff = c->rowoff;
    a.inv_lap = c->inv_lap;
    a.flag = c->flag;
    a.dt = dt;
    a.phibar = c->phibar;
    a.inv_a2 = c->inv_a2;
    a.M = M;
    a.batch = B;
    a.ncoef = c->g.ncoef;
    a.T = c->g.T;
    a.uprev = state;
    a.uprev_node = 0;
    a.uprev_member = fs;
    a.E = c->E0;
    a.E_node = 0;
    a.E_member = fs;
    double* bufs[2] = {c->ua, c->ub};
    int cur = 0;
    if (c->cfg.implicit_coriolis) {
        // f_I = L_g + L_c: every node update is a pair of tridiagonal chain solves per order
        // (the sweeps of Algorithm 2 are unchanged; f_E is N_a + N_r)
        LcArgs l{};
        l.mode = 0;
        l.un = state;
        l.uprev = state;
        l.uprev_node = 0;
        l.uprev_member = fs;
        l.E = c->E0;
        l.E_node = 0;
        l.E_member = fs;
        l.tau = c->tau + M * kMaxNodes;
        l.Q = c->Q + M * kMaxNodes * kMaxNodes;
        l.rowoff = c->rowoff;
        l.inv_lap = c->inv_lap;
        l.lc = c->lc;
        l.scratch = c->lc_scratch;
        l.beta_ws = c->lc_beta;
        l.n_of = c->n_of;
        l.m_of = c->m_of;
        l.flag = c->flag;
        l.dt = dt;
        l.phibar = c->phibar;
        l.inv_a2 = c->inv_a2;
        l.two_omega = c->two_omega;
        l.M = M;
        l.batch = B;
        l.ncoef = c->g.ncoef;
        l.T = c->g.T;
        auto solve = [&] {
            const long t = c->begin(SDC_KERNEL_UPDATE);
            launch_solve_lc(l, c->st);
            c->end(SDC_KERNEL_UPDATE, t);
        };
        run_explicit(c, state, B, c->E0, tape_at(0));
        for (int s = 1; s < K; ++s) {
            l.uout = bufs[cur];
            l.out_node = fs;
            l.out_member = (long long)M * fs;
            l.sweep = qd_sweep(c, s, M);
            l.last_only = 0;
            solve();
            run_explicit(c, bufs[cur], B * M, c->E, tape_at(s));
            l.uprev = bufs[cur];
            l.uprev_node = fs;
            l.uprev_member = (long long)M * fs;
            l.E = c->E;
            l.E_node = fs;
            l.E_member = (long long)M * fs;
            cur ^= 1;
        }
        if (!last_update) return;
        l.uout = state;
        l.out_node = 0;
        l.out_member = fs;
        l.sweep = qd_sweep(c, K, M);
        l.last_only = 1;
        solve();
        return;
    }
    if (c->lplan.node_launch) {
        // The same sweeps with the f_E of the nodes evaluated one node per launch (one member:
        // node j of a sweep is state j of the stage), after a separate update of all nodes: the
        // node loop run sequentially, as a code without the batched nodes would.  Every state's
        // transforms are independent of the others in a launch, so the result is bitwise the
        // batched step's.
        run_explicit(c, state, B, c->E0, tape_at(0));
        for (int s = 1; s < K; ++s) {
            a.uout = bufs[cur];
            a.out_node = fs;
            a.out_member = (long long)M * fs;
            a.sweep = qd_sweep(c, s, M);
            a.last_only = 0;
            run_update(c, a);
            for (int j = 0; j < M; ++j)
                run_explicit(c, bufs[cur] + j * fs, 1, c->E + j * fs,
                             tape ? tape_at(s) + (size_t)j * tape_per_state(c) : nullptr);
            a.uprev = bufs[cur];
            a.uprev_node = fs;
            a.uprev_member = (long long)M * fs;
            a.E = c->E;
            a.E_node = fs;
            a.E_member = (long long)M * fs;
            cur ^= 1;
        }
        if (!last_update) return;
        a.uout = state;
        a.out_node = 0;
        a.out_member = fs;
        a.sweep = qd_sweep(c, K, M);
        a.last_only = 1;
        run_update(c, a);
        return;
    }
    if (c->lplan.fuse_update && (M == 1 || M == 2 || M == 4)) {
        // The node update of sweep s + 1 runs inside the analysis of the f_E of sweep s (the
        // tendencies stay in the analysis workgroups): sweep s < K updates every node into
        // bufs[cur] and the synthesis input, sweep K node M into the state.
        auto set_update = [&](int s) {
            if (s < K) {
                a.uout = bufs[cur];
                a.out_node = fs;
                a.out_member = (long long)M * fs;
                a.last_only = 0;
            } else {
                a.uout = state;
                a.out_node = 0;
                a.out_member = fs;
                a.last_only = 1;
            }
            a.sweep = qd_sweep(c, s, M);
        };
        set_update(1);
        run_explicit(c, state, B, c->E0, tape_at(0), (K > 1 || last_update) ? &a : nullptr, 1);
        for (int s = 1; s < K; ++s) {
            a.uprev = bufs[cur];
            a.uprev_node = fs;
            a.uprev_member = (long long)M * fs;
            cur ^= 1;
            set_update(s + 1);
            run_explicit(c, a.uprev, B * M, c->E, tape_at(s), (s + 1 < K || last_update) ? &a : nullptr, 2);
        }
        return;
    }
    // sweep initialisation: E_0 = f_E(u_n); u_m^0 = u_n and E_m^0 = E_0 through node stride 0
    run_explicit(c, state, B, c->E0, tape_at(0));
    for (int s = 1; s < K; ++s) {
        a.uout = bufs[cur];
        a.out_node = fs;
        a.out_member = (long long)M * fs;
        a.sweep = qd_sweep(c, s, M);
        a.last_only = 0;
        run_update(c, a);
        run_explicit(c, bufs[cur], B * M, c->E, tape_at(s));
        a.uprev = bufs[cur];
        a.uprev_node = fs;
        a.uprev_member = (long long)M * fs;
        a.E = c->E;
        a.E_node = fs;
        a.E_member = (long long)M * fs;
        cur ^= 1;
    }
    if (!last_update) return;
    // last sweep: node M only, written into the state
    a.uout = state;
    a.out_node = 0;
    a.out_member = fs;
    a.sweep = qd_sweep(c, K, M);
    a.last_only = 1;
    run_update(c, a);
}

int alloc_imex2(sdc_ctx* c) {
    if (c->i2_ustar) return SDC_OK;
    const size_t n = (size_t)c->cfg.batch * 3 * c->g.ncoef * 2;
    int rc;
    if ((rc = c->alloc(c->i2_ustar, n))) return rc;
    if ((rc = c->alloc(c->i2_k1, n))) return rc;
    if ((rc = c->alloc(c->i2_k2, n))) return rc;
    return SDC_OK;
}

// One IMEX-o2 step for all members (workspaces allocated, arguments checked).
void enqueue_imex2(sdc_ctx* c, double* state, double dt, double* ustar, double* k1, double* k2) {
    const int B = c->cfg.batch;
    Imex2Args a{};
    a.cml32 = c->P32 != nullptr ? 1 : 0;       // synthesis input in the table type
    a.n_of = c->n_of;
    a.m_of = c->m_of;
    a.rowoff = c->rowoff;
    a.inv_lap = c->inv_lap;
    a.cml = c->cml;
    a.flag = c->flag;
    a.dt = dt;
    a.phibar = c->phibar;
    a.inv_a2 = c->inv_a2;
    a.batch = B;
    a.ncoef = c->g.ncoef;
    a.T = c->g.T;
    auto phase = [&](int ph, const double* in, double* out) {
        a.phase = ph;
        a.in = in;
        a.out = out;
        a.k1 = k1;
        a.k2 = k2;
        const long t = c->begin(SDC_KERNEL_UPDATE);
        launch_imex2(a, c->st);
        c->end(SDC_KERNEL_UPDATE, t);
    };
    phase(kImex2First, state, ustar);               // u* = C(dt/2) u_n
    run_explicit_cml(c, B, k1);                     // k1 = f_E(u*)
    phase(kImex2Predict, ustar, nullptr);           // synthesis input u* + dt k1
    run_explicit_cml(c, B, k2);                     // k2 = f_E(u* + dt k1)
    phase(kImex2Last, ustar, state);                // u_{n+1}
}

int alloc_seq(sdc_ctx* c) {
    if (c->seq_u[0]) return SDC_OK;
    const size_t n = (size_t)c->cfg.M * c->cfg.batch * 3 * c->g.ncoef * 2;
    int rc;
    for (int k = 0; k < 2; ++k) {
        if ((rc = c->alloc(c->seq_u[k], n))) return rc;
        if ((rc = c->alloc(c->seq_e[k], n))) return rc;
    }
    return SDC_OK;
}

// Algorithm 1 for all members: K sweeps of M sequential node updates, each followed by f_E of the
// new node (all members in one launch), except after the step's last update.
void enqueue_seq(sdc_ctx* c, double* state, double dt, int M, int K) {
    const int B = c->cfg.batch;
    const long long fsz = 3LL * c->g.ncoef * 2;     // doubles per state
    const long long nsn = (long long)B * fsz;       // node stride of the sweep buffers
    run_explicit(c, state, B, c->E0);              // E_0 = f_E(u_n)
    SeqArgs a{};
    a.cml32 = c->P32 != nullptr ? 1 : 0;       // synthesis input in the table type
    a.un = state;
    a.uold = state;
    a.uold_node = 0;
    a.eold = c->E0;
    a.eold_node = 0;
    a.n_of = c->n_of;
    a.m_of = c->m_of;
    a.rowoff = c->rowoff;
    a.inv_lap = c->inv_lap;
    a.tau = c->tau + M * kMaxNodes;
    a.Q = c->Q + M * kMaxNodes * kMaxNodes;
    a.flag = c->flag;
    a.dt = dt;
    a.phibar = c->phibar;
    a.inv_a2 = c->inv_a2;
    a.M = M;
    a.batch = B;
    a.ncoef = c->g.ncoef;
    a.T = c->g.T;
    for (int k = 0; k < K; ++k) {
        double* un = c->seq_u[k & 1];
        double* en = c->seq_e[k & 1];
        a.unew = un;
        a.enew = en;
        for (int m = 0; m < M; ++m) {
            const bool last = k == K - 1 && m == M - 1;
            a.m = m;
            a.out = last ? state : un + m * nsn;
            a.cml = last ? nullptr : c->cml;
            const long t = c->begin(SDC_KERNEL_UPDATE);
            launch_update_seq(a, c->st);
            c->end(SDC_KERNEL_UPDATE, t);
            if (!last) run_explicit_cml(c, B, en + m * nsn);
        }
        a.uold = un;
        a.uold_node = nsn;
        a.eold = en;
        a.eold_node = nsn;
    }
}

// Paths built for the paper's split only (f_I = L_g): the adjoint, the sequential SDC and IMEX-o2
// with their closed-form gravity-wave solves.
int paper_split_only(sdc_handle h, const char* what) {
    if (h->cfg.implicit_coriolis)
        return fail(SDC_EUNSUPPORTED, "%s is built for the split with f_I = L_g (implicit_coriolis = 0)", what);
    return SDC_OK;
}

int check_imex2_state(sdc_handle h, const double* state, double dt) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = paper_split_only(h, "IMEX-o2")) return rc;
    if (!state) return fail(SDC_EINVAL, "state is NULL");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(SDC_EINVAL, "dt must be positive and finite");
    return SDC_OK;
}

int check_imex2_args(sdc_handle h, const double* state, double dt) {
    if (int rc = check_imex2_state(h, state, dt)) return rc;
    return alloc_imex2(h);
}

int check_adjoint_args(sdc_handle h, const double* state_n, const double* lam_np1, const double* lam_n,
                       double dt, int M, int K) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = paper_split_only(h, "the adjoint step")) return rc;
    if (!state_n || !lam_np1 || !lam_n) return fail(SDC_EINVAL, "state_n/lam_np1/lam_n is NULL");
    if (M < 1 || M > h->cfg.M) return fail(SDC_EINVAL, "M=%d out of range 1..%d", M, h->cfg.M);
    if (K < 1 || K > h->cfg.K) return fail(SDC_EINVAL, "K=%d out of range 1..%d", K, h->cfg.K);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(SDC_EINVAL, "dt must be positive and finite");
    return SDC_OK;
}

// The reversed sweep of the adjoint step, reading the stage grid fields from `tape`: last-node
// update, then sweeps K-1..1, then the initial f_E.
void enqueue_adjoint_reverse(sdc_ctx* c, const double2* tape, const double* lam_np1, double* lam_n,
                             double dt, int M, int K) {
    const int B = c->cfg.batch;
    const long long fs = 3LL * c->g.ncoef * 2;
    auto save_at = [&](int s) { return tape + stage_states(c, s, M) * tape_per_state(c); };
    AdjUpdateArgs b{};
    b.tau = c->tau + M * kMaxNodes;
    b.Q = c->Q + M * kMaxNodes * kMaxNodes;
    b.n_of = c->n_of;
    b.dt = dt;
    b.phibar = c->phibar;
    b.inv_a2 = c->inv_a2;
    b.M = M;
    b.batch = B;
    b.ncoef = c->g.ncoef;
    b.ubar_n = c->adj_un;
    b.ubar = lam_np1;
    b.ubar_node = 0;
    b.ubar_member = fs;
    b.ubar_prev = c->adj_ubar;
    b.ebar_prev = c->adj_ebar;
    b.sweep = qd_sweep(c, K, M);
    b.last = 1;
    b.first_stage = K == 1;
    b.init_un = 1;
    if (c->lplan.fuse_update && (M == 1 || M == 2 || M == 4)) {
        // The adjoint update of sweep s runs in the epilogue of the transposed analysis that
        // completes its node adjoints, and every update writes the next transposed tendency's
        // input directly; the first stage's epilogue writes lam_n.
        b.cml = c->cml;
        b.cml32 = c->P32 != nullptr ? 1 : 0;
        b.T = c->g.T;
        b.m_of = c->m_of;
        b.rowoff = c->rowoff;
        b.neg_lap = c->neg_lap;
        launch_update_adj(b, c->st);
        AdjFuse af{};
        af.m_of = c->m_of;
        af.a = b;
        af.a.ubar = c->adj_ubar;
        af.a.ubar_node = fs;
        af.a.ubar_member = (long long)M * fs;
        af.a.last = 0;
        af.a.init_un = 0;
        af.mode = 1;
        for (int s = K - 1; s >= 1; --s) {
            af.a.sweep = qd_sweep(c, s, M);
            af.a.first_stage = s == 1;
            run_explicit_adj(c, c->adj_ebar, B * M, save_at(s), c->adj_ubar, &af, true);
        }
        AdjFuse fin{};
        fin.mode = 2;
        fin.lam_out = lam_n;
        fin.m_of = c->m_of;
        run_explicit_adj(c, c->adj_ebar, B, save_at(0), c->adj_un, &fin, true);
        return;
    }
    launch_update_adj(b, c->st);
    for (int s = K - 1; s >= 1; --s) {
        run_explicit_adj(c, c->adj_ebar, B * M, save_at(s), c->adj_ubar);
        b.ubar = c->adj_ubar;
        b.ubar_node = fs;
        b.ubar_member = (long long)M * fs;
        b.sweep = qd_sweep(c, s, M);
        b.last = 0;
        b.first_stage = s == 1;
        b.init_un = 0;
        launch_update_adj(b, c->st);
    }
    run_explicit_adj(c, c->adj_ebar, B, save_at(0), c->adj_un);
    launch_finish_adj(c->adj_un, lam_n, c->m_of, c->g.ncoef, B, c->st);
}

// Replays the cached graph of (kind, state, dt, M, K), capturing it first if needed.
template <class Enqueue>
int graph_launch(sdc_ctx* c, int kind, double* state, double dt, int M, int K, Enqueue&& enqueue) {
    sdc_ctx::GraphEntry* hit = nullptr;
    for (auto& ge : c->graphs)
        if (ge.kind == kind && ge.state == state && ge.dt == dt && ge.M == M && ge.K == K) hit = &ge;
    if (!hit) {
        if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        hipStream_t user = c->st;
        const bool timing = c->timing;
        c->st = c->cap;
        c->timing = false;
        hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
        hipGraph_t graph = nullptr;
        if (e == hipSuccess) {
            enqueue();
            e = hipStreamEndCapture(c->cap, &graph);
        }
        c->st = user;
        c->timing = timing;
        if (e != hipSuccess) return fail(SDC_EHIP, "step capture failed: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(SDC_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        if (c->graphs.size() >= 8) {          // keep a few recent shapes
            (void)hipGraphExecDestroy(c->graphs.front().exec);
            (void)hipGraphDestroy(c->graphs.front().graph);
            c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back({kind, state, dt, M, K, graph, exec});
        hit = &c->graphs.back();
    }
    HIP_TRY(hipGraphLaunch(hit->exec, c->st));
    return SDC_OK;
}

}  // namespace

extern "C" {

int sdc_step(sdc_handle h, double* state, double dt, int M, int K) {
    if (int rc = check_step_args(h, state, dt, M, K)) return rc;
    enqueue_step(h, state, dt, M, K);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_step_graph(sdc_handle h, double* state, double dt, int M, int K) {
    if (int rc = check_step_args(h, state, dt, M, K)) return rc;
    return graph_launch(h, 0, state, dt, M, K, [&] { enqueue_step(h, state, dt, M, K); });
}

int sdc_step_sequential(sdc_handle h, double* state, double dt, int M, int K) {
    if (int rc = check_step_args(h, state, dt, M, K)) return rc;
    if (int rc = paper_split_only(h, "the sequential IMEX SDC step")) return rc;
    if (int rc = alloc_seq(h)) return rc;
    enqueue_seq(h, state, dt, M, K);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_step_sequential_graph(sdc_handle h, double* state, double dt, int M, int K) {
    if (int rc = check_step_args(h, state, dt, M, K)) return rc;
    if (int rc = paper_split_only(h, "the sequential IMEX SDC step")) return rc;
    if (int rc = alloc_seq(h)) return rc;
    return graph_launch(h, 2, state, dt, M, K, [&] { enqueue_seq(h, state, dt, M, K); });
}

int imex2_step(sdc_handle h, double* state, double dt) {
    if (int rc = check_imex2_args(h, state, dt)) return rc;
    enqueue_imex2(h, state, dt, h->i2_ustar, h->i2_k1, h->i2_k2);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int imex2_step_graph(sdc_handle h, double* state, double dt) {
    if (int rc = check_imex2_args(h, state, dt)) return rc;
    return graph_launch(h, 1, state, dt, 0, 0,
                        [&] { enqueue_imex2(h, state, dt, h->i2_ustar, h->i2_k1, h->i2_k2); });
}

int imex2_step_noalloc(sdc_handle h, double* state, double dt) {
    if (int rc = check_imex2_state(h, state, dt)) return rc;
    const size_t per = (size_t)h->cfg.batch * 3 * h->g.ncoef * 2;        // doubles of one state set
    const size_t need = 3 * per * sizeof(double);
    if (need > kScratchBytes)
        return fail(SDC_EINVAL, "imex2_step_noalloc needs %zu bytes of device scratch (u*, k1, k2 of %d "
                    "members), more than its fixed %zu bytes; use imex2_step", need, h->cfg.batch,
                    kScratchBytes);
    if (!h->scratch_dev)
        return fail(SDC_EHIP, "device scratch of device %d unavailable: %s", h->dev,
                    hipGetErrorString(h->scratch_err));
    // no event pool growth either: timing events are not recorded by this call
    const bool timing = h->timing;
    h->timing = false;
    enqueue_imex2(h, state, dt, h->scratch_dev, h->scratch_dev + per, h->scratch_dev + 2 * per);
    h->timing = timing;
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_step_adjoint(sdc_handle h, const double* state_n, const double* lam_np1, double* lam_n,
                     double dt, int M, int K) {
    if (int rc = check_adjoint_args(h, state_n, lam_np1, lam_n, dt, M, K)) return rc;
    if (lam_n == state_n) return fail(SDC_EINVAL, "lam_n must not alias state_n");
    sdc_ctx* c = h;
    if (int rc = alloc_adjoint(c, true)) return rc;
    // 1. recompute the forward stages, keeping the grid fields of every f_E evaluation
    HIP_TRY(hipMemcpyAsync(c->adj_x, state_n, (size_t)c->cfg.batch * 3 * c->g.ncoef * 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, c->st));
    enqueue_step(c, c->adj_x, dt, M, K, c->adj_save, false);
    // 2. the reversed sweep
    enqueue_adjoint_reverse(c, c->adj_save, lam_np1, lam_n, dt, M, K);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_tape_size(sdc_handle h, int M, int K, long long* bytes) {
    if (int rc = check_handle(h)) return rc;
    if (!bytes) return fail(SDC_EINVAL, "bytes is NULL");
    if (M < 1 || M > h->cfg.M) return fail(SDC_EINVAL, "M=%d out of range 1..%d", M, h->cfg.M);
    if (K < 1 || K > h->cfg.K) return fail(SDC_EINVAL, "K=%d out of range 1..%d", K, h->cfg.K);
    *bytes = (long long)(stage_states(h, K, M) * tape_per_state(h) * sizeof(double2));
    return SDC_OK;
}

int sdc_step_taped(sdc_handle h, double* state, double dt, int M, int K, void* tape) {
    if (int rc = check_step_args(h, state, dt, M, K)) return rc;
    if (!tape) return fail(SDC_EINVAL, "tape is NULL");
    if (reinterpret_cast<uintptr_t>(tape) % 16) return fail(SDC_EINVAL, "tape must be 16-byte aligned");
    enqueue_step(h, state, dt, M, K, static_cast<double2*>(tape), true);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_step_adjoint_taped(sdc_handle h, const void* tape, const double* lam_np1, double* lam_n,
                           double dt, int M, int K) {
    if (!tape) return fail(SDC_EINVAL, "tape is NULL");
    if (reinterpret_cast<uintptr_t>(tape) % 16) return fail(SDC_EINVAL, "tape must be 16-byte aligned");
    if (int rc = check_adjoint_args(h, static_cast<const double*>(tape), lam_np1, lam_n, dt, M, K)) return rc;
    if (int rc = alloc_adjoint(h, false)) return rc;
    enqueue_adjoint_reverse(h, static_cast<const double2*>(tape), lam_np1, lam_n, dt, M, K);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sht_inverse(sdc_handle h, const double* spec, double* grid) {
    if (int rc = check_handle(h)) return rc;
    if (!spec || !grid) return fail(SDC_EINVAL, "spec/grid is NULL");
    const int B = h->cfg.batch;
    launch_synthesis_scalar(h->P, h->toff, h->ssyn_tasks, h->n_ssyn, spec, B, h->four, h->g, h->st);
    launch_fft_inverse_scalar(h->four, grid, h->tw, h->plan, B, h->g, h->st);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sht_inverse_adjoint(sdc_handle h, const double* grid, double* spec) {
    if (int rc = check_handle(h)) return rc;
    if (!spec || !grid) return fail(SDC_EINVAL, "spec/grid is NULL");
    const int B = h->cfg.batch;
    double2* sana = reinterpret_cast<double2*>(h->G);
    launch_fft_forward_scalar(grid, sana, h->w, h->tw, h->plan, B, 1, h->g, h->st);
    launch_analysis_scalar(h->P, h->toff, h->sana_tasks, h->n_sana, sana, B, spec, h->g, h->st);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sht_forward(sdc_handle h, const double* grid, double* spec) {
    if (int rc = check_handle(h)) return rc;
    if (!spec || !grid) return fail(SDC_EINVAL, "spec/grid is NULL");
    const int B = h->cfg.batch;
    double2* sana = reinterpret_cast<double2*>(h->G);     // [f][p][nhp][m] fits in G
    launch_fft_forward_scalar(grid, sana, h->w, h->tw, h->plan, B, 0, h->g, h->st);
    launch_analysis_scalar(h->P, h->toff, h->sana_tasks, h->n_sana, sana, B, spec, h->g, h->st);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int imex_solve(sdc_handle h, double alpha, const double* beta, double* u) {
    if (int rc = check_handle(h)) return rc;
    if (!beta || !u) return fail(SDC_EINVAL, "beta/u is NULL");
    if (!(alpha >= 0) || !std::isfinite(alpha)) return fail(SDC_EINVAL, "alpha must be >= 0 and finite");
    if (h->cfg.implicit_coriolis) {
        LcArgs l{};
        l.mode = 1;
        l.beta = beta;
        l.alpha = alpha;
        l.uout = u;
        l.out_member = 3LL * h->g.ncoef * 2;
        l.lc = h->lc;
        l.scratch = h->lc_scratch;
        l.rowoff = h->rowoff;
        l.inv_lap = h->inv_lap;
        l.flag = h->flag;
        l.tau = h->tau + kMaxNodes;       // unused by the plain solve (valid addresses only)
        l.Q = h->Q + kMaxNodes * kMaxNodes;
        l.phibar = h->phibar;
        l.inv_a2 = h->inv_a2;
        l.two_omega = h->two_omega;
        l.M = 1;
        l.batch = h->cfg.batch;
        l.ncoef = h->g.ncoef;
        l.T = h->g.T;
        l.sweep = 1;
        launch_solve_lc(l, h->st);
    } else {
        launch_solve(alpha, beta, u, h->n_of, h->phibar, h->inv_a2, h->cfg.batch, h->g.ncoef, h->st);
    }
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int eval_explicit(sdc_handle h, const double* u, double* fE) {
    if (int rc = check_handle(h)) return rc;
    if (!u || !fE) return fail(SDC_EINVAL, "u/fE is NULL");
    if (u == fE) return fail(SDC_EINVAL, "fE must not alias u");
    run_explicit(h, u, h->cfg.batch, fE);
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int eval_implicit(sdc_handle h, const double* u, double* fI) {
    if (int rc = check_handle(h)) return rc;
    if (!u || !fI) return fail(SDC_EINVAL, "u/fI is NULL");
    if (h->cfg.implicit_coriolis) {
        const size_t nb = (size_t)h->cfg.batch * 3 * h->g.ncoef * 2 * sizeof(double);
        const char *pu = (const char*)u, *pf = (const char*)fI;
        if (pu < pf + nb && pf < pu + nb)
            return fail(SDC_EINVAL, "with implicit_coriolis fI must not overlap u (L_c reads neighbouring degrees)");
        launch_implicit_lc(u, fI, h->n_of, h->m_of, h->lc, h->phibar, h->inv_a2, h->two_omega, h->g.T,
                           h->cfg.batch, h->g.ncoef, h->st);
    } else {
        launch_implicit(u, fI, h->n_of, h->phibar, h->inv_a2, h->cfg.batch, h->g.ncoef, h->st);
    }
    HIP_TRY(hipGetLastError());
    return SDC_OK;
}

int sdc_debug_poison(sdc_handle h, int on) {
    if (int rc = check_handle(h)) return rc;
    if (on != 0 && on != 1) return fail(SDC_EINVAL, "on=%d: 0 or 1", on);
    h->debug_poison = on != 0;
    h->drop_graphs();
    return SDC_OK;
}

int sdc_timing_enable(sdc_handle h, int on) {
    if (int rc = check_handle(h)) return rc;
    HIP_TRY(hipStreamSynchronize(h->st));
    h->reset_timing();
    h->timing = on != 0;
    return SDC_OK;
}

int sdc_timing_read(sdc_handle h, int kernel_class, double* total_ms, long long* launches) {
    if (int rc = check_handle(h)) return rc;
    if (kernel_class < 0 || kernel_class >= SDC_KERNEL_CLASSES)
        return fail(SDC_EINVAL, "kernel_class=%d out of range", kernel_class);
    if (!total_ms || !launches) return fail(SDC_EINVAL, "total_ms/launches is NULL");
    HIP_TRY(hipStreamSynchronize(h->st));
    double tot = 0.0;
    for (const auto& pr : h->ev_marks[kernel_class]) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev_pool[pr.first], h->ev_pool[pr.second]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (long long)h->ev_marks[kernel_class].size();
    return SDC_OK;
}

int sdc_sync(sdc_handle h) {
    if (int rc = check_handle(h)) return rc;
    HIP_TRY(hipStreamSynchronize(h->st));
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        HIP_TRY(hipMemset(h->flag, 0, sizeof(int)));
        return fail(SDC_ENONFINITE, "a step produced a non-finite value");
    }
    return SDC_OK;
}

int sdc_copy_grid(sdc_handle h, double* mu, double* w) {
    if (int rc = check_handle(h)) return rc;
    if (!mu || !w) return fail(SDC_EINVAL, "mu/w is NULL");
    HIP_TRY(hipStreamSynchronize(h->st));
    HIP_TRY(hipMemcpy(mu, h->mu, h->g.nlat * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(w, h->w, h->g.nlat * sizeof(double), hipMemcpyDeviceToHost));
    return SDC_OK;
}

int sdc_copy_coefficients(sdc_handle h, int M, double* tau, double* Q) {
    if (int rc = check_handle(h)) return rc;
    if (M < 1 || M > h->cfg.M) return fail(SDC_EINVAL, "M=%d out of range 1..%d", M, h->cfg.M);
    if (!tau || !Q) return fail(SDC_EINVAL, "tau/Q is NULL");
    HIP_TRY(hipStreamSynchronize(h->st));
    std::vector<double> t(kMaxNodes), q(kMaxNodes * kMaxNodes);
    HIP_TRY(hipMemcpy(t.data(), h->tau + M * kMaxNodes, t.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(q.data(), h->Q + M * kMaxNodes * kMaxNodes, q.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int m = 0; m < M; ++m) {
        tau[m] = t[m];
        for (int j = 0; j < M; ++j) Q[m * M + j] = q[m * kMaxNodes + j];
    }
    return SDC_OK;
}

int sdc_copy_legendre(sdc_handle h, int m, double* Pbar, double* H) {
    if (int rc = check_handle(h)) return rc;
    if (m < 0 || m > h->g.T) return fail(SDC_EINVAL, "m=%d out of range 0..T", m);
    if (!Pbar || !H) return fail(SDC_EINVAL, "Pbar/H is NULL");
    HIP_TRY(hipStreamSynchronize(h->st));
    const Geom& g = h->g;
    for (int p = 0; p < 2; ++p) {
        const int np = npk_of(g.T, m, p);
        std::vector<double> bp((size_t)((np + 3) & ~3) * g.nhp), bh(bp.size());
        if (np == 0) continue;
        HIP_TRY(hipMemcpy(bp.data(), h->P + h->h_toff[2 * m + p], bp.size() * sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(bh.data(), h->H + h->h_toff[2 * m + p], bh.size() * sizeof(double), hipMemcpyDeviceToHost));
        const int np4 = (np + 3) & ~3;
        for (int kk = 0; kk < np; ++kk) {
            const int row = p + 2 * kk;    // n - m
            for (int j = 0; j < g.nh; ++j) {
                Pbar[(size_t)row * g.nh + j] = bp[tab_index(np4, kk, j)];
                H[(size_t)row * g.nh + j] = bh[tab_index(np4, kk, j)];
            }
        }
    }
    return SDC_OK;
}

// ---------------------------------------------------------------------------------------------
// Ensembles of mixed truncations: one graph per step whose parallel branches are the members'
// handles (each with its own workspaces), forked from and joined back to one capture stream.
// ---------------------------------------------------------------------------------------------
struct sdc_group_s {
    std::vector<sdc_handle> members;
    int mode = 0;                     // 1: one launch per kernel class and phase over all members
    bool tuned = false;               // plan / plan1 timed by sdc_group_autotune for mode 1
    LegPlan plan{}, plan1{};          // Legendre variants of the merged node / one-state launches
    void* desc = nullptr;             // device copies of the merged launches' per-member arguments
    size_t desc_bytes = 0;
    hipStream_t st = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> branch;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    std::vector<double*> key_states;
    std::vector<double> key_dts;
    int key_M = 0, key_K = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~sdc_group_s() {
        if (desc) (void)hipFree(desc);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (hipStream_t b : branch) (void)hipStreamDestroy(b);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

}  // extern "C"

namespace {

// Whether the members can share one launch per kernel class and phase: the same precision, the
// same kind of node update (fused or separate), the paper's split, one launch per sweep, and FFT
// lengths the multi-handle grid kernel is built for.  msg receives the reason otherwise.
bool group_mergeable(const sdc_group_s* g, int M, std::string* msg) {
    const sdc_ctx* c0 = g->members[0];
    const bool fused0 = c0->lplan.fuse_update && (M == 1 || M == 2 || M == 4);
    for (const sdc_ctx* c : g->members) {
        if (c->cfg.precision != c0->cfg.precision) { *msg = "members of different precision"; return false; }
        if (c->cfg.implicit_coriolis) { *msg = "a member with implicit_coriolis"; return false; }
        if (c->lplan.node_launch) { *msg = "a member with node_launch"; return false; }
        if ((c->lplan.fuse_update && (M == 1 || M == 2 || M == 4)) != fused0) {
            *msg = "members with and without the fused node update";
            return false;
        }
        if (!grid_multi_supported(c->cfg.nlon)) {
            *msg = "a member's nlon is not one of 96, 192, 384, 768";
            return false;
        }
    }
    return true;
}

// Bytes of device descriptors one merged step needs at most (K f_E and K + 1 update launches).
size_t group_desc_bytes(const sdc_group_s* g) {
    int kmax = kMaxSweeps;
    for (const sdc_ctx* c : g->members) kmax = std::min(kmax, c->cfg.K);
    const size_t per_op = sizeof(SynArgs) + sizeof(GridArgs) + sizeof(AnaArgs) + sizeof(UpdArgsM);
    return (size_t)(2 * kmax + 2) * (g->members.size() * per_op + 4 * 16) + 256;   // + 16-byte alignment
}

// Records every member's step, builds one descriptor list per launch (workgroup ranges of the
// members back to back, each starting at a multiple of 8), copies them to the device and captures
// one launch per kernel class and phase on g->cap.
int group_capture_merged(sdc_group_s* g, double* const* states, const double* dts, int M, int K,
                         hipGraph_t* graph) {
    const size_t n = g->members.size();
    std::vector<std::vector<StepOp>> ops(n);
    for (size_t h = 0; h < n; ++h) {
        sdc_ctx* c = g->members[h];
        c->rec = &ops[h];
        enqueue_step(c, states[h], dts[h], M, K);
        c->rec = nullptr;
    }
    for (size_t h = 1; h < n; ++h) {
        if (ops[h].size() != ops[0].size()) return fail(SDC_EUNSUPPORTED, "members record different steps");
        for (size_t i = 0; i < ops[0].size(); ++i)
            if (ops[h][i].kind != ops[0][i].kind || ops[h][i].fuse_mode != ops[0][i].fuse_mode ||
                (ops[h][i].states == nullptr) != (ops[0][i].states == nullptr))
                return fail(SDC_EUNSUPPORTED, "members record different steps");
    }
    // the variants of the member with the most work serve every member (all variants give the
    // same results)
    size_t lead = 0;
    for (size_t h = 1; h < n; ++h)
        if ((double)g->members[h]->g.ncoef * g->members[h]->cfg.batch >
            (double)g->members[lead]->g.ncoef * g->members[lead]->cfg.batch)
            lead = h;
    const sdc_ctx* cl = g->members[lead];
    const bool fp32 = cl->P32 != nullptr;
    const int tt = cl->table_type();
    int nlon_max = 0;
    for (const sdc_ctx* c : g->members) nlon_max = std::max(nlon_max, c->cfg.nlon);
    // host image of the descriptors
    std::vector<char> img;
    auto put = [&](const void* p, size_t nb) {
        const size_t off = (img.size() + 15) / 16 * 16;
        img.resize(off + nb);
        std::memcpy(img.data() + off, p, nb);
        return off;
    };
    struct Launch {
        int kind;
        LegPlan plan;
        bool state_in;
        size_t syn, grid, ana, upd;
        int syn_blocks, grid_blocks, ana_blocks, upd_blocks;
    };
    std::vector<Launch> launches;
    for (size_t i = 0; i < ops[0].size(); ++i) {
        Launch L{};
        L.kind = ops[0][i].kind;
        if (L.kind == 0) {
            // one-state launches (a step's first f_E) and node launches have their own variants
            const bool one = ops[0][i].S == g->members[0]->cfg.batch;
            const LegPlan lp = g->tuned ? (one ? g->plan1 : g->plan) : cl->plan_for(ops[lead][i].S);
            L.plan = lp;
            L.state_in = ops[0][i].states != nullptr;
            std::vector<SynArgs> sy(n);
            std::vector<GridArgs> gr(n);
            std::vector<AnaArgs> an(n);
            int fs = 0, fg = 0, fa = 0;
            for (size_t h = 0; h < n; ++h) {
                sdc_ctx* c = g->members[h];
                const StepOp& op = ops[h][i];
                sy[h] = make_syn_args(c->tables(), c->toff, c->rowoff, c->syn_list(lp), c->syn_count(lp), c->cml,
                                      op.S, reinterpret_cast<double*>(c->four), c->g, op.states);
                sy[h].first = fs;
                fs += (sy[h].blocks + 7) / 8 * 8;
                gr[h] = make_grid_args(c->four, c->G, c->mu, c->w, c->tw, op.S, c->two_omega_explicit, op.save,
                                       c->g);
                gr[h].first = fg;
                fg += (gr[h].blocks + 7) / 8 * 8;
                an[h] = make_ana_args(c->tables(), lp, c->toff, c->ana_tasks, c->n_ana_wg, c->G, op.S, c->neg_lap,
                                      op.out, c->g, op.fuse_mode ? &op.upd : nullptr, op.fuse_mode);
                an[h].first = fa;
                fa += (an[h].blocks + 7) / 8 * 8;
            }
            L.syn = put(sy.data(), n * sizeof(SynArgs));
            L.grid = put(gr.data(), n * sizeof(GridArgs));
            L.ana = put(an.data(), n * sizeof(AnaArgs));
            L.syn_blocks = fs;
            L.grid_blocks = fg;
            L.ana_blocks = fa;
        } else {
            std::vector<UpdArgsM> up(n);
            int fu = 0;
            for (size_t h = 0; h < n; ++h) {
                const StepOp& op = ops[h][i];
                up[h].a = op.upd;
                up[h].gx = (2 * op.upd.ncoef + 63) / 64;
                up[h].blocks = up[h].gx * op.upd.batch;
                up[h].first = fu;
                fu += (up[h].blocks + 7) / 8 * 8;
            }
            L.upd = put(up.data(), n * sizeof(UpdArgsM));
            L.upd_blocks = fu;
        }
        launches.push_back(L);
    }
    if (img.size() > g->desc_bytes) return fail(SDC_EINVAL, "merged step needs more descriptor space than reserved");
    HIP_TRY(hipStreamSynchronize(g->st));            // a replay of the previous graph may read them
    HIP_TRY(hipMemcpy(g->desc, img.data(), img.size(), hipMemcpyHostToDevice));
    const char* d = static_cast<const char*>(g->desc);
    HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    for (const Launch& L : launches) {
        if (L.kind == 0) {
            launch_synthesis_multi(L.plan, tt, L.state_in, reinterpret_cast<const SynArgs*>(d + L.syn), (int)n,
                                   L.syn_blocks, g->cap);
            launch_grid_multi(fp32, nlon_max, reinterpret_cast<const GridArgs*>(d + L.grid), (int)n, L.grid_blocks,
                              g->cap);
            launch_analysis_multi(L.plan, tt, reinterpret_cast<const AnaArgs*>(d + L.ana), (int)n, L.ana_blocks,
                                  g->cap);
        } else {
            launch_update_multi(M, reinterpret_cast<const UpdArgsM*>(d + L.upd), (int)n, L.upd_blocks, g->cap);
        }
    }
    const hipError_t e = hipStreamEndCapture(g->cap, graph);
    if (e != hipSuccess) return fail(SDC_EHIP, "group step capture failed: %s", hipGetErrorString(e));
    (void)K;
    return SDC_OK;
}

// One graph branch per member, each with the member's own launches.
int group_capture_branches(sdc_group_s* g, double* const* states, const double* dts, int M, int K,
                           hipGraph_t* graph) {
    const size_t n = g->members.size();
    hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipEventRecord(g->fork, g->cap);
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        sdc_ctx* c = g->members[i];
        e = hipStreamWaitEvent(g->branch[i], g->fork, 0);
        if (e != hipSuccess) break;
        const hipStream_t saved = c->st;
        const bool saved_timing = c->timing;
        c->st = g->branch[i];
        c->timing = false;
        enqueue_step(c, states[i], dts[i], M, K);
        c->st = saved;
        c->timing = saved_timing;
        e = hipEventRecord(g->join[i], g->branch[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(g->cap, g->join[i], 0);
    }
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g->cap, &gr);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(SDC_EHIP, "group step capture failed: %s", hipGetErrorString(e));
    }
    *graph = gr;
    return SDC_OK;
}

// Times one merged synthesis and one merged analysis launch of every built Legendre variant at the
// node shape (batch x M states per member) and at the one-state shape, the states read in place
// as in a step, and keeps the fastest of each in g->plan / g->plan1.
int group_tune_legendre(sdc_group_s* g, int M, int reps) {
    const size_t n = g->members.size();
    const int tt = g->members[0]->table_type();
    for (sdc_ctx* c : g->members) {         // finite operands in the workspaces
        HIP_TRY(hipMemsetAsync(c->ua, 0, (size_t)c->smax * 3 * c->g.ncoef * 2 * sizeof(double), g->st));
        HIP_TRY(hipMemsetAsync(c->cml, 0, (size_t)c->g.nrows * c->smax * kCmlVals * sizeof(double), g->st));
        HIP_TRY(hipMemsetAsync(c->G, 0, (size_t)(c->g.T + 1) * 2 * c->g.nhp * c->smax * kAnaStride * sizeof(double),
                               g->st));
    }
    HIP_TRY(hipStreamSynchronize(g->st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SDC_EHIP, "hipEventCreate failed");
    }
    hipError_t err = hipSuccess;
    auto time_it = [&](auto&& launch) {
        float ms = 0.f;
        launch();
        hipError_t e = hipEventRecord(e0, g->st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, g->st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) err = e;
        return ms;
    };
    constexpr int kSyn = 14;
    const int shapes[kSyn][3] = {{1, 8, 0}, {1, 4, 0}, {2, 4, 0}, {2, 2, 0}, {3, 2, 0},
                                 {4, 2, 0}, {4, 1, 0}, {6, 1, 0}, {1, 8, 1}, {1, 4, 1},
                                 {2, 4, 1}, {2, 2, 1}, {4, 2, 1}, {4, 1, 1}};
    for (int one = 0; one < 2 && err == hipSuccess; ++one) {
        LegPlan best = g->members[0]->lplan;
        float best_ms = 1e30f;
        for (int k = 0; k < kSyn && err == hipSuccess; ++k) {
            LegPlan lp = best;
            lp.syn_tiles = shapes[k][0];
            lp.syn_depth = shapes[k][1];
            lp.syn_recur = shapes[k][2];
            std::vector<SynArgs> sy(n);
            int fs = 0;
            for (size_t h = 0; h < n; ++h) {
                sdc_ctx* c = g->members[h];
                const int S = one ? c->cfg.batch : c->cfg.batch * M;
                sy[h] = make_syn_args(c->tables(), c->toff, c->rowoff, c->syn_list(lp), c->syn_count(lp), c->cml, S,
                                      reinterpret_cast<double*>(c->four), c->g, c->ua);
                sy[h].first = fs;
                fs += (sy[h].blocks + 7) / 8 * 8;
            }
            err = hipMemcpy(g->desc, sy.data(), n * sizeof(SynArgs), hipMemcpyHostToDevice);
            if (err != hipSuccess) break;
            const float ms = time_it([&] {
                launch_synthesis_multi(lp, tt, true, static_cast<const SynArgs*>(g->desc), (int)n, fs, g->st);
            });
            if (ms < best_ms) {
                best_ms = ms;
                best.syn_tiles = lp.syn_tiles;
                best.syn_depth = lp.syn_depth;
                best.syn_recur = lp.syn_recur;
            }
        }
        best_ms = 1e30f;
        LegPlan ana_best = best;
        for (int k = 0; k < 8 && err == hipSuccess; ++k) {
            LegPlan lp = best;
            lp.ana_depth = (k & 2) ? 2 : 4;
            lp.ana_interleave = (k & 1) ? 0 : 1;
            lp.ana_recur = k >> 2;
            std::vector<AnaArgs> an(n);
            int fa = 0;
            for (size_t h = 0; h < n; ++h) {
                sdc_ctx* c = g->members[h];
                const int S = one ? c->cfg.batch : c->cfg.batch * M;
                an[h] = make_ana_args(c->tables(), lp, c->toff, c->ana_tasks, c->n_ana_wg, c->G, S, c->neg_lap, c->E,
                                      c->g, nullptr, 0);
                an[h].first = fa;
                fa += (an[h].blocks + 7) / 8 * 8;
            }
            err = hipMemcpy(g->desc, an.data(), n * sizeof(AnaArgs), hipMemcpyHostToDevice);
            if (err != hipSuccess) break;
            const float ms = time_it([&] {
                launch_analysis_multi(lp, tt, static_cast<const AnaArgs*>(g->desc), (int)n, fa, g->st);
            });
            if (ms < best_ms) {
                best_ms = ms;
                ana_best = lp;
            }
        }
        (one ? g->plan1 : g->plan) = ana_best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(SDC_EHIP, "group autotune launch failed: %s", hipGetErrorString(err));
    g->tuned = true;
    return SDC_OK;
}

}  // namespace

extern "C" {

int sdc_group_create(const sdc_handle* members, int n, void* hip_stream, sdc_group* out) {
    if (!out) return fail(SDC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || n < 1 || n > 64) return fail(SDC_EINVAL, "members/n invalid (1 <= n <= 64)");
    for (int i = 0; i < n; ++i) {
        if (!members[i]) return fail(SDC_EINVAL, "member %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return fail(SDC_EINVAL, "member %d repeated", i);
    }
    sdc_group_s* g = new (std::nothrow) sdc_group_s();
    if (!g) return fail(SDC_ENOMEM, "host allocation failed");
    g->members.assign(members, members + n);
    g->st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        hipStream_t b = nullptr;
        hipEvent_t j = nullptr;
        e = hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
        if (e == hipSuccess) g->branch.push_back(b);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e == hipSuccess) g->join.push_back(j);
    }
    if (e != hipSuccess) {
        delete g;
        return fail(SDC_EHIP, "group stream/event creation failed: %s", hipGetErrorString(e));
    }
    g->desc_bytes = group_desc_bytes(g);
    if (hipMalloc(&g->desc, g->desc_bytes) != hipSuccess) {
        (void)hipGetLastError();
        g->desc = nullptr;
        delete g;
        return fail(SDC_ENOMEM, "group descriptor allocation failed");
    }
    std::string why;
    g->mode = group_mergeable(g, g->members[0]->cfg.M, &why) ? 1 : 0;
    *out = g;
    return SDC_OK;
}

int sdc_group_set_mode(sdc_group g, int mode) {
    if (!g) return fail(SDC_EINVAL, "group is NULL");
    if (mode != 0 && mode != 1) return fail(SDC_EINVAL, "mode=%d: 0 or 1", mode);
    if (mode != g->mode && g->exec) {              // recaptured on the next step
        (void)hipGraphExecDestroy(g->exec);
        (void)hipGraphDestroy(g->graph);
        g->exec = nullptr;
        g->graph = nullptr;
    }
    g->mode = mode;
    return SDC_OK;
}

int sdc_group_get_mode(sdc_group g, int* mode) {
    if (!g || !mode) return fail(SDC_EINVAL, "group/mode is NULL");
    *mode = g->mode;
    return SDC_OK;
}

int sdc_group_autotune(sdc_group g, double* const* states, const double* dts, int M, int K, int reps, int* mode) {
    if (!g) return fail(SDC_EINVAL, "group is NULL");
    if (!states || !dts) return fail(SDC_EINVAL, "states/dts is NULL");
    if (reps < 1 || reps > 1000) return fail(SDC_EINVAL, "reps = %d outside [1, 1000]", reps);
    const size_t n = g->members.size();
    for (size_t i = 0; i < n; ++i)
        if (int rc = check_step_args(g->members[i], states[i], dts[i], M, K)) return rc;
    std::string why;
    if (!group_mergeable(g, M, &why)) {
        if (g->mode != 0) (void)sdc_group_set_mode(g, 0);
        if (mode) *mode = 0;
        return SDC_OK;
    }
    if (g->exec) {                          // its descriptors are overwritten by the timing below
        (void)hipStreamSynchronize(g->st);
        (void)hipGraphExecDestroy(g->exec);
        (void)hipGraphDestroy(g->graph);
        g->exec = nullptr;
        g->graph = nullptr;
    }
    if (int rc = group_tune_legendre(g, M, reps)) return rc;
    // whole steps in both modes, on copies of the states (restored afterwards)
    std::vector<void*> saved(n, nullptr);
    std::vector<size_t> nb(n);
    int rc = SDC_OK;
    for (size_t i = 0; i < n && rc == SDC_OK; ++i) {
        nb[i] = (size_t)g->members[i]->cfg.batch * 3 * g->members[i]->g.ncoef * 2 * sizeof(double);
        if (hipMalloc(&saved[i], nb[i]) != hipSuccess) {
            (void)hipGetLastError();
            saved[i] = nullptr;
            rc = fail(SDC_ENOMEM, "group autotune: state copy allocation failed");
        } else if (hipMemcpyAsync(saved[i], states[i], nb[i], hipMemcpyDeviceToDevice, g->st) != hipSuccess) {
            rc = fail(SDC_EHIP, "group autotune: state copy failed");
        }
    }
    float ms[2] = {0.f, 0.f};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == SDC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(SDC_EHIP, "hipEventCreate failed");
    for (int md = 1; md >= 0 && rc == SDC_OK; --md) {
        (void)sdc_group_set_mode(g, md);
        if ((rc = sdc_group_step(g, states, dts, M, K))) break;          // capture + warm-up
        if (hipEventRecord(e0, g->st) != hipSuccess) rc = fail(SDC_EHIP, "event record failed");
        for (int r = 0; r < reps && rc == SDC_OK; ++r) rc = sdc_group_step(g, states, dts, M, K);
        if (rc == SDC_OK && (hipEventRecord(e1, g->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms[md], e0, e1) != hipSuccess))
            rc = fail(SDC_EHIP, "group autotune timing failed");
    }
    for (size_t i = 0; i < n; ++i)
        if (saved[i]) {
            (void)hipMemcpyAsync(states[i], saved[i], nb[i], hipMemcpyDeviceToDevice, g->st);
            (void)hipStreamSynchronize(g->st);
            (void)hipFree(saved[i]);
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    (void)sdc_group_set_mode(g, ms[1] <= ms[0] ? 1 : 0);
    if (mode) *mode = g->mode;
    return SDC_OK;
}

int sdc_group_free(sdc_group g) {
    if (!g) return SDC_OK;
    (void)hipStreamSynchronize(g->st);
    delete g;
    return SDC_OK;
}

int sdc_group_step(sdc_group g, double* const* states, const double* dts, int M, int K) {
    if (!g) return fail(SDC_EINVAL, "group is NULL");
    if (!states || !dts) return fail(SDC_EINVAL, "states/dts is NULL");
    const size_t n = g->members.size();
    for (size_t i = 0; i < n; ++i)
        if (int rc = check_step_args(g->members[i], states[i], dts[i], M, K)) return rc;
    bool same = g->exec && g->key_M == M && g->key_K == K;
    for (size_t i = 0; same && i < n; ++i) same = g->key_states[i] == states[i] && g->key_dts[i] == dts[i];
    if (!same) {
        if (g->exec) {
            (void)hipGraphExecDestroy(g->exec);
            (void)hipGraphDestroy(g->graph);
            g->exec = nullptr;
            g->graph = nullptr;
        }
        hipGraph_t graph = nullptr;
        if (g->mode == 1) {
            std::string why;
            if (!group_mergeable(g, M, &why))
                return fail(SDC_EUNSUPPORTED, "one launch per phase over the members: %s (use mode 0)", why.c_str());
            if (int rc = group_capture_merged(g, states, dts, M, K, &graph)) return rc;
        } else if (int rc = group_capture_branches(g, states, dts, M, K, &graph)) {
            return rc;
        }
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(SDC_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        g->graph = graph;
        g->exec = exec;
        g->key_states.assign(states, states + n);
        g->key_dts.assign(dts, dts + n);
        g->key_M = M;
        g->key_K = K;
    }
    HIP_TRY(hipGraphLaunch(g->exec, g->st));
    return SDC_OK;
}

int sdc_group_sync(sdc_group g) {
    if (!g) return fail(SDC_EINVAL, "group is NULL");
    HIP_TRY(hipStreamSynchronize(g->st));
    int rc_all = SDC_OK;
    for (sdc_handle h : g->members) {
        const int rc = sdc_sync(h);
        if (rc != SDC_OK && rc_all == SDC_OK) rc_all = rc;
    }
    return rc_all;
}

}  // extern "C"
