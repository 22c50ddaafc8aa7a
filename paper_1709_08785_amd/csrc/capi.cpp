// The C ABI of include/wc.h: argument checks, lattice lifetime, operator
// applications and the per-kernel event timing.  Solvers live in solver.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

static thread_local std::string g_last_error;

int wc_fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

extern "C" const char *wc_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// allocation helpers
// ---------------------------------------------------------------------------
int dev_alloc(void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return wc_fail(WC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return WC_OK;
}

int buf_get(void **slot, size_t *have, size_t bytes, hipStream_t s) {
    if (*slot && *have >= bytes) return WC_OK;
    if (*slot) {
        WC_HIP(hipStreamSynchronize(s));
        WC_HIP(hipFree(*slot));
        *slot = nullptr;
        *have = 0;
    }
    if (int rc = dev_alloc(slot, bytes)) return rc;
    *have = bytes;
    return WC_OK;
}

int arena_alloc(Arena &a, int S, hipStream_t s) {
    a.S = S;
    const size_t nd = sizeof(double) * NUM_LEVELS * S_COUNT * S, ni = sizeof(int) * NUM_LEVELS * F_COUNT * S;
    if (int rc = dev_alloc((void **)&a.scalars, nd)) return rc;
    if (int rc = dev_alloc((void **)&a.flags, ni)) return rc;
    if (hipHostMalloc((void **)&a.h_scalars, nd, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&a.h_flags, ni, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return wc_fail(WC_ENOMEM, "pinned host allocation failed");
    }
    std::memset(a.h_scalars, 0, nd);
    std::memset(a.h_flags, 0, ni);
    WC_HIP(hipMemsetAsync(a.scalars, 0, nd, s));
    WC_HIP(hipMemsetAsync(a.flags, 0, ni, s));
    return WC_OK;
}

void arena_drop_graphs(Arena &a) {
    for (auto &g : a.graphs) (void)hipGraphExecDestroy(g.exec);
    a.graphs.clear();
}

void arena_free(Arena &a) {
    arena_drop_graphs(a);
    if (a.scalars) (void)hipFree(a.scalars);
    if (a.flags) (void)hipFree(a.flags);
    if (a.h_scalars) (void)hipHostFree(a.h_scalars);
    if (a.h_flags) (void)hipHostFree(a.h_flags);
    a = Arena{};
}

void arena_bind(Arena &a, int k, SysState &st) {
    st.scalars = a.scalars + (size_t)k * NUM_LEVELS * S_COUNT;
    st.flags = a.flags + (size_t)k * NUM_LEVELS * F_COUNT;
    st.h_scalars = a.h_scalars + (size_t)k * NUM_LEVELS * S_COUNT;
    st.h_flags = a.h_flags + (size_t)k * NUM_LEVELS * F_COUNT;
}

int sync_arena(const Arena &a, hipStream_t s) {
    WC_HIP(hipMemcpyAsync(a.h_scalars, a.scalars, sizeof(double) * NUM_LEVELS * S_COUNT * a.S, hipMemcpyDeviceToHost,
                          s));
    WC_HIP(hipMemcpyAsync(a.h_flags, a.flags, sizeof(int) * NUM_LEVELS * F_COUNT * a.S, hipMemcpyDeviceToHost, s));
    WC_HIP(hipStreamSynchronize(s));
    return WC_OK;
}

static int lwork(wc_lattice *lat, int id, size_t bytes, void **out) {
    if (int rc = buf_get(&lat->lwork[id], &lat->lwork_bytes[id], bytes, lat->stream)) return rc;
    *out = lat->lwork[id];
    return WC_OK;
}

static void free_work(SysWork &w) {
    for (int k = 0; k < W_SYS_COUNT; k++)
        if (w.buf[k]) (void)hipFree(w.buf[k]);
    w = SysWork{};
}

static void free_batch(BatchCache *b) {
    if (!b) return;
    arena_free(b->arena);
    for (auto &st : b->sys)
        if (st.partials) (void)hipFree(st.partials);
    for (auto &w : b->work) free_work(w);
    delete b;
}

// allocate (or keep) the solve vectors of one system on lattice lat; a moved
// buffer invalidates the graphs captured for the arena
static int ensure_work(wc_lattice *lat, SysWork &w, int iprec, bool pipe, Arena &arena) {
    const size_t d = spinor_bytes(P64, lat->Vh), i = spinor_bytes(iprec, lat->Vh),
                 x = spinor_bytes(iprec == P64 ? P64 : P32, lat->Vh), ip = pipe ? i : 0;
    const size_t need[W_SYS_COUNT] = {2 * d, 2 * d, d, d, d, d, d, d, d, d, d, i, i, i, i, i, i, x, ip, ip, ip, ip};
    for (int k = 0; k < W_SYS_COUNT; k++) {
        if (need[k] == 0) continue;  // not used by this solve
        void *before = w.buf[k];
        if (int rc = buf_get(&w.buf[k], &w.bytes[k], need[k], lat->stream)) return rc;
        if (w.buf[k] != before) arena_drop_graphs(arena);
    }
    return WC_OK;
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
static hipEvent_t take_event(wc_lattice *lat) {
    if (!lat->event_pool.empty()) {
        hipEvent_t e = lat->event_pool.back();
        lat->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timing_begin(wc_lattice *lat, int slot, double bytes, TimedLaunch &t) {
    t.slot = slot;
    t.bytes = bytes;
    t.a = take_event(lat);
    t.b = take_event(lat);
    if (t.a) (void)hipEventRecord(t.a, lat->stream);
}

void timing_end(wc_lattice *lat, TimedLaunch &t) {
    if (t.b) (void)hipEventRecord(t.b, lat->stream);
    if (t.a && t.b) lat->launches.push_back(t);
}

void timing_settle(wc_lattice *lat, size_t from, const std::vector<StopPoint> &stops) {
    auto stopped = [&](const int *fl, int iter, int phase) {
        for (const auto &sp : stops)
            if (sp.fl == fl) return iter > sp.iter || (iter == sp.iter && phase >= sp.phase);
        return false;
    };
    for (size_t k = from; k < lat->launches.size(); k++) {
        TimedLaunch &t = lat->launches[k];
        if (t.iter < 0 || t.parts.empty()) continue;
        double live = 0.0;
        for (const auto &part : t.parts) {
            bool any = false;
            for (const int *o : part.owners) any = any || !stopped(o, t.iter, t.phase);
            if (any) live += part.bytes;
        }
        t.bytes = live;
        t.skipped = live == 0.0;
    }
}

static const char *kSlotNames[KS_COUNT] = {
    "mult_hopinv_fp64", "mult_hopinv_fp32", "mult_hopinv_fp16", "mult_dhat_fp64",
    "mult_dhat_fp32",   "mult_dhat_fp16",   "mult_other",       "blas",
};

struct SlotStats {
    long n = 0;
    double ms = 0, bytes = 0;
};

static int collect_stats(wc_lattice *lat, SlotStats *st) {
    WC_HIP(hipStreamSynchronize(lat->stream));
    for (auto &t : lat->launches) {
        if (t.skipped) continue;  // converged systems only: the kernel returned at once
        float ms = 0.f;
        WC_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        st[t.slot].n++;
        st[t.slot].ms += ms;
        st[t.slot].bytes += t.bytes;
    }
    return WC_OK;
}

extern "C" int wc_set_barrier_timeout(double seconds) {
    if (!(seconds >= 0.0) || !std::isfinite(seconds)) return wc_fail(WC_EINVAL, "barrier timeout must be >= 0 and finite");
    g_barrier_timeout_s.store(seconds);
    return WC_OK;
}

extern "C" int wc_set_timing(wc_lattice *lat, int enable) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    lat->timing = enable != 0;
    return WC_OK;
}

extern "C" int wc_kernel_slots(void) { return KS_COUNT; }

extern "C" int wc_kernel_stats(wc_lattice *lat, int slot, const char **name, long *launches, double *total_ms,
                               double *total_bytes) {
    if (!lat || slot < 0 || slot >= KS_COUNT) return wc_fail(WC_EINVAL, "bad lattice or slot");
    SlotStats st[KS_COUNT];
    int rc = collect_stats(lat, st);
    if (rc) return rc;
    if (name) *name = kSlotNames[slot];
    if (launches) *launches = st[slot].n;
    if (total_ms) *total_ms = st[slot].ms;
    if (total_bytes) *total_bytes = st[slot].bytes;
    return WC_OK;
}

extern "C" int wc_reset_kernel_stats(wc_lattice *lat) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    WC_HIP(hipStreamSynchronize(lat->stream));
    for (auto &t : lat->launches) {
        lat->event_pool.push_back(t.a);
        lat->event_pool.push_back(t.b);
    }
    lat->launches.clear();
    return WC_OK;
}

// ---------------------------------------------------------------------------
// lattice lifetime
// ---------------------------------------------------------------------------
static void free_all(wc_lattice *lat) {
    for (int p = 0; p < 3; p++) {
        if (lat->links[p]) (void)hipFree(lat->links[p]);
        if (lat->clov[p]) (void)hipFree(lat->clov[p]);
        if (lat->clovinv[p]) (void)hipFree(lat->clovinv[p]);
    }
    if (lat->links8) (void)hipFree(lat->links8);
    if (lat->links18) (void)hipFree(lat->links18);
    if (lat->recon_min) (void)hipFree(lat->recon_min);
    if (lat->recon_err) (void)hipFree(lat->recon_err);
    if (lat->clov_bad) (void)hipFree(lat->clov_bad);
    for (int k = 0; k < LW_COUNT; k++)
        if (lat->lwork[k]) (void)hipFree(lat->lwork[k]);
    free_work(lat->swork);
    if (lat->sys.partials) (void)hipFree(lat->sys.partials);
    if (lat->sys.partials2) (void)hipFree(lat->sys.partials2);
    if (lat->sys.bar) (void)hipFree(lat->sys.bar);
    arena_free(lat->arena);
    free_batch(lat->batch);
    lat->batch = nullptr;
    for (auto &t : lat->launches) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : lat->event_pool) (void)hipEventDestroy(e);
    if (lat->capture_stream) (void)hipStreamDestroy(lat->capture_stream);
}

extern "C" int wc_create_lattice(const int dims[4], void *stream, wc_lattice **out) {
    if (!dims || !out) return wc_fail(WC_EINVAL, "null dims or out pointer");
    *out = nullptr;
    long V = 1;
    for (int d = 0; d < 4; d++) {
        if (dims[d] < 2 || (dims[d] & 1))
            return wc_fail(WC_EINVAL, "every lattice extent must be even and >= 2 (got " + std::to_string(dims[d]) +
                                          " in direction " + std::to_string(d) + ")");
        V *= dims[d];
    }
    if (V / 2 > (1L << 30)) return wc_fail(WC_EINVAL, "lattice too large (V/2 must fit in 30 bits)");
    static std::atomic<unsigned long long> next_serial{1};
    wc_lattice *lat = new wc_lattice();
    lat->serial = next_serial.fetch_add(1);
    for (int d = 0; d < 4; d++) {
        lat->dims[d] = dims[d];
        lat->g.L[d] = dims[d];
    }
    lat->V = V;
    lat->Vh = (int)(V / 2);
    lat->g.Lxh = dims[0] / 2;
    lat->g.Vh = lat->Vh;
    lat->stream = (hipStream_t)stream;
    lat->nblocks = (lat->Vh + 255) / 256;
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
            lat->lds_per_cu = lds;  // left 0 (no wave cap) if the device does not say
    }
    int rc = arena_alloc(lat->arena, 1, lat->stream);
    if (!rc) {
        arena_bind(lat->arena, 0, lat->sys);
        rc = dev_alloc((void **)&lat->sys.partials,
                       sizeof(double) * kMaxRed * (size_t)blocks_of(lat->Vh, kMinBlock));
        if (!rc) rc = dev_alloc((void **)&lat->sys.partials2, sizeof(double) * kMaxRed * (size_t)lat->nblocks);
        const size_t bar_bytes = sizeof(unsigned long long) * ((size_t)lat->nblocks + 2);
        if (!rc) rc = dev_alloc((void **)&lat->sys.bar, bar_bytes);
        if (!rc && hipMemsetAsync(lat->sys.bar, 0, bar_bytes, lat->stream) != hipSuccess)
            rc = wc_fail(WC_EHIP, "clearing the grid barrier words");
    }
    if (!rc && hipStreamSynchronize(lat->stream) != hipSuccess)
        rc = wc_fail(WC_EHIP, std::string("initialising lattice scratch: ") + hipGetErrorString(hipGetLastError()));
    if (rc) {
        free_all(lat);
        delete lat;
        return rc;
    }
    *out = lat;
    return WC_OK;
}

extern "C" void wc_destroy_lattice(wc_lattice *lat) {
    if (!lat) return;
    (void)hipStreamSynchronize(lat->stream);
    free_all(lat);
    delete lat;
}

extern "C" int wc_set_stream(wc_lattice *lat, void *stream) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    lat->stream = (hipStream_t)stream;
    return WC_OK;
}

extern "C" void wc_solve_params_default(wc_solve_params *p) {
    if (!p) return;
    p->inner_prec = WC_FP32;
    p->inner_tol = 0.0;  // 0 = default of the precision
    p->inner_maxit = 5000;
    p->outer_maxit = 100;
    p->fixed_work = 0;
    p->check_every = 8;
    p->adjoint = 0;
    p->use_graph = 1;
    p->outer = WC_OUTER_BICGSTAB;
    p->inner_method = WC_INNER_BICGSTAB;
    p->persistent = 0;
}

static int check_links_for(const wc_lattice *lat, int prec);

static int check_params(const wc_solve_params &P, double tol) {
    if (!(tol > 0.0) || !(tol < 1.0)) return wc_fail(WC_EINVAL, "tol must lie in (0, 1)");
    if (P.inner_prec < 0 || P.inner_prec > 2) return wc_fail(WC_EINVAL, "bad inner precision");
    if (P.inner_maxit < 1 || P.outer_maxit < 1 || P.check_every < 1 || P.fixed_work < 0 || P.inner_tol < 0.0 ||
        P.inner_tol >= 1.0)
        return wc_fail(WC_EINVAL, "bad solver parameters");
    if (P.outer != WC_OUTER_BICGSTAB && P.outer != WC_OUTER_DC) return wc_fail(WC_EINVAL, "bad outer method");
    if (P.inner_method != WC_INNER_BICGSTAB && P.inner_method != WC_INNER_PIPELINED)
        return wc_fail(WC_EINVAL, "bad inner method");
    return WC_OK;
}

static int prepare_lattice(wc_lattice *lat, double kappa, double csw) {
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "solve before wc_load_links");
    if (!lat->have_clover || lat->kappa != kappa || lat->csw != csw)
        if (int rc = wc_build_clover(lat, kappa, csw)) return rc;
    return WC_OK;
}

static int report(std::vector<SolveSys> &sys, wc_solve_info *info) {
    int worst = WC_OK;
    for (size_t k = 0; k < sys.size(); k++) {
        if (info) info[k] = sys[k].info;
        if (sys[k].status != WC_OK && worst == WC_OK) worst = sys[k].status;
    }
    if (worst != WC_OK) {
        double r = 0;
        for (auto &s : sys) r = std::max(r, s.info.true_rel_residual);
        return wc_fail(worst, "solve stopped at true relative residual " + std::to_string(r));
    }
    return WC_OK;
}

extern "C" int wc_solve(wc_lattice *lat, const void *b_dev, double kappa, double csw, double tol,
                        const wc_solve_params *pin, void *x_dev, int x0_is_guess, wc_solve_info *info) {
    if (!lat || !b_dev || !x_dev) return wc_fail(WC_EINVAL, "null argument");
    wc_solve_params P;
    wc_solve_params_default(&P);
    if (pin) P = *pin;
    if (int rc = check_params(P, tol)) return rc;
    if (int rc = check_links_for(lat, P.inner_prec)) return rc;
    if (int rc = prepare_lattice(lat, kappa, csw)) return rc;
    if (int rc = ensure_work(lat, lat->swork, P.inner_prec, P.inner_method == WC_INNER_PIPELINED, lat->arena)) return rc;
    std::vector<SolveSys> sys(1);
    sys[0].lat = lat;
    sys[0].st = &lat->sys;
    sys[0].work = &lat->swork;
    sys[0].b_dev = b_dev;
    sys[0].x_dev = x_dev;
    sys[0].kappa = kappa;
    sys[0].csw = csw;
    if (int rc = solve_systems(sys, lat->arena, tol, P, x0_is_guess)) return rc;
    return report(sys, info);
}

extern "C" int wc_solve_multi(int n, wc_lattice *const *lats, const void *const *b_dev, void *const *x_dev,
                              const double *kappa, const double *csw, double tol, const wc_solve_params *pin,
                              wc_solve_info *info) {
    if (n < 1 || n > kMaxSys) return wc_fail(WC_EINVAL, "n must lie in [1, 16]");
    if (!lats || !b_dev || !x_dev || !kappa || !csw) return wc_fail(WC_EINVAL, "null argument");
    for (int k = 0; k < n; k++)
        if (!lats[k] || !b_dev[k] || !x_dev[k]) return wc_fail(WC_EINVAL, "null lattice or field");
    wc_solve_params P;
    wc_solve_params_default(&P);
    if (pin) P = *pin;
    if (int rc = check_params(P, tol)) return rc;
    for (int k = 0; k < n; k++) {
        for (int j = 0; j < k; j++)
            if (lats[j] == lats[k] && (kappa[j] != kappa[k] || csw[j] != csw[k]))
                return wc_fail(WC_EINVAL, "systems on one lattice must share kappa and csw");
        if (lats[k]->recon != lats[0]->recon)
            return wc_fail(WC_EINVAL, "lattices of one batched solve must share the link reconstruction");
        if (int rc = check_links_for(lats[k], P.inner_prec)) return rc;
    }
    wc_lattice *lead = lats[0];
    // Every lattice works on the lead lattice's stream for the duration.  Work
    // already queued on another lattice's own stream is ordered before it by
    // an event, and the clover rebuilds below then run on the lead stream too,
    // so nothing of the solve can overtake them.
    std::vector<hipStream_t> saved(n);
    for (int k = 0; k < n; k++) saved[k] = lats[k]->stream;
    auto restore = [&] {
        for (int k = 0; k < n; k++) lats[k]->stream = saved[k];
    };
    {
        hipEvent_t ev = nullptr;
        for (int k = 0; k < n; k++) {
            bool seen = saved[k] == lead->stream;
            for (int j = 0; j < k && !seen; j++) seen = saved[j] == saved[k];
            if (seen) continue;
            if (!ev) WC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            hipError_t e = hipEventRecord(ev, saved[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(lead->stream, ev, 0);
            if (e != hipSuccess) {
                (void)hipEventDestroy(ev);
                return wc_fail(WC_EHIP, std::string("ordering the lattices' streams: ") + hipGetErrorString(e));
            }
        }
        if (ev) WC_HIP(hipEventDestroy(ev));
    }
    for (int k = 0; k < n; k++) lats[k]->stream = lead->stream;
    for (int k = 0; k < n; k++)
        if (int rc = prepare_lattice(lats[k], kappa[k], csw[k])) {
            restore();
            return rc;
        }
    // the cached systems are reused only for the same lattices, named by their
    // serial numbers: a destroyed lattice's address may come back with a new one
    BatchCache *bc = lead->batch;
    bool reuse = bc && (int)bc->serials.size() == n;
    for (int k = 0; reuse && k < n; k++) reuse = bc->serials[k] == lats[k]->serial;
    if (!reuse) {
        free_batch(bc);
        lead->batch = bc = new BatchCache();
        for (int k = 0; k < n; k++) bc->serials.push_back(lats[k]->serial);
        bc->sys.resize(n);
        bc->work.resize(n);
        if (int rc = arena_alloc(bc->arena, n, lead->stream)) {
            restore();
            return rc;
        }
        for (int k = 0; k < n; k++) {
            arena_bind(bc->arena, k, bc->sys[k]);
            if (int rc = buf_get((void **)&bc->sys[k].partials, &bc->sys[k].partials_bytes,
                                 sizeof(double) * kMaxRed * (size_t)blocks_of(lats[k]->Vh, kMinBlock),
                                 lead->stream)) {
                restore();
                return rc;
            }
        }
    }
    std::vector<SolveSys> sys(n);
    for (int k = 0; k < n; k++) {
        if (int rc = ensure_work(lats[k], bc->work[k], P.inner_prec, P.inner_method == WC_INNER_PIPELINED, bc->arena)) {
            restore();
            return rc;
        }
        sys[k].lat = lats[k];
        sys[k].st = &bc->sys[k];
        sys[k].work = &bc->work[k];
        sys[k].b_dev = b_dev[k];
        sys[k].x_dev = x_dev[k];
        sys[k].kappa = kappa[k];
        sys[k].csw = csw[k];
    }
    int rc = solve_systems(sys, bc->arena, tol, P, 0);
    restore();
    if (rc) return rc;
    return report(sys, info);
}

extern "C" int wc_solve_batch(wc_lattice *lat, int n, const void *const *b_dev, void *const *x_dev, double kappa,
                              double csw, double tol, const wc_solve_params *p, wc_solve_info *info) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (n < 1 || n > kMaxSys) return wc_fail(WC_EINVAL, "n must lie in [1, 16]");
    wc_lattice *lats[kMaxSys];
    double ks[kMaxSys], cs[kMaxSys];
    for (int k = 0; k < n; k++) {
        lats[k] = lat;
        ks[k] = kappa;
        cs[k] = csw;
    }
    return wc_solve_multi(n, lats, b_dev, x_dev, ks, cs, tol, p, info);
}

extern "C" size_t wc_spinor_bytes(const wc_lattice *lat, int prec) {
    if (!lat || prec < 0 || prec > 2) return 0;
    return spinor_bytes(prec, lat->Vh);
}

// reconstruct-8 copies of the current links; refuses links whose first row
// puts (almost) all its weight on U00, where the parametrisation breaks down
static int build_recon8(wc_lattice *lat) {
    if (!lat->links8) {
        int rc = dev_alloc(&lat->links8, 8 * link8_slab_bytes(lat->Vh));
        if (rc) return rc;
    }
    if (!lat->recon_min) {
        int rc = dev_alloc((void **)&lat->recon_min, sizeof(unsigned));
        if (rc) return rc;
    }
    const unsigned init = 0x7f7fffffu;  // FLT_MAX
    WC_HIP(hipMemcpyAsync(lat->recon_min, &init, sizeof(init), hipMemcpyHostToDevice, lat->stream));
    if (int rc = launch_links_recon8(lat, lat->recon_min)) return rc;
    unsigned bits = 0;
    WC_HIP(hipMemcpyAsync(&bits, lat->recon_min, sizeof(bits), hipMemcpyDeviceToHost, lat->stream));
    WC_HIP(hipStreamSynchronize(lat->stream));
    float nmin;
    std::memcpy(&nmin, &bits, sizeof(nmin));
    if (!(nmin >= kRecon8MinN))
        return wc_fail(WC_EINVAL, "reconstruct-8 needs |U01|^2 + |U02|^2 >= " + std::to_string(kRecon8MinN) +
                                      " on every link; smallest found: " + std::to_string(nmin));
    return WC_OK;
}

// the full FP32 copies of the current links
static int build_full32(wc_lattice *lat) {
    if (!lat->links18) {
        int rc = dev_alloc(&lat->links18, 8 * link18_slab_bytes(lat->Vh));
        if (rc) return rc;
    }
    return launch_links_full32(lat);
}

static void set_recon(wc_lattice *lat, int recon, bool automatic) {
    if (recon != lat->recon) {
        lat->recon = recon;
        lat->bs_tuned[P32] = 0;  // the FP32 stencil changed: tune again
        lat->chunk_tuned[P32] = -1;
        lat->cap_tuned[P32][0] = lat->cap_tuned[P32][1] = -1;
        lat->gen++;
    }
    lat->recon_auto = automatic;
}

extern "C" int wc_load_links(wc_lattice *lat, const void *U_dev) {
    if (!lat || !U_dev) return wc_fail(WC_EINVAL, "null lattice or link pointer");
    for (int p = 0; p < 3; p++) {
        if (!lat->links[p]) {
            int rc = dev_alloc(&lat->links[p], 8 * link_slab_bytes(p, lat->Vh));
            if (rc) return rc;
        }
    }
    if (!lat->recon_err) {
        int rc = dev_alloc((void **)&lat->recon_err, sizeof(unsigned));
        if (rc) return rc;
    }
    WC_HIP(hipMemsetAsync(lat->recon_err, 0, sizeof(unsigned), lat->stream));
    int rc = launch_load_links(lat, U_dev, lat->recon_err);
    if (rc) return rc;
    unsigned bits = 0;
    WC_HIP(hipMemcpyAsync(&bits, lat->recon_err, sizeof(bits), hipMemcpyDeviceToHost, lat->stream));
    WC_HIP(hipStreamSynchronize(lat->stream));
    std::memcpy(&lat->su3_err, &bits, sizeof(bits));
    lat->gen++;
    lat->have_clover = false;
    if (!std::isfinite(lat->su3_err)) {
        lat->have_links = false;  // the copies now hold the bad entries
        lat->su3_err = 0.f;
        return wc_fail(WC_EINVAL, "the links have non-finite entries");
    }
    lat->have_links = true;
    if (lat->su3_err > kSU3MaxErr) {
        // not SU(3) to single precision: no two-column form holds, so the
        // FP32 stencil reads the links in full (FP16 is refused)
        if (int r = build_full32(lat)) return r;
        if (lat->recon != 18) set_recon(lat, 18, true);
        return WC_OK;
    }
    if (lat->recon_auto) set_recon(lat, lat->recon_user, false);  // SU(3) again: the caller's form
    if (lat->recon == 18) return build_full32(lat);
    if (lat->recon == 8) {
        // keep the reconstruct-8 copies in step; links they cannot hold switch it off
        rc = build_recon8(lat);
        if (rc) {
            set_recon(lat, 12, false);
            lat->recon_user = 12;
        }
        return rc;
    }
    return WC_OK;
}

extern "C" int wc_set_link_recon(wc_lattice *lat, int recon) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (recon != 12 && recon != 8 && recon != 18) return wc_fail(WC_EINVAL, "link form must be 12, 8 or 18");
    if (recon != 18 && lat->have_links && lat->su3_err > kSU3MaxErr)
        return wc_fail(WC_EINVAL, "the loaded links are not SU(3) to single precision (largest third-column error " +
                                      std::to_string(lat->su3_err) + "); only the full form 18 holds them");
    if (recon == lat->recon) {
        lat->recon_auto = false;
        lat->recon_user = recon;
        return WC_OK;
    }
    if (recon == 8) {
        if (!lat->have_links) return wc_fail(WC_ENOTREADY, "wc_set_link_recon(8) before wc_load_links");
        if (int rc = build_recon8(lat)) return rc;
    }
    if (recon == 18) {
        if (!lat->have_links) return wc_fail(WC_ENOTREADY, "wc_set_link_recon(18) before wc_load_links");
        if (int rc = build_full32(lat)) return rc;
    }
    set_recon(lat, recon, false);
    lat->recon_user = recon;
    return WC_OK;
}

extern "C" double wc_link_su3_error(const wc_lattice *lat) { return lat ? (double)lat->su3_err : -1.0; }

extern "C" int wc_link_recon(const wc_lattice *lat) { return lat ? lat->recon : 0; }

extern "C" int wc_build_clover(wc_lattice *lat, double kappa, double csw) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "wc_build_clover before wc_load_links");
    if (!(kappa >= 0.0) || !(csw >= 0.0) || !std::isfinite(kappa) || !std::isfinite(csw))
        return wc_fail(WC_EINVAL, "need finite kappa >= 0 and csw >= 0");
    for (int p = 0; p < 3; p++) {
        if (!lat->clov[p]) {
            int rc = dev_alloc(&lat->clov[p], 2 * clover_slab_bytes(p, lat->Vh));
            if (rc) return rc;
        }
        if (!lat->clovinv[p]) {
            int rc = dev_alloc(&lat->clovinv[p], 2 * clover_slab_bytes(p, lat->Vh));
            if (rc) return rc;
        }
    }
    if (!lat->clov_bad) {
        int rc = dev_alloc((void **)&lat->clov_bad, sizeof(unsigned));
        if (rc) return rc;
    }
    // whatever happens below, the blocks being overwritten are no longer the
    // clover term of any (kappa, csw)
    lat->have_clover = false;
    lat->gen++;
    WC_HIP(hipMemsetAsync(lat->clov_bad, 0, sizeof(unsigned), lat->stream));
    int rc = launch_build_clover(lat, kappa, csw, lat->clov_bad);
    if (rc) return rc;
    unsigned bad = 0;
    WC_HIP(hipMemcpyAsync(&bad, lat->clov_bad, sizeof(bad), hipMemcpyDeviceToHost, lat->stream));
    WC_HIP(hipStreamSynchronize(lat->stream));
    if (bad)
        return wc_fail(WC_EINVAL, std::to_string(bad) + " of the " + std::to_string(2 * lat->V) +
                                      " 6x6 clover blocks are not positive definite at kappa = " +
                                      std::to_string(kappa) + ", csw = " + std::to_string(csw) +
                                      " (a non-positive or non-finite elimination pivot)");
    lat->kappa = kappa;
    lat->csw = csw;
    lat->have_clover = true;
    return WC_OK;
}

static int check_prec(int prec) {
    if (prec < 0 || prec > 2) return wc_fail(WC_EINVAL, "precision must be WC_FP64, WC_FP32 or WC_FP16");
    return WC_OK;
}

// the FP16 stencil keeps two link columns, valid for SU(3) links only
static int check_links_for(const wc_lattice *lat, int prec) {
    if (prec == WC_FP16 && lat->have_links && lat->su3_err > kSU3MaxErr)
        return wc_fail(WC_EINVAL, "the loaded links are not SU(3) to single precision (largest third-column error " +
                                      std::to_string(lat->su3_err) + "); the FP16 stencil keeps two columns");
    return WC_OK;
}

static int check_ready(const wc_lattice *lat) {
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "no links loaded");
    if (!lat->have_clover) return wc_fail(WC_ENOTREADY, "no clover term built");
    return WC_OK;
}

extern "C" int wc_pack_spinor(wc_lattice *lat, void *eo_out, const void *canon_in, int prec) {
    if (!lat || !eo_out || !canon_in) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    return launch_pack_spinor(lat, prec, eo_out, canon_in);
}

extern "C" int wc_unpack_spinor(wc_lattice *lat, void *canon_out, const void *eo_in, int prec) {
    if (!lat || !canon_out || !eo_in) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    return launch_unpack_spinor(lat, prec, canon_out, eo_in);
}

static MultCall mult_call(int prec, int mode, int out_par, void *out, const void *in, const void *center,
                          double coef) {
    MultCall c;
    std::memset(&c, 0, sizeof(c));
    c.prec = prec;
    c.mode = mode;
    c.red = R_NONE;
    c.out_par = out_par;
    c.out = out;
    c.in = in;
    c.center = center;
    c.aux = nullptr;
    c.coef = coef;
    c.inverse = false;
    c.done = nullptr;
    return c;
}

// ---------------------------------------------------------------------------
// launch-shape tuner and its persistent cache
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::string g_tune_cache;  // file of tuned shapes ("" = none)

extern "C" int wc_set_tune_cache(const char *path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache = path ? path : "";
    return WC_OK;
}

// the cache key of (device, lattice, precision, link form, pinned waves per CU or -1)
static std::string tune_key(const wc_lattice *lat, int prec) {
    int dev = 0;
    hipDeviceProp_t p;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        cus = p.multiProcessorCount;
    }
    for (auto &ch : arch)
        if (ch == ' ') ch = '_';
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s %d %d %d %d %d %d %d %d", arch.c_str(), cus, lat->dims[0], lat->dims[1],
                  lat->dims[2], lat->dims[3], prec, prec == P32 ? lat->recon : 12, lat->wave_cap[prec]);
    return buf;
}

// the last entry for key in the cache file: block size, chunk, wave caps of
// the two kernel classes, microseconds per pair at the block sizes 64, 128, 256
static bool tune_lookup(const std::string &key, int *bs, int *chunk, int caps[2], double us[3]) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_tune_cache.empty()) return false;
    std::FILE *f = std::fopen(g_tune_cache.c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string head = "wc-tune-v3 " + key + " ";
    while (std::fgets(line, sizeof(line), f)) {
        if (std::strncmp(line, head.c_str(), head.size()) != 0) continue;
        int b = 0, c = -1, w0 = -1, w1 = -1;
        double u[3] = {0, 0, 0};
        if (std::sscanf(line + head.size(), "%d %d %d %d %lf %lf %lf", &b, &c, &w0, &w1, &u[0], &u[1], &u[2]) == 7 &&
            valid_block_size(b) && c >= 0 && valid_wave_cap(w0) && valid_wave_cap(w1)) {
            *bs = b;
            *chunk = c;
            caps[0] = w0;
            caps[1] = w1;
            for (int k = 0; k < 3; k++) us[k] = u[k];
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_store(const std::string &key, int bs, int chunk, const int caps[2], const double us[3]) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_tune_cache.empty()) return;
    std::FILE *f = std::fopen(g_tune_cache.c_str(), "a");
    if (!f) return;  // a cache that cannot be written only costs a later tuning
    std::fprintf(f, "wc-tune-v3 %s %d %d %d %d %.3f %.3f %.3f\n", key.c_str(), bs, chunk, caps[0], caps[1], us[0], us[1],
                 us[2]);
    std::fclose(f);
}

// Time the inner loop's stencil pair (F_oo^-1 H_oe into the odd parity, then
// the D-hat half with its fused dot) on zero vectors at each block size and
// XCD chunk, and keep the fastest.  The default shape (256 threads, chunk
// kDefaultChunk) is displaced only by a shape at least 3% faster, in the
// sweep and again in three alternating timings against it, so that timing
// noise does not flip the choice on large lattices.  A pinned chunk is the
// only one timed.  Then, unless the caller pinned a wave cap, the two kernels
// are timed on their own at the chosen shape under caps of 0, 8 and 12 waves
// per CU, and each keeps the cap that beats the precision's default by 3%,
// again confirmed by alternating timings.  With a cache file set, a stored
// result for the same device, lattice, precision, link form and pinned cap
// is taken instead of timing.  A pinned block size or chunk bypasses the file
// both ways: a stored shape was chosen over every size and chunk, and a
// constrained choice must not be handed to a later, unconstrained tuning.
int tune_block_size(wc_lattice *lat, int prec, double us[3], int *chosen) {
    if (!lat->have_links || !lat->have_clover)
        return wc_fail(WC_ENOTREADY, "block-size tuning needs links and clover");
    const std::string key = tune_key(lat, prec);
    const bool use_cache = !lat->bs_pin && lat->chunk_pin < 0;
    if (use_cache) {
        int b = 0, c = -1, w[2] = {-1, -1};
        double u[3];
        if (tune_lookup(key, &b, &c, w, u)) {
            lat->bs_tuned[prec] = b;
            lat->chunk_tuned[prec] = c;
            lat->cap_tuned[prec][0] = w[0];
            lat->cap_tuned[prec][1] = w[1];
            lat->gen++;
            if (us)
                for (int k = 0; k < 3; k++) us[k] = u[k];
            if (chosen) *chosen = b;
            return WC_OK;
        }
    }
    const size_t sb = spinor_bytes(prec, lat->Vh);
    char *buf = nullptr;
    const size_t bytes = 3 * sb + 256;
    if (int rc = dev_alloc((void **)&buf, bytes)) return rc;
    int rc = WC_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timing = lat->timing;
    const long dcount = lat->dslash_count;
    lat->timing = false;
    // the block size and chunk are timed under the precision's default cap
    lat->cap_tuned[prec][0] = lat->cap_tuned[prec][1] = -1;
    const int cand[3] = {64, 128, 256};
    std::vector<int> chunks;
    if (lat->chunk_pin >= 0) chunks.push_back(lat->chunk_pin);
    else chunks = {kDefaultChunk, 8, 16, 64};
    std::vector<double> t(3 * chunks.size(), 0.0);
    size_t best = 2;
    int caps[2] = {default_wave_cap(prec), default_wave_cap(prec)};
    // which: 3 = the pair, 1 = the MULT alone, 2 = the D-hat half alone
    auto pair = [&](int bs, int which) -> int {
        if (which & 1) {
            MultCall c1 = mult_call(prec, M_HOPINV, 1, buf + sb, buf, nullptr, 0.0);
            c1.bs = bs;
            if (int r = launch_mult(lat, c1)) return r;
        }
        if (which & 2) {
            MultCall c2 = mult_call(prec, M_DHAT, 0, buf + 2 * sb, buf + sb, buf, -lat->kappa * lat->kappa);
            c2.bs = bs;
            c2.red = R_DOT;
            c2.aux = buf;
            c2.red_to = RedTarget{lat->sys.partials, (double *)(buf + 3 * sb)};
            if (int r = launch_mult(lat, c2)) return r;
        }
        return WC_OK;
    };
    auto timed = [&](int bs, int reps, double *ms, int which = 3) -> int {
        for (int w = 0; w < 2; w++)
            if (int r = pair(bs, which)) return r;
        WC_HIP(hipEventRecord(e0, lat->stream));
        for (int r = 0; r < reps; r++)
            if (int q = pair(bs, which)) return q;
        WC_HIP(hipEventRecord(e1, lat->stream));
        WC_HIP(hipEventSynchronize(e1));
        float f = 0.f;
        WC_HIP(hipEventElapsedTime(&f, e0, e1));
        *ms = f / reps;
        return WC_OK;
    };
    do {
        if (hipMemsetAsync(buf, 0, bytes, lat->stream) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = wc_fail(WC_EHIP, "block-size tuning: setting up buffers and events");
            break;
        }
        // about 2 ms of pairs per candidate, between 4 and 64
        double ms = 0;
        lat->chunk_force = chunks[0];
        if ((rc = timed(256, 2, &ms))) break;
        const int reps = std::max(4, std::min(64, (int)(2.0 / std::max(ms, 1e-3))));
        for (size_t h = 0; h < chunks.size() && !rc; h++) {
            lat->chunk_force = chunks[h];
            for (int c = 0; c < 3 && !rc; c++) rc = timed(cand[c], reps, &t[3 * h + c]);
        }
        if (rc) break;
        // start from 256 threads (or the pinned size) at the first chunk;
        // another shape must win by 3%.  A pinned block size is the only one
        // the choice of chunk and caps considers.
        const int pin = lat->bs_pin;
        const size_t start = pin ? (pin == 64 ? 0 : pin == 128 ? 1 : 2) : 2;
        best = start;
        for (size_t k = 0; k < t.size(); k++)
            if ((!pin || cand[k % 3] == pin) && t[k] < 0.97 * t[best]) best = k;
        // One timing of about 2 ms can favour a shape by a few percent by
        // chance, so a challenger is timed again against the starting shape,
        // alternately, three times each, and keeps its place only if the
        // better of its times still wins by 3%.
        auto confirm = [&](auto run_a, auto run_b, bool *b_wins) -> int {
            double ta = 1e30, tb = 1e30, m = 0;
            for (int k = 0; k < 3; k++) {
                if (int r = run_a(&m)) return r;
                ta = std::min(ta, m);
                if (int r = run_b(&m)) return r;
                tb = std::min(tb, m);
            }
            *b_wins = tb < 0.97 * ta;
            return WC_OK;
        };
        if (best != start) {
            bool wins = false;
            rc = confirm(
                [&](double *m) {
                    lat->chunk_force = chunks[start / 3];
                    return timed(cand[start % 3], reps, m);
                },
                [&](double *m) {
                    lat->chunk_force = chunks[best / 3];
                    return timed(cand[best % 3], reps, m);
                },
                &wins);
            if (rc) break;
            if (!wins) best = start;
        }
        // the wave cap of each kernel class at that shape
        if (lat->wave_cap[prec] >= 0 || lat->lds_per_cu <= 0) break;
        lat->chunk_force = chunks[best / 3];
        const int bsb = cand[best % 3];
        const int def = default_wave_cap(prec);
        double tk[2];
        lat->cap_force = def;
        for (int j = 0; j < 2 && !rc; j++) rc = timed(bsb, reps, &tk[j], j + 1);
        for (int cap : {0, 8, 12}) {
            if (cap == def || rc) continue;
            lat->cap_force = cap;
            for (int j = 0; j < 2 && !rc; j++) {
                double tc = 0;
                rc = timed(bsb, reps, &tc, j + 1);
                if (!rc && tc < 0.97 * tk[j]) {
                    tk[j] = tc;
                    caps[j] = cap;
                }
            }
        }
        for (int j = 0; j < 2 && !rc; j++) {
            if (caps[j] == def) continue;
            bool wins = false;
            rc = confirm(
                [&](double *m) {
                    lat->cap_force = def;
                    return timed(bsb, reps, m, j + 1);
                },
                [&](double *m) {
                    lat->cap_force = caps[j];
                    return timed(bsb, reps, m, j + 1);
                },
                &wins);
            if (!rc && !wins) caps[j] = def;
        }
    } while (false);
    lat->chunk_force = -1;
    lat->cap_force = -1;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(lat->stream);
    (void)hipFree(buf);
    lat->timing = timing;
    lat->dslash_count = dcount;
    if (rc) return rc;
    const size_t h = best / 3;
    lat->bs_tuned[prec] = cand[best % 3];
    lat->chunk_tuned[prec] = chunks[h];
    if (lat->wave_cap[prec] < 0) {
        lat->cap_tuned[prec][0] = caps[0];
        lat->cap_tuned[prec][1] = caps[1];
    }
    lat->gen++;  // captured graphs hold the old launch shape
    double u[3];
    for (int c = 0; c < 3; c++) u[c] = t[3 * h + c] * 1e3;
    if (us)
        for (int c = 0; c < 3; c++) us[c] = u[c];
    if (chosen) *chosen = cand[best % 3];
    if (use_cache) tune_store(key, cand[best % 3], chunks[h], caps, u);
    return WC_OK;
}

extern "C" int wc_set_block_size(wc_lattice *lat, int threads) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (threads != 0 && !valid_block_size(threads)) return wc_fail(WC_EINVAL, "block size must be 0, 64, 128 or 256");
    if (threads != lat->bs_pin) lat->gen++;
    lat->bs_pin = threads;
    return WC_OK;
}

extern "C" int wc_set_multi_rhs(wc_lattice *lat, int systems_per_thread) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (systems_per_thread != -1 && systems_per_thread != 0 && systems_per_thread != 2 && systems_per_thread != 4)
        return wc_fail(WC_EINVAL, "systems per thread must be -1, 0, 2 or 4");
    if (systems_per_thread != lat->mrhs) lat->gen++;  // recorded graphs hold the old kernels
    lat->mrhs = systems_per_thread;
    return WC_OK;
}

extern "C" int wc_multi_rhs(const wc_lattice *lat, int prec) {
    if (!lat || prec < 0 || prec > 2) return -1;
    return prec == P64 ? 0 : mrhs_for(lat, prec);
}

extern "C" int wc_set_xcd_chunk(wc_lattice *lat, int tiles) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (tiles < -1 || tiles > (1 << 20)) return wc_fail(WC_EINVAL, "XCD chunk must be -1 or lie in [0, 2^20] tiles");
    if (tiles != lat->chunk_pin) lat->gen++;  // recorded graphs hold the old launch arguments
    lat->chunk_pin = tiles;
    return WC_OK;
}

extern "C" int wc_xcd_chunk(const wc_lattice *lat, int prec) {
    if (!lat || prec < 0 || prec > 2) return -2;
    return lattice_chunk(lat, prec);
}

extern "C" int wc_set_wave_cap(wc_lattice *lat, int prec, int waves_per_cu) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (int rc = check_prec(prec)) return rc;
    if (waves_per_cu != -1 && !valid_wave_cap(waves_per_cu))
        return wc_fail(WC_EINVAL, "waves per CU must be -1 (default), 0 (no cap), 4, 8, 12 or 16");
    if (waves_per_cu != lat->wave_cap[prec]) {
        lat->gen++;  // recorded graphs hold the old launch shape
        lat->bs_tuned[prec] = 0;  // the tuned shape was timed under the old cap
        lat->chunk_tuned[prec] = -1;
        lat->cap_tuned[prec][0] = lat->cap_tuned[prec][1] = -1;
    }
    lat->wave_cap[prec] = waves_per_cu;
    return WC_OK;
}

extern "C" int wc_wave_cap(const wc_lattice *lat, int prec, int dhat) {
    if (!lat || prec < 0 || prec > 2) return -2;
    return lat->lds_per_cu > 0 ? wave_cap_for(lat, prec, dhat ? M_DHAT : M_HOPINV) : 0;
}

extern "C" int wc_block_size(const wc_lattice *lat, int prec) {
    if (!lat || prec < 0 || prec > 2) return 0;
    return lat->bs_pin ? lat->bs_pin : lat->bs_tuned[prec];
}

extern "C" int wc_tune_block_size(wc_lattice *lat, int prec, double us_per_pair[3], int *threads) {
    if (!lat) return wc_fail(WC_EINVAL, "null lattice");
    if (int rc = check_prec(prec)) return rc;
    return tune_block_size(lat, prec, us_per_pair, threads);
}


extern "C" int wc_apply_D(wc_lattice *lat, void *out_dev, const void *in_dev, int prec) {
    if (!lat || !out_dev || !in_dev) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    if (prec == WC_FP16) return wc_fail(WC_EINVAL, "wc_apply_D supports WC_FP64 and WC_FP32");
    if (int rc = check_ready(lat)) return rc;
    const size_t sb = spinor_bytes(prec, lat->Vh);
    void *in2, *out2;
    if (int rc = lwork(lat, LW_APPLY_IN, 2 * sb, &in2)) return rc;
    if (int rc = lwork(lat, LW_APPLY_OUT, 2 * sb, &out2)) return rc;
    if (int rc = launch_pack_spinor(lat, prec, in2, in_dev)) return rc;
    for (int par = 0; par < 2; par++) {
        MultCall c = mult_call(prec, M_DFULL, par, (char *)out2 + par * sb, (const char *)in2 + (1 - par) * sb,
                               (const char *)in2 + par * sb, -lat->kappa);
        if (int rc = launch_mult(lat, c)) return rc;
    }
    return launch_unpack_spinor(lat, prec, out_dev, out2);
}

extern "C" int wc_apply_mult(wc_lattice *lat, void *out, const void *in, int out_parity, int prec) {
    if (!lat || !out || !in) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    if (out_parity != 0 && out_parity != 1) return wc_fail(WC_EINVAL, "out_parity must be 0 or 1");
    if (int rc = check_ready(lat)) return rc;
    if (int rc = check_links_for(lat, prec)) return rc;
    MultCall c = mult_call(prec, M_HOPINV, out_parity, out, in, nullptr, 0.0);
    return launch_mult(lat, c);
}

extern "C" int wc_apply_mult_batch(wc_lattice *lat, int n, void *const *out, const void *const *in, int out_parity,
                                   int prec) {
    if (!lat || !out || !in) return wc_fail(WC_EINVAL, "null argument");
    if (n < 1 || n > kMaxSys) return wc_fail(WC_EINVAL, "n must lie in [1, 16]");
    for (int k = 0; k < n; k++)
        if (!out[k] || !in[k]) return wc_fail(WC_EINVAL, "null field");
    if (int rc = check_prec(prec)) return rc;
    if (out_parity != 0 && out_parity != 1) return wc_fail(WC_EINVAL, "out_parity must be 0 or 1");
    if (int rc = check_ready(lat)) return rc;
    if (int rc = check_links_for(lat, prec)) return rc;
    MultCall calls[kMaxSys];
    for (int k = 0; k < n; k++) {
        calls[k] = mult_call(prec, M_HOPINV, out_parity, out[k], in[k], nullptr, 0.0);
        calls[k].lat = lat;
        calls[k].bs = lattice_bs(lat, prec);
    }
    return launch_mult_batch(lat->stream, calls, n);
}

extern "C" int wc_apply_Dee_oo_batch(wc_lattice *lat, int n, void *const *out_e, const void *const *in_e, int prec) {
    if (!lat || !out_e || !in_e) return wc_fail(WC_EINVAL, "null argument");
    if (n < 1 || n > kMaxSys) return wc_fail(WC_EINVAL, "n must lie in [1, 16]");
    for (int k = 0; k < n; k++) {
        if (!out_e[k] || !in_e[k]) return wc_fail(WC_EINVAL, "null field");
        if (out_e[k] == in_e[k]) return wc_fail(WC_EINVAL, "wc_apply_Dee_oo_batch cannot work in place");
    }
    if (int rc = check_prec(prec)) return rc;
    if (int rc = check_ready(lat)) return rc;
    if (int rc = check_links_for(lat, prec)) return rc;
    const size_t sb = spinor_bytes(prec, lat->Vh);
    char *tmp;
    if (int rc = lwork(lat, LW_APPLY_TMP, (size_t)n * sb, (void **)&tmp)) return rc;
    MultCall c1[kMaxSys], c2[kMaxSys];
    for (int k = 0; k < n; k++) {
        c1[k] = mult_call(prec, M_HOPINV, 1, tmp + k * sb, in_e[k], nullptr, 0.0);
        c2[k] = mult_call(prec, M_DHAT, 0, out_e[k], tmp + k * sb, in_e[k], -lat->kappa * lat->kappa);
        c1[k].lat = c2[k].lat = lat;
        c1[k].bs = c2[k].bs = lattice_bs(lat, prec);
    }
    if (int rc = launch_mult_batch(lat->stream, c1, n)) return rc;
    return launch_mult_batch(lat->stream, c2, n);
}

extern "C" int wc_apply_Dee_oo(wc_lattice *lat, void *out_e, const void *in_e, int prec) {
    if (!lat || !out_e || !in_e) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    if (out_e == in_e) return wc_fail(WC_EINVAL, "wc_apply_Dee_oo cannot work in place");
    if (int rc = check_ready(lat)) return rc;
    if (int rc = check_links_for(lat, prec)) return rc;
    void *tmp;
    if (int rc = lwork(lat, LW_APPLY_TMP, spinor_bytes(prec, lat->Vh), &tmp)) return rc;
    MultCall c1 = mult_call(prec, M_HOPINV, 1, tmp, in_e, nullptr, 0.0);
    if (int rc = launch_mult(lat, c1)) return rc;
    MultCall c2 = mult_call(prec, M_DHAT, 0, out_e, tmp, in_e, -lat->kappa * lat->kappa);
    return launch_mult(lat, c2);
}

extern "C" int wc_apply_clover(wc_lattice *lat, void *out, const void *in, int parity, int inverse, int prec) {
    if (!lat || !out || !in) return wc_fail(WC_EINVAL, "null argument");
    if (int rc = check_prec(prec)) return rc;
    if (parity != 0 && parity != 1) return wc_fail(WC_EINVAL, "parity must be 0 or 1");
    if (int rc = check_ready(lat)) return rc;
    MultCall c = mult_call(prec, M_CLOV, parity, out, nullptr, in, 0.0);
    c.inverse = inverse != 0;
    return launch_mult(lat, c);
}

extern "C" int wc_link_grad(wc_lattice *lat, const void *lam_dev, const void *x_dev, double kappa, double csw,
                            int include_clover, void *gradU_dev) {
    if (!lat || !lam_dev || !x_dev || !gradU_dev) return wc_fail(WC_EINVAL, "null argument");
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "wc_link_grad before wc_load_links");
    if (!(kappa >= 0.0) || !(csw >= 0.0)) return wc_fail(WC_EINVAL, "need kappa >= 0 and csw >= 0");
    const size_t sb = spinor_bytes(P64, lat->Vh);
    void *lam, *x, *N = nullptr;
    if (int rc = lwork(lat, LW_GLAM, 2 * sb, &lam)) return rc;
    if (int rc = lwork(lat, LW_GX, 2 * sb, &x)) return rc;
    const bool clover = include_clover && csw != 0.0;
    if (clover)
        if (int rc = lwork(lat, LW_GN, (size_t)6 * 2 * 9 * 16 * lat->Vh, &N)) return rc;
    if (int rc = launch_pack_spinor(lat, P64, lam, lam_dev)) return rc;
    if (int rc = launch_pack_spinor(lat, P64, x, x_dev)) return rc;
    return launch_link_grad(lat, lam, x, gradU_dev, N, kappa, csw, clover);
}
