// Solver drivers: the nested BiCGStab of Algorithms 1 (FP64 outer, flexible)
// and 2 (low-precision inner, source normalised to unit length), the
// all-FP64 BiCGStab on the same even-odd system, and the even-odd set-up and
// reconstruction of Sec. II-B (eqs. 6 and 7), for one or several systems.
//
// Several systems (several sources on one lattice, or lattices of different
// sizes) run in lockstep: every phase is one batched launch over the systems
// that are still iterating, each system keeps its own scalars and done flag,
// and one copy of the scalar arena per check serves all of them.
//
// Readings of the printed algorithms (both listings agree on them):
//   alpha = rho0 / <r~|q>             (the listings omit "rho0 /")
//   beta  = (rho1 / rho0) (alpha / omega)   (the listings divide by alpha/omega)
//   D-hat_ee = 1 - kappa^2 H-tilde_eo H-tilde_oe   (eq. 8 prints H-tilde_eo twice)
// Convergence of the outer loop is judged on its recursive residual, then
// confirmed on the true residual ||b - D x|| / ||b|| of the full system in
// FP64; when that check fails the outer loop restarts from the true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "internal.hpp"

namespace {

// slot pairs of the outer level used for set-up norms (S_AUX..S_AUX+3)
constexpr int S_NB_E = S_AUX;      // ||b_e||^2, then ||b-hat||^2, then ||res_e||^2
constexpr int S_NB_O = S_AUX + 2;  // ||b_o||^2, then ||res_o||^2

struct Run {
    std::vector<SolveSys> *sys;
    hipStream_t stream;
    wc_lattice *tl;     // receives timing records
    Arena *arena;
    bool use_graph;
    bool pipe;          // pipelined inner loop (two reduction phases per iteration)
    bool persistent;    // one cooperative launch per inner solve when the lattice allows
    int bs;             // threads per block of every stencil and vector launch of the solve
    int iprec;
    double itol;
    int imaxit, omaxit, fixed_work, check_every;
    // per system
    std::vector<double> src, tol_eo, tol2_in, bnorm;
    std::vector<int> conv, dead;
    std::vector<long> dslash;
};

SolveSys &S_(Run &R, int k) { return (*R.sys)[k]; }
void *W(Run &R, int k, int id) { return S_(R, k).work->buf[id]; }
size_t sb64(Run &R, int k) { return spinor_bytes(P64, S_(R, k).lat->Vh); }
char *par_half(Run &R, int k, int id, int par) { return (char *)W(R, k, id) + par * sb64(R, k); }

int sync(Run &R) { return sync_arena(*R.arena, R.stream); }

MultCall mc(Run &R, int k, int prec, int mode, int out_par, void *out, const void *in, const void *center,
            double coef) {
    MultCall c;
    std::memset(&c, 0, sizeof(c));
    c.lat = S_(R, k).lat;
    c.prec = prec;
    c.mode = mode;
    c.red = R_NONE;
    c.out_par = out_par;
    c.out = out;
    c.in = in;
    c.center = center;
    c.coef = coef;
    c.bs = R.bs;
    return c;
}

VecCall vc(Run &R, int k, int lvl, void *a, void *b = nullptr, void *c = nullptr, void *d = nullptr,
           void *e = nullptr) {
    VecCall v;
    std::memset(&v, 0, sizeof(v));
    SolveSys &s = S_(R, k);
    v.Vh = s.lat->Vh;
    v.a = a;
    v.b = b;
    v.c = c;
    v.d = d;
    v.e = e;
    v.sc = s.st->sc(lvl);
    v.fl = s.st->fl(lvl);
    v.partials = s.st->partials;
    v.tol2 = R.tol2_in[k];
    v.bs = R.bs;
    return v;
}

// one batched stencil launch over the systems in `act`
template <class F> int mult_over(Run &R, const std::vector<int> &act, F &&make) {
    MultCall calls[kMaxSys];
    int n = 0;
    for (int k : act) {
        calls[n++] = make(k);
        R.dslash[k]++;
    }
    return launch_mult_batch(R.stream, calls, n, R.tl);
}

template <class F> int vec_over(Run &R, const std::vector<int> &act, int op, int prec, F &&make) {
    VecCall calls[kMaxSys];
    int n = 0;
    for (int k : act) calls[n++] = make(k);
    return launch_vec_batch(R.stream, R.tl, op, prec, calls, n);
}

// out = D-hat_ee in (two MULTs, eq. 8) for each system, with an optional fused
// <aux, out> (and ||out||^2) into slot `slot` of level `lvl`
int dhat(Run &R, const std::vector<int> &act, int prec, int out_id, int in_id, int tmp_id, int red, int aux_id,
         int lvl, int slot, bool guarded) {
    if (int rc = mult_over(R, act, [&](int k) {
            MultCall c = mc(R, k, prec, M_HOPINV, 1, W(R, k, tmp_id), W(R, k, in_id), nullptr, 0.0);
            c.done = guarded ? S_(R, k).st->fl(lvl) : nullptr;
            return c;
        }))
        return rc;
    return mult_over(R, act, [&](int k) {
        SolveSys &s = S_(R, k);
        MultCall c = mc(R, k, prec, M_DHAT, 0, W(R, k, out_id), W(R, k, tmp_id), W(R, k, in_id),
                        -s.lat->kappa * s.lat->kappa);
        c.red = red;
        c.aux = aux_id >= 0 ? W(R, k, aux_id) : nullptr;
        c.red_to = RedTarget{s.st->partials, s.st->sc(lvl) + slot};
        c.done = guarded ? s.st->fl(lvl) : nullptr;
        return c;
    });
}

VecCall vc9(Run &R, int k, int lvl, void *a, void *b, void *c, void *d, void *e, void *f, void *g, void *h,
            void *j = nullptr) {
    VecCall v = vc(R, k, lvl, a, b, c, d, e);
    v.f = f;
    v.g = g;
    v.h = h;
    v.j = j;
    return v;
}

// One chunk of n iterations of the pipelined BiCGStab (Cools and Vanroose,
// Parallel Computing 65, 2017) on D-hat_ee: the same Krylov iterates as
// Algorithm 2, with the recurrences rearranged so that each iteration has two
// reduction phases instead of four.  It keeps s = A p, z = A s, w = A r,
// t = A w and v = A z as vectors and updates them by recurrence, at the cost
// of more vector traffic.  Per iteration:
//   phase 0: p, s, z updates with the sums <y, q>, ||y||^2, ||q||^2, <r~, s>,
//            <r~, z> (q = r - alpha s, y = w - alpha z) -> omega, half-step check
//   phase 1: v = A z; x, r, w updates with <r~, r>, <r~, w>, ||r||^2 -> beta,
//            the next alpha, full-step check
//   phase 2: t = A w
int inner_chunk_pipe(Run &R, const std::vector<int> &act, int n, int base = 0) {
    const int L = 0, P = R.iprec;
    auto loop = [&](VecCall v) {
        v.iter_dev = 1;
        v.guard = 1;
        return v;
    };
    auto tag = [&](int it, int ph) {
        R.tl->tag_iter = it;
        R.tl->tag_phase = ph;
    };
    for (int j = 0; j < n; j++) {
        tag(base + j, 0);
        if (int rc = vec_over(R, act, V_PIPE_A, P, [&](int k) {
                return loop(vc9(R, k, L, W(R, k, W_IR), W(R, k, W_IW), W(R, k, W_IT), W(R, k, W_IP), W(R, k, W_IS),
                                W(R, k, W_IZ), W(R, k, W_IV), W(R, k, W_IRT)));
            }))
            return rc;
        tag(base + j, 1);
        if (int rc = dhat(R, act, P, W_IV, W_IZ, W_ITMP, R_NONE, -1, L, 0, true)) return rc;
        if (int rc = vec_over(R, act, V_PIPE_B, P, [&](int k) {
                return loop(vc9(R, k, L, W(R, k, W_IX), W(R, k, W_IP), W(R, k, W_IR), W(R, k, W_IS), W(R, k, W_IW),
                                W(R, k, W_IZ), W(R, k, W_IT), W(R, k, W_IV), W(R, k, W_IRT)));
            }))
            return rc;
        tag(base + j, 2);
        if (int rc = dhat(R, act, P, W_IT, W_IW, W_ITMP, R_NONE, -1, L, 0, true)) return rc;
    }
    tag(-1, 0);
    return WC_OK;
}

// one chunk of n iterations of Algorithm 2 for the systems in act; every
// kernel takes the iteration index from the system's device flags, so the
// same launches serve any chunk (and can be recorded once as a graph)
int inner_chunk(Run &R, const std::vector<int> &act, int n, int base = 0) {
    const int L = 0, P = R.iprec;
    auto loop = [&](VecCall v) {
        v.iter_dev = 1;
        v.guard = 1;
        return v;
    };
    // tags for the timing records: iteration and phase (0: first D-hat and the
    // s update, 1: second D-hat and the x, r update, 2: the p update)
    auto tag = [&](int it, int ph) {
        R.tl->tag_iter = it;
        R.tl->tag_phase = ph;
    };
    for (int j = 0; j < n; j++) {
        tag(base + j, 0);
        if (int rc = dhat(R, act, P, W_IQ, W_IP, W_ITMP, R_DOT, W_IRT, L, S_RQ, true)) return rc;
        if (int rc = vec_over(R, act, V_INNER_A, P,
                              [&](int k) { return loop(vc(R, k, L, W(R, k, W_IR), W(R, k, W_IQ))); }))
            return rc;
        tag(base + j, 1);
        if (int rc = dhat(R, act, P, W_IT, W_IR, W_ITMP, R_DOTNORM, W_IR, L, S_ST, true)) return rc;
        if (int rc = vec_over(R, act, V_INNER_B, P, [&](int k) {
                return loop(vc(R, k, L, W(R, k, W_IX), W(R, k, W_IR), W(R, k, W_IP), W(R, k, W_IT), W(R, k, W_IRT)));
            }))
            return rc;
        tag(base + j, 2);
        if (int rc = vec_over(R, act, V_INNER_C, P,
                              [&](int k) { return loop(vc(R, k, L, W(R, k, W_IP), W(R, k, W_IR), W(R, k, W_IQ))); }))
            return rc;
    }
    tag(-1, 0);
    return WC_OK;
}

// run a chunk through a graph recorded once per (systems, precision, length,
// lattice generations); recording happens on the lattice's private stream,
// replay on the solve's stream
int inner_chunk_graph(Run &R, const std::vector<int> &act, int n) {
    unsigned long long key = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) { key = (key ^ v) * 1099511628211ull; };
    mix((unsigned long long)R.iprec);
    mix((unsigned long long)n);
    mix((unsigned long long)R.pipe);
    mix((unsigned long long)R.bs);
    for (int k : act) {
        mix((unsigned long long)k);
        mix(S_(R, k).lat->serial);
        mix((unsigned long long)S_(R, k).lat->gen);
    }
    hipGraphExec_t exec = nullptr;
    for (auto &g : R.arena->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        wc_lattice *lead = R.tl;
        if (!lead->capture_stream) WC_HIP(hipStreamCreateWithFlags(&lead->capture_stream, hipStreamNonBlocking));
        const hipStream_t user = R.stream;
        const std::vector<long> saved = R.dslash;
        R.stream = lead->capture_stream;
        WC_HIP(hipStreamBeginCapture(R.stream, hipStreamCaptureModeThreadLocal));
        const int rc = R.pipe ? inner_chunk_pipe(R, act, n) : inner_chunk(R, act, n);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(R.stream, &graph);
        R.stream = user;
        R.dslash = saved;
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return wc_fail(WC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return wc_fail(WC_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        if (R.arena->graphs.size() >= 64) arena_drop_graphs(*R.arena);
        R.arena->graphs.push_back(GraphEntry{key, exec});
    }
    WC_HIP(hipGraphLaunch(exec, R.stream));
    for (int k : act) R.dslash[k] += 4 * n;
    return WC_OK;
}

// v = M src for every system in act: Algorithm 2 on the inner level (0)
int inner_solve(Run &R, const std::vector<int> &act, int src_id, int v_id) {
    const int L = 0, P = R.iprec;
    if (R.fixed_work > 0)
        for (int k : act) R.tol2_in[k] = 0.0;
    if (int rc = vec_over(R, act, V_NORM2, P64, [&](int k) {
            VecCall v = vc(R, k, L, W(R, k, src_id));
            v.result = S_(R, k).st->sc(L) + S_NORM;
            return v;
        }))
        return rc;
    if (R.pipe) {
        // r = r~ = b, x = 0; w = A r with <r~, w>; t = A w; alpha_0 = <r~, r> / <r~, w>
        if (int rc = vec_over(R, act, V_PIPE_INIT, P, [&](int k) {
                return vc9(R, k, L, W(R, k, src_id), W(R, k, W_IR), W(R, k, W_IRT), W(R, k, W_IX), W(R, k, W_IP),
                           W(R, k, W_IS), W(R, k, W_IZ), W(R, k, W_IV));
            }))
            return rc;
        if (int rc = dhat(R, act, P, W_IW, W_IR, W_ITMP, R_DOT, W_IRT, L, S_RQ, true)) return rc;
        if (int rc = dhat(R, act, P, W_IT, W_IW, W_ITMP, R_NONE, -1, L, 0, true)) return rc;
        FinArgs f[kMaxSys];
        int nf = 0;
        for (int k : act) {
            FinArgs a = FinArgs{};
            a.op = FIN_PIPE_INIT;
            a.sc = S_(R, k).st->sc(L);
            a.fl = S_(R, k).st->fl(L);
            a.guard = a.fl;
            f[nf++] = a;
        }
        if (int rc = launch_fin_batch(R.stream, f, nf, 1)) return rc;
    } else if (int rc = vec_over(R, act, V_INNER_INIT, P, [&](int k) {
                   return vc(R, k, L, W(R, k, src_id), W(R, k, W_IR), W(R, k, W_IRT), W(R, k, W_IP), W(R, k, W_IX));
               })) {
        return rc;
    }
    const int maxit = R.fixed_work > 0 ? R.fixed_work : R.imaxit;
    const bool graph = R.use_graph && !R.tl->timing;
    const size_t timed_from = R.tl->launches.size();
    const std::vector<long> dslash_before = R.dslash;
    int queued = 0;
    // one system of a small lattice: the whole loop as one cooperative launch
    // (not under kernel timing, whose per-launch records it would bypass)
    if (R.persistent && !R.pipe && act.size() == 1 && !R.tl->timing && S_(R, act[0]).st->partials2 &&
        S_(R, act[0]).st->bar) {
        const int k = act[0];
        SolveSys &s = S_(R, k);
        PersistCall c;
        c.lat = s.lat;
        c.prec = P;
        c.r = W(R, k, W_IR);
        c.rt = W(R, k, W_IRT);
        c.p = W(R, k, W_IP);
        c.q = W(R, k, W_IQ);
        c.t = W(R, k, W_IT);
        c.tmp = W(R, k, W_ITMP);
        c.x = W(R, k, W_IX);
        c.part0 = s.st->partials;
        c.part1 = s.st->partials2;
        c.sc = s.st->sc(L);
        c.fl = s.st->fl(L);
        c.maxit = maxit;
        c.bar = s.st->bar;
        if (++s.st->bar_epoch == 0) {
            // the call counter wrapped: clear the words so the new tags exceed them
            const size_t words = (size_t)s.lat->nblocks + 2;  // as allocated with the lattice
            if (hipMemsetAsync(s.st->bar, 0, words * sizeof(unsigned long long), R.stream) != hipSuccess)
                return wc_fail(WC_EHIP, "clearing the grid barrier words");
            s.st->bar_epoch = 1;
        }
        c.epoch = s.st->bar_epoch;
        bool ran = false;
        if (int rc = launch_inner_persistent(c, R.stream, &ran)) return rc;
        if (ran) {
            if (int rc = sync(R)) return rc;
            if (s.st->hf(L, F_STOPPH) == 3)
                return wc_fail(WC_EHIP, "one-launch inner loop: a grid barrier wait ran out of time");
            queued = maxit;  // the loop below is done
            s.info.persistent_calls++;
        }
    }
    while (queued < maxit) {
        const int n = std::min(R.check_every, maxit - queued);
        if (int rc = graph    ? inner_chunk_graph(R, act, n)
                     : R.pipe ? inner_chunk_pipe(R, act, n, queued)
                              : inner_chunk(R, act, n, queued))
            return rc;
        queued += n;
        if (int rc = sync(R)) return rc;
        bool all = true;
        for (int k : act) all = all && S_(R, k).st->hf(L, F_DONE) != DONE_NO;
        if (all) break;
    }
    if (R.tl->timing) {
        // launches queued after a system stopped did no work for it
        std::vector<StopPoint> stops;
        for (int k : act) {
            const SysState &st = *S_(R, k).st;
            const int ph = st.hf(L, F_STOPPH);
            if (st.hf(L, F_DONE) == DONE_NO || ph == 0) continue;
            const int it = st.hf(L, F_ITERS);
            stops.push_back(StopPoint{st.fl(L), ph == 1 ? it : it - 1, ph});
        }
        timing_settle(R.tl, timed_from, stops);
    }
    std::vector<int> fix;
    for (int k : act) {
        SolveSys &s = S_(R, k);
        const int code = s.st->hf(L, F_DONE);
        int iters = s.st->hf(L, F_ITERS);
        if (code == DONE_HALF) {
            fix.push_back(k);
            iters += 1;
        }
        s.info.inner_iters_total += iters;
        s.info.inner_calls += 1;
        // MULTs done: four per full iteration, two for a half-step exit (the
        // launches queued after the stop returned at once)
        const int stopph = s.st->hf(L, F_STOPPH);
        const long full = s.st->hf(L, F_ITERS);
        // the pipelined loop also applies D-hat twice to set up, and its
        // half-step check comes before that iteration's D-hat
        R.dslash[k] = dslash_before[k] + 4 * full +
                      (R.pipe ? 4 : ((code != DONE_NO && stopph == 1) ? 2 : 0));
    }
    if (!fix.empty())
        if (int rc = vec_over(R, fix, R.pipe ? V_PIPE_FIX : V_INNER_FIX, P, [&](int k) {
                VecCall v = vc(R, k, L, W(R, k, W_IX), W(R, k, W_IP));
                v.iter = S_(R, k).st->hf(L, F_ITERS);
                return v;
            }))
            return rc;
    return vec_over(R, act, V_INNER_FINAL, P, [&](int k) { return vc(R, k, L, W(R, k, v_id), W(R, k, W_IX)); });
}

// r = b-hat - D-hat x_e, ||r||^2 to the outer level's S_RR
int eo_residual(Run &R, const std::vector<int> &act) {
    if (int rc = dhat(R, act, P64, W_Q, W_X, W_TMP64, R_NONE, -1, 1, 0, false)) return rc;
    return vec_over(R, act, V_SUB_NORM, P64, [&](int k) {
        VecCall v = vc(R, k, 1, W(R, k, W_R), W(R, k, W_BHAT), W(R, k, W_Q));
        v.result = S_(R, k).st->sc(1) + S_RR;
        return v;
    });
}

// x_o from eq. 7 and the squared true residual of the full system per system
int reconstruct_and_check(Run &R, const std::vector<int> &act, std::vector<double> &res2) {
    // x_o = F_oo^-1 (b_o + kappa H_oe x_e)
    if (int rc = mult_over(R, act, [&](int k) {
            return mc(R, k, P64, M_INVSRC, 1, par_half(R, k, W_X, 1), par_half(R, k, W_X, 0), par_half(R, k, W_B, 1),
                      S_(R, k).lat->kappa);
        }))
        return rc;
    // (D x)_e = F_ee x_e - kappa H_eo x_o, (D x)_o likewise
    if (int rc = mult_over(R, act, [&](int k) {
            return mc(R, k, P64, M_DFULL, 0, W(R, k, W_Q), par_half(R, k, W_X, 1), par_half(R, k, W_X, 0),
                      -S_(R, k).lat->kappa);
        }))
        return rc;
    if (int rc = vec_over(R, act, V_SUB_NORM, P64, [&](int k) {
            VecCall v = vc(R, k, 1, W(R, k, W_RES), par_half(R, k, W_B, 0), W(R, k, W_Q));
            v.result = S_(R, k).st->sc(1) + S_NB_E;
            return v;
        }))
        return rc;
    if (int rc = mult_over(R, act, [&](int k) {
            return mc(R, k, P64, M_DFULL, 1, W(R, k, W_TMP64), par_half(R, k, W_X, 0), par_half(R, k, W_X, 1),
                      -S_(R, k).lat->kappa);
        }))
        return rc;
    if (int rc = vec_over(R, act, V_SUB_NORM, P64, [&](int k) {
            VecCall v = vc(R, k, 1, W(R, k, W_RES), par_half(R, k, W_B, 1), W(R, k, W_TMP64));
            v.result = S_(R, k).st->sc(1) + S_NB_O;
            return v;
        }))
        return rc;
    if (int rc = sync(R)) return rc;
    for (int k : act) res2[k] = S_(R, k).st->hs(1, S_NB_E) + S_(R, k).st->hs(1, S_NB_O);
    return WC_OK;
}

// drop converged / failed systems from act
void prune(Run &R, std::vector<int> &act) {
    std::vector<int> keep;
    for (int k : act)
        if (!R.conv[k] && !R.dead[k]) keep.push_back(k);
    act.swap(keep);
}

// check the outer recursive residuals after an update; false on breakdown
void outer_check(Run &R, std::vector<int> &act) {
    for (int k : act) {
        SolveSys &s = S_(R, k);
        const double rr = s.st->hs(1, S_RR);
        s.info.eo_rel_residual = std::sqrt(rr) / R.src[k];
        if (!std::isfinite(rr)) R.dead[k] = WC_EBREAKDOWN;
        else if (std::sqrt(rr) / R.src[k] < R.tol_eo[k]) R.conv[k] = 1;
    }
    prune(R, act);
}

// Algorithm 1 from the current x_e of every system in act
int outer_flexible(Run &R, std::vector<int> act, bool x_is_zero) {
    const int L = 1;
    if (x_is_zero) {
        if (int rc = vec_over(R, act, V_COPY, P64, [&](int k) { return vc(R, k, L, W(R, k, W_R), W(R, k, W_BHAT)); }))
            return rc;
    } else {
        if (int rc = eo_residual(R, act)) return rc;
    }
    if (int rc = vec_over(R, act, V_NORM2, P64, [&](int k) {
            VecCall v = vc(R, k, L, W(R, k, W_R));
            v.result = S_(R, k).st->sc(L) + S_RHO0;
            return v;
        }))
        return rc;
    if (int rc = vec_over(R, act, V_COPY, P64, [&](int k) { return vc(R, k, L, W(R, k, W_RT), W(R, k, W_R)); }))
        return rc;
    if (int rc = vec_over(R, act, V_COPY, P64, [&](int k) { return vc(R, k, L, W(R, k, W_P), W(R, k, W_R)); }))
        return rc;
    if (int rc = sync(R)) return rc;
    for (int k : act) {
        const double rr = S_(R, k).st->hs(L, S_RHO0);
        S_(R, k).info.eo_rel_residual = std::sqrt(rr) / R.src[k];
        if (std::sqrt(rr) / R.src[k] < R.tol_eo[k]) R.conv[k] = 1;
    }
    prune(R, act);
    for (int it = 0; it < R.omaxit && !act.empty(); it++) {
        for (int k : act) S_(R, k).info.outer_iters++;
        // v = M p;  q = D-hat v with <r~, q>
        if (int rc = inner_solve(R, act, W_P, W_V)) return rc;
        if (int rc = dhat(R, act, P64, W_Q, W_V, W_TMP64, R_DOT, W_RT, L, S_RQ, false)) return rc;
        if (int rc = vec_over(R, act, V_OUTER_A, P64, [&](int k) {
                VecCall v = vc(R, k, L, W(R, k, W_X), W(R, k, W_R), W(R, k, W_V), W(R, k, W_Q));
                v.iter = it;
                return v;
            }))
            return rc;
        if (int rc = sync(R)) return rc;
        outer_check(R, act);
        if (act.empty()) break;
        // v = M r;  t = D-hat v with <r, t>, ||t||^2
        if (int rc = inner_solve(R, act, W_R, W_V)) return rc;
        if (int rc = dhat(R, act, P64, W_T, W_V, W_TMP64, R_DOTNORM, W_R, L, S_ST, false)) return rc;
        if (int rc = vec_over(R, act, V_OUTER_B, P64, [&](int k) {
                VecCall v = vc(R, k, L, W(R, k, W_X), W(R, k, W_R), W(R, k, W_V), W(R, k, W_T), W(R, k, W_RT));
                v.iter = it;
                return v;
            }))
            return rc;
        if (int rc = sync(R)) return rc;
        outer_check(R, act);
        for (int k : act) {
            const int slot = ((it + 1) & 1) ? S_RHO1 : S_RHO0;
            if (S_(R, k).st->hs(L, slot) == 0.0 && S_(R, k).st->hs(L, slot + 1) == 0.0) R.dead[k] = WC_EBREAKDOWN;
        }
        prune(R, act);
        if (act.empty()) break;
        if (int rc = vec_over(R, act, V_INNER_C, P64, [&](int k) {
                VecCall v = vc(R, k, L, W(R, k, W_P), W(R, k, W_R), W(R, k, W_Q));
                v.iter = it;
                return v;
            }))
            return rc;
    }
    return WC_OK;
}

// Defect correction from the current x_e of every system in act: each step
// solves D-hat v = r_e with the low-precision inner solver (Algorithm 2),
// adds v to x_e and recomputes r_e = b-hat - D-hat x_e in FP64.  Each inner
// solve aims at the inner tolerance, or at half the reduction still needed
// when that is looser, so the last step does not over-solve.  A step that
// does not lower ||r_e|| ends the system's iteration (reported as no
// convergence unless the tolerance is met).
int outer_dc(Run &R, std::vector<int> act, bool x_is_zero) {
    if (x_is_zero) {
        if (int rc = vec_over(R, act, V_COPY, P64, [&](int k) { return vc(R, k, 1, W(R, k, W_R), W(R, k, W_BHAT)); }))
            return rc;
        if (int rc = vec_over(R, act, V_NORM2, P64, [&](int k) {
                VecCall v = vc(R, k, 1, W(R, k, W_R));
                v.result = S_(R, k).st->sc(1) + S_RR;
                return v;
            }))
            return rc;
    } else {
        if (int rc = eo_residual(R, act)) return rc;
    }
    if (int rc = sync(R)) return rc;
    std::vector<double> last(R.src.size(), 0.0);
    for (int it = 0; !act.empty(); it++) {
        std::vector<int> run;
        for (int k : act) {
            const double rn = std::sqrt(S_(R, k).st->hs(1, S_RR));
            S_(R, k).info.eo_rel_residual = rn / R.src[k];
            if (!std::isfinite(rn)) {
                R.dead[k] = WC_EBREAKDOWN;
            } else if (rn / R.src[k] < R.tol_eo[k]) {
                R.conv[k] = 1;
            } else if (it < R.omaxit && (it == 0 || rn < last[k])) {
                const double t = std::max(R.itol, 0.5 * R.tol_eo[k] * R.src[k] / rn);
                R.tol2_in[k] = t * t;
                last[k] = rn;
                S_(R, k).info.outer_iters++;
                run.push_back(k);
            }
        }
        act.swap(run);
        if (act.empty()) break;
        if (int rc = inner_solve(R, act, W_R, W_V)) return rc;
        if (int rc = vec_over(R, act, V_AXPY, P64, [&](int k) {
                VecCall v = vc(R, k, 1, W(R, k, W_X), W(R, k, W_V));
                v.coef = 1.0;
                return v;
            }))
            return rc;
        if (int rc = eo_residual(R, act)) return rc;
        if (int rc = sync(R)) return rc;
    }
    for (auto &t : R.tol2_in) t = R.itol * R.itol;
    return WC_OK;
}

// plain FP64 BiCGStab on D-hat_ee (the inner machinery in FP64) for D-hat v = r_e,
// x_e += v, for every system in act
int fp64_pass(Run &R, std::vector<int> act, bool x_is_zero) {
    if (x_is_zero) {
        if (int rc = vec_over(R, act, V_COPY, P64, [&](int k) { return vc(R, k, 1, W(R, k, W_R), W(R, k, W_BHAT)); }))
            return rc;
        if (int rc = vec_over(R, act, V_NORM2, P64, [&](int k) {
                VecCall v = vc(R, k, 1, W(R, k, W_R));
                v.result = S_(R, k).st->sc(1) + S_RR;
                return v;
            }))
            return rc;
    } else {
        if (int rc = eo_residual(R, act)) return rc;
    }
    if (int rc = sync(R)) return rc;
    std::vector<int> run;
    for (int k : act) {
        const double rn = std::sqrt(S_(R, k).st->hs(1, S_RR));
        S_(R, k).info.eo_rel_residual = rn / R.src[k];
        if (rn / R.src[k] < R.tol_eo[k]) {
            R.conv[k] = 1;
        } else {
            const double t = R.tol_eo[k] * R.src[k] / rn;
            R.tol2_in[k] = t * t;
            S_(R, k).info.outer_iters++;
            run.push_back(k);
        }
    }
    if (run.empty()) return WC_OK;
    if (int rc = inner_solve(R, run, W_R, W_V)) return rc;
    if (int rc = vec_over(R, run, V_AXPY, P64, [&](int k) {
            VecCall v = vc(R, k, 1, W(R, k, W_X), W(R, k, W_V));
            v.coef = 1.0;
            return v;
        }))
        return rc;
    if (int rc = eo_residual(R, run)) return rc;
    if (int rc = sync(R)) return rc;
    for (int k : run) {
        const double rr = std::sqrt(S_(R, k).st->hs(1, S_RR));
        S_(R, k).info.eo_rel_residual = rr / R.src[k];
        R.conv[k] = rr / R.src[k] < R.tol_eo[k];
    }
    return WC_OK;
}

}  // namespace

int solve_systems(std::vector<SolveSys> &sys, Arena &arena, double tol, const wc_solve_params &P,
                  int x0_is_guess) {
    const int S = (int)sys.size();
    if (S < 1 || S > kMaxSys) return wc_fail(WC_EINVAL, "between 1 and 16 systems per solve");
    auto t0 = std::chrono::steady_clock::now();
    Run R;
    R.sys = &sys;
    R.stream = sys[0].lat->stream;
    R.tl = sys[0].lat;
    R.arena = &arena;
    R.use_graph = P.use_graph != 0;
    R.pipe = P.inner_method == WC_INNER_PIPELINED;
    R.persistent = P.persistent != 0;
    // block size: each lattice's pinned or tuned value for the inner
    // precision (tuned now if neither); a batch over several lattices runs
    // with the largest lattice's, which dominates its cost
    {
        wc_lattice *big = sys[0].lat;
        for (auto &s : sys) {
            if ((!s.lat->bs_pin && !s.lat->bs_tuned[P.inner_prec]) ||
                (s.lat->chunk_pin < 0 && s.lat->chunk_tuned[P.inner_prec] < 0)) {
                const int rc = tune_block_size(s.lat, P.inner_prec, nullptr, nullptr);
                if (rc == WC_ENOMEM) {  // no room to time: the defaults
                    s.lat->bs_tuned[P.inner_prec] = 256;
                    s.lat->chunk_tuned[P.inner_prec] = kDefaultChunk;
                }
                else if (rc) return rc;
            }
            if (s.lat->Vh > big->Vh) big = s.lat;
        }
        R.bs = lattice_bs(big, P.inner_prec);
    }
    R.iprec = P.inner_prec;
    R.itol = P.inner_tol > 0.0 ? P.inner_tol : (P.inner_prec == WC_FP16 ? 1e-3 : 1e-6);
    R.imaxit = P.inner_maxit;
    R.omaxit = P.outer_maxit;
    R.fixed_work = P.fixed_work;
    R.check_every = P.check_every;
    R.src.assign(S, 0.0);
    R.tol_eo.assign(S, 0.0);
    R.tol2_in.assign(S, R.itol * R.itol);
    R.bnorm.assign(S, 0.0);
    R.conv.assign(S, 0);
    R.dead.assign(S, 0);
    R.dslash.assign(S, 0);
    for (auto &s : sys) {
        std::memset(&s.info, 0, sizeof(s.info));
        s.status = WC_ENOCONV;
    }
    std::vector<int> all(S);
    for (int k = 0; k < S; k++) all[k] = k;

    // b -> EO FP64 and ||b||.  The adjoint system D^dag x = b is solved as
    // D y = g5 b, x = g5 y (g5 D g5 = D^dag).
    for (int k = 0; k < S; k++)
        if (int rc = launch_pack_spinor(sys[k].lat, P64, W(R, k, W_B), sys[k].b_dev)) return rc;
    if (P.adjoint)
        if (int rc = vec_over(R, all, V_GAMMA5, P64, [&](int k) { return vc(R, k, 1, W(R, k, W_B)); })) return rc;
    for (int par = 0; par < 2; par++)
        if (int rc = vec_over(R, all, V_NORM2, P64, [&](int k) {
                VecCall v = vc(R, k, 1, par_half(R, k, W_B, par));
                v.result = sys[k].st->sc(1) + (par ? S_NB_O : S_NB_E);
                return v;
            }))
            return rc;
    if (int rc = sync(R)) return rc;
    std::vector<int> act;
    for (int k = 0; k < S; k++) {
        const double b2 = sys[k].st->hs(1, S_NB_E) + sys[k].st->hs(1, S_NB_O);
        R.bnorm[k] = std::sqrt(b2);
        if (!std::isfinite(b2)) return wc_fail(WC_EINVAL, "b has non-finite entries");
        if (b2 == 0.0) {
            // x = 0 solves D x = 0 exactly
            if (int rc = vec_over(R, {k}, V_ZERO, P64, [&](int j) { return vc(R, j, 1, par_half(R, j, W_X, 0)); })) return rc;
            if (int rc = vec_over(R, {k}, V_ZERO, P64, [&](int j) { return vc(R, j, 1, par_half(R, j, W_X, 1)); })) return rc;
            sys[k].status = WC_OK;
            R.conv[k] = 1;
        } else {
            act.push_back(k);
        }
    }
    // b-hat_e = F_ee^-1 (b_e + kappa H_eo F_oo^-1 b_o)      (eq. 6)
    if (!act.empty()) {
        if (int rc = mult_over(R, act, [&](int k) {
                MultCall c = mc(R, k, P64, M_CLOV, 1, W(R, k, W_TMP64), nullptr, par_half(R, k, W_B, 1), 0.0);
                c.inverse = true;
                return c;
            }))
            return rc;
        if (int rc = mult_over(R, act, [&](int k) {
                return mc(R, k, P64, M_INVSRC, 0, W(R, k, W_BHAT), W(R, k, W_TMP64), par_half(R, k, W_B, 0),
                          sys[k].lat->kappa);
            }))
            return rc;
        if (int rc = vec_over(R, act, V_NORM2, P64, [&](int k) {
                VecCall v = vc(R, k, 1, W(R, k, W_BHAT));
                v.result = sys[k].st->sc(1) + S_NB_E;
                return v;
            }))
            return rc;
        for (int k : act) {
            if (x0_is_guess) {
                if (int rc = launch_pack_spinor(sys[k].lat, P64, W(R, k, W_X), sys[k].x_dev)) return rc;
            }
        }
        if (x0_is_guess && P.adjoint)
            if (int rc = vec_over(R, act, V_GAMMA5, P64, [&](int k) { return vc(R, k, 1, W(R, k, W_X)); })) return rc;
        if (!x0_is_guess) {
            for (int par = 0; par < 2; par++)
                if (int rc = vec_over(R, act, V_ZERO, P64, [&](int k) { return vc(R, k, 1, par_half(R, k, W_X, par)); }))
                    return rc;
        }
        if (int rc = sync(R)) return rc;
        for (int k : act) {
            R.src[k] = std::sqrt(sys[k].st->hs(1, S_NB_E));
            R.tol_eo[k] = 0.5 * tol * R.bnorm[k] / R.src[k];
        }
    }

    const int max_passes = 6;
    std::vector<double> res2(S, 0.0);
    for (int pass = 0; pass < max_passes && !act.empty(); pass++) {
        for (int k : act) R.conv[k] = 0;
        const bool xz = (!x0_is_guess) && pass == 0;
        int rc = (R.iprec == WC_FP64)       ? fp64_pass(R, act, xz)
                 : (P.outer == WC_OUTER_DC) ? outer_dc(R, act, xz)
                                            : outer_flexible(R, act, xz);
        if (rc) return rc;
        if (int rc2 = reconstruct_and_check(R, act, res2)) return rc2;
        std::vector<int> again;
        for (int k : act) {
            sys[k].info.true_rel_residual = std::sqrt(res2[k]) / R.bnorm[k];
            if (sys[k].info.true_rel_residual <= tol) {
                sys[k].status = WC_OK;
            } else if (R.dead[k] && pass + 1 < max_passes) {
                R.dead[k] = 0;  // breakdown: restart from the true residual
                sys[k].info.restarts++;
                again.push_back(k);
            } else if (R.conv[k] || R.iprec == WC_FP64) {
                sys[k].info.restarts++;
                again.push_back(k);
            } else {
                sys[k].status = R.dead[k] ? R.dead[k] : WC_ENOCONV;  // iteration cap
            }
        }
        act.swap(again);
    }
    for (int k : act)
        if (sys[k].status == WC_ENOCONV && R.dead[k]) sys[k].status = R.dead[k];

    if (P.adjoint)
        if (int rc = vec_over(R, all, V_GAMMA5, P64, [&](int k) { return vc(R, k, 1, W(R, k, W_X)); })) return rc;
    for (int k = 0; k < S; k++)
        if (int rc = launch_unpack_spinor(sys[k].lat, P64, sys[k].x_dev, W(R, k, W_X))) return rc;
    WC_HIP(hipStreamSynchronize(R.stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < S; k++) {
        sys[k].info.seconds = secs;
        sys[k].info.block_size = R.bs;
        sys[k].info.dslash_count = R.dslash[k];
        sys[k].info.status = sys[k].status;
    }
    return WC_OK;
}
