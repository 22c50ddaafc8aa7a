// Solver drivers: the nested BiCGStab of Algorithms 1 (FP64 outer, flexible)
// and 2 (low-precision inner, source normalised to unit length), the
// all-FP64 BiCGStab on the same even-odd system, and the even-odd set-up and
// reconstruction of Sec. II-B (eqs. 6 and 7).
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
#include <cstring>

#include "internal.hpp"
#include "work.hpp"

namespace {

struct Ctx {
    wc_lattice *lat;
    int iprec;   // inner storage precision
    int xprec;   // inner solution precision
    double itol;
    int imaxit, omaxit, fixed_work, check_every;
    size_t sb64, sbi, sbx;
    void *b, *x, *bhat, *r, *rt, *p, *v, *q, *t, *tmp64, *res;
    void *ir, *irt, *ip, *iq, *it, *itmp, *ix;
    wc_solve_info info;
    bool inner_broke = false;
};

int sync_scalars(wc_lattice *lat) {
    WC_HIP(hipMemcpyAsync(lat->host_scalars, lat->scalars, sizeof(double) * NUM_LEVELS * S_COUNT,
                          hipMemcpyDeviceToHost, lat->stream));
    WC_HIP(hipMemcpyAsync(lat->host_flags, lat->flags, sizeof(int) * NUM_LEVELS * F_COUNT, hipMemcpyDeviceToHost,
                          lat->stream));
    WC_HIP(hipStreamSynchronize(lat->stream));
    return WC_OK;
}

double hs(wc_lattice *lat, int lvl, int slot) { return lat->host_scalars[lvl * S_COUNT + slot]; }
int hf(wc_lattice *lat, int lvl, int slot) { return lat->host_flags[lvl * F_COUNT + slot]; }

MultCall mc(int prec, int mode, int out_par, void *out, const void *in, const void *center, double coef) {
    MultCall c;
    std::memset(&c, 0, sizeof(c));
    c.prec = prec;
    c.mode = mode;
    c.red = R_NONE;
    c.out_par = out_par;
    c.out = out;
    c.in = in;
    c.center = center;
    c.coef = coef;
    return c;
}

// out_e = D-hat_ee in_e (two MULTs, eq. 8); optional fused <aux, out> (and ||out||^2)
int dhat(wc_lattice *lat, int prec, void *out, const void *in, void *tmp, int red, const void *aux, RedTarget to,
         const int *done) {
    MultCall c1 = mc(prec, M_HOPINV, 1, tmp, in, nullptr, 0.0);
    c1.done = done;
    if (int rc = launch_mult(lat, c1)) return rc;
    MultCall c2 = mc(prec, M_DHAT, 0, out, tmp, in, -lat->kappa * lat->kappa);
    c2.red = red;
    c2.aux = aux;
    c2.red_to = to;
    c2.done = done;
    return launch_mult(lat, c2);
}

// v = M src: Algorithm 2 on the inner level (0) in the inner precision
int inner_solve(Ctx &C, const void *src, void *v) {
    wc_lattice *lat = C.lat;
    const int L = 0;
    const int *done = lat->level_flags(L);
    if (int rc = launch_norm2_p64(lat, src, red_target(lat, L, S_NORM))) return rc;
    if (int rc = launch_inner_init(lat, C.iprec, C.xprec, src, C.ir, C.irt, C.ip, C.ix, L)) return rc;
    lat->host_tol2[L] = C.fixed_work > 0 ? 0.0 : C.itol * C.itol;
    const int maxit = C.fixed_work > 0 ? C.fixed_work : C.imaxit;
    const double k2 = -lat->kappa * lat->kappa;
    (void)k2;
    int queued = 0;
    while (queued < maxit) {
        const int n = std::min(C.check_every, maxit - queued);
        for (int j = 0; j < n; j++) {
            const int k = queued + j;
            if (int rc = dhat(lat, C.iprec, C.iq, C.ip, C.itmp, R_DOT, C.irt, red_target(lat, L, S_RQ), done))
                return rc;
            if (int rc = launch_inner_a(lat, C.iprec, C.ir, C.iq, k, L)) return rc;
            if (int rc = dhat(lat, C.iprec, C.it, C.ir, C.itmp, R_DOTNORM, C.ir, red_target(lat, L, S_ST), done))
                return rc;
            if (int rc = launch_inner_b(lat, C.iprec, C.xprec, C.ix, C.ir, C.ip, C.it, C.irt, k, L)) return rc;
            if (int rc = launch_inner_c(lat, C.iprec, C.ip, C.ir, C.iq, k, L, true)) return rc;
        }
        queued += n;
        if (int rc = sync_scalars(lat)) return rc;
        if (hf(lat, L, F_DONE)) break;
    }
    const int code = hf(lat, L, F_DONE);
    int iters = hf(lat, L, F_ITERS);
    if (code == DONE_HALF) {
        if (int rc = launch_inner_fix(lat, C.iprec, C.xprec, C.ix, C.ip, iters, L)) return rc;
        iters += 1;
    }
    if (code == DONE_BREAK) C.inner_broke = true;
    C.info.inner_iters_total += iters;
    C.info.inner_calls += 1;
    return launch_inner_final(lat, C.xprec, v, C.ix, L);
}

// r = b-hat - D-hat x_e, ||r||^2 to the outer level's S_RR
int eo_residual(Ctx &C) {
    wc_lattice *lat = C.lat;
    if (int rc = dhat(lat, P64, C.q, C.x, C.tmp64, R_NONE, nullptr, RedTarget{}, nullptr)) return rc;
    return launch_sub_norm_p64(lat, C.r, C.bhat, C.q, red_target(lat, 1, S_RR));
}

// x_o from eq. 7 and the true residual of the full system; returns ||b - D x||^2
int reconstruct_and_check(Ctx &C, double &res2) {
    wc_lattice *lat = C.lat;
    char *xe = (char *)C.x, *xo = (char *)C.x + C.sb64;
    char *be = (char *)C.b, *bo = (char *)C.b + C.sb64;
    // x_o = F_oo^-1 (b_o + kappa H_oe x_e)
    if (int rc = launch_mult(lat, mc(P64, M_INVSRC, 1, xo, xe, bo, lat->kappa))) return rc;
    // (D x)_e = F_ee x_e - kappa H_eo x_o, (D x)_o likewise
    if (int rc = launch_mult(lat, mc(P64, M_DFULL, 0, C.q, xo, xe, -lat->kappa))) return rc;
    if (int rc = launch_sub_norm_p64(lat, C.res, be, C.q, red_target(lat, 1, S_AUX))) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    double re2 = hs(lat, 1, S_AUX);
    if (int rc = launch_mult(lat, mc(P64, M_DFULL, 1, C.tmp64, xe, xo, -lat->kappa))) return rc;
    if (int rc = launch_sub_norm_p64(lat, C.res, bo, C.tmp64, red_target(lat, 1, S_AUX))) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    res2 = re2 + hs(lat, 1, S_AUX);
    return WC_OK;
}

// Algorithm 1 from the current x_e; returns 0 when the recursive residual met tol_eo
int outer_flexible(Ctx &C, double src, double tol_eo, bool x_is_zero, bool &converged) {
    wc_lattice *lat = C.lat;
    const int L = 1;
    converged = false;
    if (x_is_zero) {
        if (int rc = launch_copy(lat, C.r, C.bhat, C.sb64)) return rc;
    } else {
        if (int rc = eo_residual(C)) return rc;
    }
    if (int rc = launch_norm2_p64(lat, C.r, red_target(lat, L, S_RHO0))) return rc;
    if (int rc = launch_copy(lat, C.rt, C.r, C.sb64)) return rc;
    if (int rc = launch_copy(lat, C.p, C.r, C.sb64)) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    double rr = hs(lat, L, S_RHO0);
    C.info.eo_rel_residual = std::sqrt(rr) / src;
    if (std::sqrt(rr) / src < tol_eo) {
        converged = true;
        return WC_OK;
    }
    for (int k = 0; k < C.omaxit; k++) {
        C.info.outer_iters++;
        // v = M p;  q = D-hat v with <r~, q>
        if (int rc = inner_solve(C, C.p, C.v)) return rc;
        if (int rc = dhat(lat, P64, C.q, C.v, C.tmp64, R_DOT, C.rt, red_target(lat, L, S_RQ), nullptr)) return rc;
        if (int rc = launch_outer_a(lat, C.x, C.r, C.v, C.q, k, L)) return rc;
        if (int rc = sync_scalars(lat)) return rc;
        rr = hs(lat, L, S_RR);
        C.info.eo_rel_residual = std::sqrt(rr) / src;
        if (!std::isfinite(rr)) return WC_EBREAKDOWN;
        if (std::sqrt(rr) / src < tol_eo) {
            converged = true;
            return WC_OK;
        }
        // v = M r;  t = D-hat v with <r, t>, ||t||^2
        if (int rc = inner_solve(C, C.r, C.v)) return rc;
        if (int rc = dhat(lat, P64, C.t, C.v, C.tmp64, R_DOTNORM, C.r, red_target(lat, L, S_ST), nullptr)) return rc;
        if (int rc = launch_outer_b(lat, C.x, C.r, C.v, C.t, C.rt, k, L)) return rc;
        if (int rc = sync_scalars(lat)) return rc;
        rr = hs(lat, L, S_RR);
        C.info.eo_rel_residual = std::sqrt(rr) / src;
        if (!std::isfinite(rr)) return WC_EBREAKDOWN;
        if (std::sqrt(rr) / src < tol_eo) {
            converged = true;
            return WC_OK;
        }
        const double r1re = hs(lat, L, (k + 1) & 1 ? S_RHO1 : S_RHO0);
        const double r1im = hs(lat, L, ((k + 1) & 1 ? S_RHO1 : S_RHO0) + 1);
        if (r1re == 0.0 && r1im == 0.0) return WC_EBREAKDOWN;
        if (int rc = launch_inner_c(lat, P64, C.p, C.r, C.q, k, L, false)) return rc;
    }
    return WC_OK;
}

// plain FP64 BiCGStab on D-hat_ee (the inner machinery in FP64), x_e += solution of
// D-hat v = r_e, repeated from the true residual until tol_eo is met
int fp64_pass(Ctx &C, double src, double tol_eo, bool x_is_zero, bool &converged) {
    wc_lattice *lat = C.lat;
    converged = false;
    if (x_is_zero) {
        if (int rc = launch_copy(lat, C.r, C.bhat, C.sb64)) return rc;
        if (int rc = launch_norm2_p64(lat, C.r, red_target(lat, 1, S_RR))) return rc;
    } else {
        if (int rc = eo_residual(C)) return rc;
    }
    if (int rc = sync_scalars(lat)) return rc;
    const double rn = std::sqrt(hs(lat, 1, S_RR));
    C.info.eo_rel_residual = rn / src;
    if (rn / src < tol_eo) {
        converged = true;
        return WC_OK;
    }
    C.info.outer_iters++;
    C.itol = tol_eo * src / rn;
    if (int rc = inner_solve(C, C.r, C.v)) return rc;
    if (int rc = launch_axpy_p64(lat, C.x, C.v, 1.0)) return rc;
    if (int rc = eo_residual(C)) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    const double rr = std::sqrt(hs(lat, 1, S_RR));
    C.info.eo_rel_residual = rr / src;
    converged = rr / src < tol_eo;
    return WC_OK;
}

}  // namespace

extern "C" int wc_solve(wc_lattice *lat, const void *b_dev, double kappa, double csw, double tol,
                        const wc_solve_params *pin, void *x_dev, int x0_is_guess, wc_solve_info *info) {
    if (!lat || !b_dev || !x_dev) return wc_fail(WC_EINVAL, "null argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return wc_fail(WC_EINVAL, "tol must lie in (0, 1)");
    wc_solve_params P;
    wc_solve_params_default(&P);
    if (pin) P = *pin;
    if (P.inner_prec < 0 || P.inner_prec > 2) return wc_fail(WC_EINVAL, "bad inner precision");
    if (P.inner_maxit < 1 || P.outer_maxit < 1 || P.check_every < 1 || P.fixed_work < 0 || P.inner_tol < 0.0 ||
        P.inner_tol >= 1.0)
        return wc_fail(WC_EINVAL, "bad solver parameters");
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "wc_solve before wc_load_links");
    auto t0 = std::chrono::steady_clock::now();
    if (!lat->have_clover || lat->kappa != kappa || lat->csw != csw) {
        if (int rc = wc_build_clover(lat, kappa, csw)) return rc;
    }
    Ctx C;
    std::memset(&C.info, 0, sizeof(C.info));
    C.lat = lat;
    C.iprec = P.inner_prec;
    C.xprec = (P.inner_prec == WC_FP64) ? P64 : P32;
    C.itol = P.inner_tol > 0.0 ? P.inner_tol : (P.inner_prec == WC_FP16 ? 1e-3 : 1e-6);
    C.imaxit = P.inner_maxit;
    C.omaxit = P.outer_maxit;
    C.fixed_work = P.fixed_work;
    C.check_every = P.check_every;
    C.sb64 = spinor_bytes(P64, lat->Vh);
    C.sbi = spinor_bytes(C.iprec, lat->Vh);
    C.sbx = spinor_bytes(C.xprec, lat->Vh);
    struct {
        int id;
        size_t bytes;
        void **p;
    } bufs[] = {
        {W_B, 2 * C.sb64, &C.b},   {W_X, 2 * C.sb64, &C.x},  {W_BHAT, C.sb64, &C.bhat}, {W_R, C.sb64, &C.r},
        {W_RT, C.sb64, &C.rt},     {W_P, C.sb64, &C.p},      {W_V, C.sb64, &C.v},       {W_Q, C.sb64, &C.q},
        {W_T, C.sb64, &C.t},       {W_TMP64, C.sb64, &C.tmp64}, {W_RES, C.sb64, &C.res}, {W_IR, C.sbi, &C.ir},
        {W_IRT, C.sbi, &C.irt},    {W_IP, C.sbi, &C.ip},     {W_IQ, C.sbi, &C.iq},      {W_IT, C.sbi, &C.it},
        {W_ITMP, C.sbi, &C.itmp},  {W_IX, C.sbx, &C.ix},
    };
    for (auto &bf : bufs)
        if (int rc = work_get(lat, bf.id, bf.bytes, bf.p)) return rc;
    const long dslash0 = lat->dslash_count;

    // b -> EO FP64; ||b||.  The adjoint system D^dag x = b is solved as
    // D y = g5 b, x = g5 y (g5 D g5 = D^dag).
    if (int rc = launch_pack_spinor(lat, P64, C.b, b_dev)) return rc;
    if (P.adjoint)
        if (int rc = launch_gamma5_p64(lat, C.b, 2)) return rc;
    char *be = (char *)C.b, *bo = (char *)C.b + C.sb64;
    if (int rc = launch_norm2_p64(lat, be, red_target(lat, 1, S_AUX))) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    double b2 = hs(lat, 1, S_AUX);
    if (int rc = launch_norm2_p64(lat, bo, red_target(lat, 1, S_AUX))) return rc;
    if (int rc = sync_scalars(lat)) return rc;
    b2 += hs(lat, 1, S_AUX);
    const double bnorm = std::sqrt(b2);
    if (bnorm == 0.0 || !std::isfinite(bnorm)) {
        if (!std::isfinite(bnorm)) return wc_fail(WC_EINVAL, "b has non-finite entries");
        WC_HIP(hipMemsetAsync(x_dev, 0, (size_t)lat->V * 12 * 16, lat->stream));
        WC_HIP(hipStreamSynchronize(lat->stream));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->status = WC_OK;
        }
        return WC_OK;
    }
    // b-hat_e = F_ee^-1 (b_e + kappa H_eo F_oo^-1 b_o)      (eq. 6)
    if (int rc = launch_mult(lat, [&] {
            MultCall c = mc(P64, M_CLOV, 1, C.tmp64, nullptr, bo, 0.0);
            c.inverse = true;
            return c;
        }()))
        return rc;
    if (int rc = launch_mult(lat, mc(P64, M_INVSRC, 0, C.bhat, C.tmp64, be, lat->kappa))) return rc;
    if (int rc = launch_norm2_p64(lat, C.bhat, red_target(lat, 1, S_AUX))) return rc;
    bool x_zero = true;
    if (x0_is_guess) {
        if (int rc = launch_pack_spinor(lat, P64, C.x, x_dev)) return rc;
        if (P.adjoint)
            if (int rc = launch_gamma5_p64(lat, C.x, 2)) return rc;
        x_zero = false;
    } else {
        if (int rc = launch_zero(lat, C.x, 2 * C.sb64)) return rc;
    }
    if (int rc = sync_scalars(lat)) return rc;
    const double src = std::sqrt(hs(lat, 1, S_AUX));
    const double tol_eo = 0.5 * tol * bnorm / src;

    int status = WC_ENOCONV;
    const int max_restarts = 6;
    for (int pass = 0; pass < max_restarts; pass++) {
        bool conv = false;
        int rc = (C.iprec == WC_FP64) ? fp64_pass(C, src, tol_eo, x_zero && pass == 0, conv)
                                      : outer_flexible(C, src, tol_eo, x_zero && pass == 0, conv);
        if (rc == WC_EBREAKDOWN) {
            C.info.restarts++;
            continue;
        }
        if (rc) return rc;
        double res2 = 0.0;
        if (int rc2 = reconstruct_and_check(C, res2)) return rc2;
        C.info.true_rel_residual = std::sqrt(res2) / bnorm;
        if (C.info.true_rel_residual <= tol) {
            status = WC_OK;
            break;
        }
        if (!conv && C.iprec != WC_FP64) break;  // iteration cap: give up
        C.info.restarts++;
    }
    if (P.adjoint)
        if (int rc = launch_gamma5_p64(lat, C.x, 2)) return rc;
    if (int rc = launch_unpack_spinor(lat, P64, x_dev, C.x)) return rc;
    WC_HIP(hipStreamSynchronize(lat->stream));
    auto t1 = std::chrono::steady_clock::now();
    C.info.seconds = std::chrono::duration<double>(t1 - t0).count();
    C.info.dslash_count = lat->dslash_count - dslash0;
    C.info.status = status;
    if (info) *info = C.info;
    if (status != WC_OK)
        return wc_fail(status, "solve stopped at true relative residual " + std::to_string(C.info.true_rel_residual));
    return WC_OK;
}
