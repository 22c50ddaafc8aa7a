// Host-side view of a lattice: device buffers, scalar blocks, timing, and the
// kernel launchers shared between the C ABI and the solver drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "wc.h"
#include "common.hpp"

// ---------------------------------------------------------------------------
// device scalar block: one per solver level (inner, outer, batch slots).
// Reductions write their final sums here and the update kernels read the
// BiCGStab coefficients from it, so no scalar round-trips through the host.
// ---------------------------------------------------------------------------
enum ScalarSlot {
    S_RQ = 0,      // <r~, q>            (complex, 2 doubles)
    S_SS = 2,      // ||s||^2  (half-step residual)
    S_ST = 3,      // <s, t>             (complex)
    S_TT = 5,      // ||t||^2
    S_RR = 6,      // ||r||^2
    S_RHO0 = 7,    // rho, slot 0        (complex)
    S_RHO1 = 9,    // rho, slot 1        (complex)
    S_NORM = 11,   // source norm ||p|| of the inner call (Algorithm 2, first step)
    S_AUX = 12,    // scratch norm / dot (3 doubles)
    S_TOL2 = 15,   // tol^2 * ||b||^2 target of the running loop
    S_COUNT = 16
};
// flags block (ints): done code, iterations completed
enum FlagSlot { F_DONE = 0, F_ITERS = 1, F_COUNT = 4 };
enum DoneCode { DONE_NO = 0, DONE_FULL = 1, DONE_HALF = 2, DONE_BREAK = 4 };

enum { NUM_LEVELS = 2 };  // 0 = inner loop, 1 = outer / FP64 loop

// kinds of timed kernel launches
enum KernelSlot {
    KS_MULT_HOPINV_P64, KS_MULT_HOPINV_P32, KS_MULT_HOPINV_P16,
    KS_MULT_DHAT_P64, KS_MULT_DHAT_P32, KS_MULT_DHAT_P16,
    KS_MULT_OTHER,
    KS_BLAS,
    KS_COUNT
};

struct TimedLaunch {
    int slot;
    double bytes;
    hipEvent_t a, b;
};

struct wc_lattice {
    Geom g;
    int dims[4];
    long V;
    int Vh;
    hipStream_t stream = nullptr;

    // gauge links per precision: 8 slabs ([mu][parity]) of link_slab_bytes
    void *links[3] = {nullptr, nullptr, nullptr};
    // clover F and F^-1 per precision: 2 slabs ([parity]) of clover_slab_bytes
    void *clov[3] = {nullptr, nullptr, nullptr};
    void *clovinv[3] = {nullptr, nullptr, nullptr};
    bool have_links = false, have_clover = false;
    double kappa = 0.0, csw = 0.0;

    // reductions
    double *partials = nullptr;      // [8][max_blocks]
    double *scalars = nullptr;       // [NUM_LEVELS][S_COUNT]
    int *flags = nullptr;            // [NUM_LEVELS][F_COUNT]
    double *host_scalars = nullptr;  // pinned mirror of scalars
    int *host_flags = nullptr;       // pinned mirror of flags
    int max_blocks = 0;
    double host_tol2[NUM_LEVELS] = {0.0, 0.0};  // convergence target (squared) handed to the kernels

    // solver work vectors, allocated on first use and kept until destroy
    void *work[32] = {};
    size_t work_bytes[32] = {};

    // timing
    bool timing = false;
    std::vector<TimedLaunch> launches;
    std::vector<hipEvent_t> event_pool;
    long dslash_count = 0;

    double *level_scalars(int lvl) { return scalars + lvl * S_COUNT; }
    int *level_flags(int lvl) { return flags + lvl * F_COUNT; }
};

// ---------------------------------------------------------------------------
// error reporting (thread-local text behind wc_last_error)
// ---------------------------------------------------------------------------
int wc_fail(int code, const std::string &msg);
#define WC_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return wc_fail(WC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// ---------------------------------------------------------------------------
// timing hooks around launches
// ---------------------------------------------------------------------------
void timing_begin(wc_lattice *lat, int slot, double bytes, TimedLaunch &t);
void timing_end(wc_lattice *lat, TimedLaunch &t);

// ---------------------------------------------------------------------------
// reduction target handed to kernels
// ---------------------------------------------------------------------------
struct RedTarget {
    double *partials;
    double *result;  // final sums written here (nres doubles)
};

inline RedTarget red_target(wc_lattice *lat, int lvl, int slot) {
    return RedTarget{lat->partials, lat->level_scalars(lvl) + slot};
}

// second stage of a reduction (blas.hip): sums the per-block partials in block
// order, then applies `op` in one thread
enum FinOp {
    FIN_STORE = 0,   // result[0..n) = sums
    FIN_INIT,        // rho0 = (sum, 0); reset the level's done flag and iteration count
    FIN_INNER_A,     // ||s||^2; done = HALF below tol2, BREAK on a non-finite alpha or sum
    FIN_INNER_B,     // ||r||^2, rho1 = <r~, r>, iterations = iter + 1; done = FULL / BREAK
    FIN_OUTER_B      // ||r||^2, rho1 = <r~, r>
};
struct FinArgs {
    int n;             // values per block (1..3)
    int blocks;        // number of partials per value
    int op;
    const double *partials;
    double *result;    // FIN_STORE destination
    double *sc;        // scalar block of the level
    int *fl;           // flag block of the level
    const int *guard;  // skip when *guard != 0 (the producing kernel skipped too); may be null
    int iter;
    double tol2;
};
int launch_finalize(wc_lattice *lat, const FinArgs &f);

// ---------------------------------------------------------------------------
// launchers (layout.hip, clover.hip, dslash.hip, blas.hip)
// ---------------------------------------------------------------------------
int launch_pack_spinor(wc_lattice *lat, int prec, void *eo_out, const void *canon_in);
int launch_unpack_spinor(wc_lattice *lat, int prec, void *canon_out, const void *eo_in);
int launch_load_links(wc_lattice *lat, const void *U);
int launch_build_clover(wc_lattice *lat, double kappa, double csw);

enum MultMode { M_HOPINV = 0, M_DHAT = 1, M_DFULL = 2, M_INVSRC = 3, M_HOP = 4, M_CLOV = 5 };
enum MultRed { R_NONE = 0, R_DOT = 1, R_DOTNORM = 2 };

struct MultCall {
    int prec;
    int mode;
    int red;
    int out_par;
    void *out;
    const void *in;      // other-parity input (hopping)
    const void *center;  // same-parity input (DHAT, DFULL, INVSRC, CLOV)
    const void *aux;     // same-parity vector of the fused dot <aux, out>
    double coef;
    bool inverse;        // CLOV: use F^-1 instead of F
    RedTarget red_to;
    const int *done;     // skip the launch body when *done != 0
};
int launch_mult(wc_lattice *lat, const MultCall &c);

// BLAS-1 (blas.hip); all vectors are single-parity EO slabs
int launch_norm2_p64(wc_lattice *lat, const void *v, RedTarget to);
int launch_sub_norm_p64(wc_lattice *lat, void *r, const void *a, const void *b, RedTarget to);  // r = a - b
int launch_copy(wc_lattice *lat, void *dst, const void *src, size_t bytes);
int launch_zero(wc_lattice *lat, void *dst, size_t bytes);
int launch_axpy_p64(wc_lattice *lat, void *y, const void *x, double a);  // y += a x

// inner BiCGStab (Algorithm 2) on storage precision prec, x kept in xprec
int launch_inner_init(wc_lattice *lat, int prec, int xprec, const void *src64, void *r, void *rt, void *p, void *x,
                      int lvl);
int launch_inner_a(wc_lattice *lat, int prec, void *r, const void *q, int iter, int lvl);
int launch_inner_b(wc_lattice *lat, int prec, int xprec, void *x, void *r, const void *p, const void *t,
                   const void *rt, int iter, int lvl);
int launch_inner_c(wc_lattice *lat, int prec, void *p, const void *r, const void *q, int iter, int lvl, bool guard);
int launch_inner_fix(wc_lattice *lat, int prec, int xprec, void *x, const void *p, int iter, int lvl);
int launch_inner_final(wc_lattice *lat, int xprec, void *v64, const void *x, int lvl);
// outer flexible BiCGStab (Algorithm 1), FP64
int launch_outer_a(wc_lattice *lat, void *x, void *r, const void *v, const void *q, int iter, int lvl);
int launch_outer_b(wc_lattice *lat, void *x, void *r, const void *v, const void *t, const void *rt, int iter,
                   int lvl);

// gradient kernels (grad.hip)
int launch_gamma5_p64(wc_lattice *lat, void *eo, int nslabs);
int launch_link_grad(wc_lattice *lat, const void *lam_eo, const void *x_eo, void *G, void *Nbuf, double kappa,
                     double csw, bool clover);
