// Host-side view of lattices and linear systems: device buffers, solver state,
// timing, and the batched kernel launchers shared by the C ABI and the solver
// drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "wc.h"
#include "common.hpp"

// ---------------------------------------------------------------------------
// device scalar block: one per solver level of each system.  Reductions write
// their final sums here and the update kernels read the BiCGStab coefficients
// from it, so no scalar round-trips through the host.
// ---------------------------------------------------------------------------
enum ScalarSlot {
    S_RQ = 0,      // <r~, q>            (complex, 2 doubles)
    S_SS = 2,      // ||s||^2  (half-step residual)
    S_ST = 3,      // <s, t>             (complex)
    S_TT = 5,      // ||t||^2
    S_RR = 6,      // ||r||^2
    S_RHO0 = 7,    // rho, slot 0        (complex)
    S_RHO1 = 9,    // rho, slot 1        (complex)
    // the pipelined inner loop keeps its coefficients in fixed slots:
    //   alpha in S_RQ, omega in S_ST, beta in S_RHO1, rho = <r~, r> in S_RHO0,
    //   <r~, s> and <r~, z> in S_AUX and S_AUX + 2, ||q||^2 in S_SS, ||y||^2 in S_TT
    S_NORM = 11,   // ||p||^2 of the inner call's source (Algorithm 2, first step)
    S_AUX = 12,    // scratch norms (4 doubles)
    S_TOL2 = 16,   // squared relative tolerance of the running inner loop
    S_COUNT = 20
};
// flags block (ints): done code, iterations completed
// F_STOPPH: where the inner loop stopped: 1 at the half-step check (after the
// first D-hat), 2 at the full-step check (after the second), 3 when a grid
// barrier of the one-launch loop ran out of time (the call then fails)
enum FlagSlot { F_DONE = 0, F_ITERS = 1, F_STOPPH = 2, F_COUNT = 4 };
enum DoneCode { DONE_NO = 0, DONE_FULL = 1, DONE_HALF = 2, DONE_BREAK = 4 };

enum { NUM_LEVELS = 2 };  // 0 = inner loop, 1 = outer / FP64 loop
constexpr int kMaxSys = 16;  // systems per batched launch
constexpr int kMaxRed = 8;   // values one fused reduction may carry (partials are sized for it)
// block sizes the solver's per-site kernels may run with (64-site tiles per
// block: 1, 2 or 4); reduction partials are sized for the smallest
constexpr int kMinBlock = 64;
inline bool valid_block_size(int bs) { return bs == 64 || bs == 128 || bs == 256; }
__host__ __device__ inline int blocks_of(int Vh, int bs) { return (Vh + bs - 1) / bs; }
// block size of a launch given a call's field (0 = the default 256)
inline int launch_bs(int bs) { return bs ? bs : 256; }
// the block size that calls on lat in precision prec use now: pinned, else
// tuned, else 256
inline int lattice_bs(const wc_lattice *lat, int prec);
constexpr float kRecon8MinN = 1e-6f;  // smallest |U01|^2 + |U02|^2 reconstruct-8 accepts
// largest |third column - conj(col0 x col1)| over the links for which the
// two-column forms (FP32 reconstruct-12 and -8, FP16) are accepted; above it
// the links are not SU(3) to single precision and FP32 keeps them in full
constexpr float kSU3MaxErr = 1e-5f;

// kinds of timed kernel launches
enum KernelSlot {
    KS_MULT_HOPINV_P64, KS_MULT_HOPINV_P32, KS_MULT_HOPINV_P16,
    KS_MULT_DHAT_P64, KS_MULT_DHAT_P32, KS_MULT_DHAT_P16,
    KS_MULT_OTHER,
    KS_BLAS,
    KS_COUNT
};

// One timed launch.  Inner-loop launches carry the iteration and phase they
// belong to (phase 0: first D-hat and the s update, 1: second D-hat and the
// x, r update, 2: the p update) and their algorithmic bytes split by system
// (keyed by the system's flag block) and by lattice operator (keyed by the
// flag blocks of the systems that share it), so that the work of systems
// that had already converged -- those kernels return at once -- can be taken
// out afterwards.
struct TimedPart {
    std::vector<const int *> owners;  // the part counts while any owner still runs
    double bytes;
};
struct TimedLaunch {
    int slot;
    double bytes;
    hipEvent_t a, b;
    int iter = -1, phase = 0;
    std::vector<TimedPart> parts;
    bool skipped = false;  // every system of the launch had stopped: no work done
};

// One linear system's device-side solver state: scalar and flag blocks per
// level, reduction partials, and pinned host mirrors.  The scalars and flags
// of the systems of one solve sit in one contiguous arena so that a single
// copy brings all of them to the host.
struct SysState {
    double *scalars = nullptr;     // [NUM_LEVELS][S_COUNT]
    int *flags = nullptr;          // [NUM_LEVELS][F_COUNT]
    double *partials = nullptr;    // [kMaxRed][blocks]: room for the 64-thread block count of the lattice
    size_t partials_bytes = 0;
    double *partials2 = nullptr;   // a second set, for the one-launch inner loop (single-system state only)
    unsigned long long *bar = nullptr;  // its grid barrier: [blocks] arrivals, release, abort (zeroed once)
    unsigned int bar_epoch = 0;         // one-launch calls so far (tags of a call exceed all earlier ones)
    double *h_scalars = nullptr;   // pinned mirror
    int *h_flags = nullptr;
    double *sc(int lvl) const { return scalars + lvl * S_COUNT; }
    int *fl(int lvl) const { return flags + lvl * F_COUNT; }
    double hs(int lvl, int slot) const { return h_scalars[lvl * S_COUNT + slot]; }
    int hf(int lvl, int slot) const { return h_flags[lvl * F_COUNT + slot]; }
};

// captured inner-loop chunks, keyed by (active systems, precision, length)
struct GraphEntry {
    unsigned long long key;
    hipGraphExec_t exec;
};

struct Arena {
    int S = 0;
    double *scalars = nullptr;
    int *flags = nullptr;
    double *h_scalars = nullptr;
    int *h_flags = nullptr;
    std::vector<GraphEntry> graphs;  // valid while the systems' buffers stay in place
};
void arena_drop_graphs(Arena &a);

struct wc_lattice;

// work buffers of one system in a solve (FP64 state and inner-precision state)
enum WorkId {
    W_B = 0,  // b, both parities
    W_X,      // x, both parities
    W_BHAT,   // b-hat_e
    W_R, W_RT, W_P, W_V, W_Q, W_T, W_TMP64, W_RES,   // single parity
    W_IR, W_IRT, W_IP, W_IQ, W_IT, W_ITMP, W_IX,     // inner precision
    W_IW, W_IS, W_IZ, W_IV,                          // inner precision, pipelined loop only
    W_SYS_COUNT
};

struct SysWork {
    void *buf[W_SYS_COUNT] = {};
    size_t bytes[W_SYS_COUNT] = {};
};

// A cached set of systems (arena, per-system partials and work vectors) for
// batched solves on a given list of lattices.
struct BatchCache {
    std::vector<unsigned long long> serials;  // serial numbers of its lattices (wc_lattice::serial)
    Arena arena;
    std::vector<SysState> sys;
    std::vector<SysWork> work;
};

// lattice-owned scratch buffers (operator applications, gradients)
enum LatWorkId { LW_APPLY_IN = 0, LW_APPLY_OUT, LW_APPLY_TMP, LW_GLAM, LW_GX, LW_GN, LW_COUNT };

struct wc_lattice {
    // process-unique number of this handle (never reused, unlike its address):
    // cached batches and recorded graphs name their lattices by it
    unsigned long long serial = 0;
    Geom g;
    int dims[4];
    long V;
    int Vh;
    int nblocks;   // 256-thread blocks covering one parity
    hipStream_t stream = nullptr;
    // threads per block of the solver's stencil and vector launches: pinned
    // by the caller, else chosen per precision by the tuner (0 = not yet)
    int bs_pin = 0;
    int bs_tuned[3] = {0, 0, 0};
    // systems per thread of the multi-system stencil that batched solves on
    // this lattice use in their inner loop (2 or 4), 0 for one system per
    // thread, -1 for the default of the precision (mrhs_for)
    int mrhs = -1;
    // stretch of sites, in 64-site tiles, that the stencils' block remap hands
    // to one XCD at a time (0: one contiguous slab per XCD): pinned by the
    // caller (>= 0), else tuned per precision with the block size (-1 = not yet)
    int chunk_pin = -1;
    int chunk_tuned[3] = {-1, -1, -1};
    int chunk_force = -1;  // set by the tuner while it times a candidate
    // waves per CU that the one-system stencils are held to, per precision:
    // pinned by the caller (>= 0; 0 = no cap), else tuned per kernel class
    // ([0]: MULT and the other stencils, [1]: the D-hat half) with the block
    // size, else the precision's default (wave_cap_for); the LDS bytes per CU
    // of the device, through which the cap is applied
    int wave_cap[3] = {-1, -1, -1};
    int cap_tuned[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
    int cap_force = -1;  // set by the tuner while it times a candidate
    int lds_per_cu = 0;

    // gauge links per precision: 8 slabs ([mu][parity]) of link_slab_bytes
    void *links[3] = {nullptr, nullptr, nullptr};
    // reconstruct-8 FP32 copy (8 slabs of link8_slab_bytes), built on request;
    // recon = 8 makes the FP32 stencils read it
    void *links8 = nullptr;
    // full FP32 copy (8 slabs of link18_slab_bytes): recon = 18
    void *links18 = nullptr;
    int recon = 12;
    bool recon_auto = false;        // 18 chosen by wc_load_links for links that are not SU(3)
    int recon_user = 12;            // the form last chosen by the caller, restored for SU(3) links
    unsigned *recon_min = nullptr;  // device word: smallest N as FP32 bits
    unsigned *recon_err = nullptr;  // device word: largest reconstruct-12 error as FP32 bits
    unsigned *clov_bad = nullptr;   // device word: clover blocks that are not positive definite
    float su3_err = 0.f;            // that error for the loaded links (0 before any)
    // clover F and F^-1 per precision: 2 slabs ([parity]) of clover_slab_bytes
    void *clov[3] = {nullptr, nullptr, nullptr};
    void *clovinv[3] = {nullptr, nullptr, nullptr};
    bool have_links = false, have_clover = false;
    double kappa = 0.0, csw = 0.0;
    unsigned gen = 0;              // bumped whenever links or clover change (invalidates captured graphs)
    hipStream_t capture_stream = nullptr;  // private stream that records graphs

    // single-system state (operator calls and non-batched solves)
    Arena arena;
    SysState sys;
    SysWork swork;
    void *lwork[LW_COUNT] = {};
    size_t lwork_bytes[LW_COUNT] = {};
    BatchCache *batch = nullptr;   // last batched solve's systems, reused when the lattices match

    // timing
    bool timing = false;
    int tag_iter = -1, tag_phase = 0;  // inner-loop position of the launches being queued
    std::vector<TimedLaunch> launches;
    std::vector<hipEvent_t> event_pool;
    long dslash_count = 0;
};

// systems per thread of the multi-system stencil in precision prec: the
// setting, else 2 for FP32 and 4 for FP16 (the faster of the two in each
// precision on the 12-source batch)
inline int mrhs_for(const wc_lattice *lat, int prec) {
    if (lat->mrhs >= 0) return lat->mrhs;
    return prec == P16 ? 4 : 2;
}

// the link copy a stencil in precision prec reads, and its slab size
inline const void *link_base(const wc_lattice *lat, int prec) {
    if (prec == P32 && lat->recon == 8) return lat->links8;
    if (prec == P32 && lat->recon == 18) return lat->links18;
    return lat->links[prec];
}
inline size_t link_slab_for(const wc_lattice *lat, int prec) {
    if (prec == P32 && lat->recon == 8) return link8_slab_bytes(lat->Vh);
    if (prec == P32 && lat->recon == 18) return link18_slab_bytes(lat->Vh);
    return link_slab_bytes(prec, lat->Vh);
}

constexpr int kDefaultChunk = 32;  // tiles per XCD chunk before tuning
inline int lattice_chunk(const wc_lattice *lat, int prec) {
    if (lat->chunk_force >= 0) return lat->chunk_force;
    if (lat->chunk_pin >= 0) return lat->chunk_pin;
    const int t = lat->chunk_tuned[prec];
    return t >= 0 ? t : kDefaultChunk;
}

inline int lattice_bs(const wc_lattice *lat, int prec) {
    if (lat->bs_pin) return lat->bs_pin;
    const int t = lat->bs_tuned[prec];
    return t ? t : 256;
}

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

// allocation helpers (capi.cpp)
int dev_alloc(void **p, size_t bytes);
int buf_get(void **slot, size_t *have, size_t bytes, hipStream_t s);  // grow-only device buffer
int arena_alloc(Arena &a, int S, hipStream_t s);
void arena_free(Arena &a);
void arena_bind(Arena &a, int k, SysState &st);
int sync_arena(const Arena &a, hipStream_t s);

// ---------------------------------------------------------------------------
// timing hooks around launches
// ---------------------------------------------------------------------------
void timing_begin(wc_lattice *lat, int slot, double bytes, TimedLaunch &t);
void timing_end(wc_lattice *lat, TimedLaunch &t);
// after an inner solve: take out the bytes of systems that had stopped before
// each tagged launch of lat->launches[from..]; stop = (iteration, phase) per
// flag block
struct StopPoint {
    const int *fl;
    int iter, phase;
};
void timing_settle(wc_lattice *lat, size_t from, const std::vector<StopPoint> &stops);

// ---------------------------------------------------------------------------
// reductions: target of stage 1, and stage 2 (blas.hip)
// ---------------------------------------------------------------------------
struct RedTarget {
    double *partials;
    double *result;  // final sums written here (FIN_STORE)
};

enum FinOp {
    FIN_STORE = 0,   // result[0..n) = sums
    FIN_INIT,        // rho0 = (sum, 0); reset the level's done flag and iteration count
    FIN_INNER_A,     // ||s||^2; done = HALF below tol2, BREAK on a non-finite alpha or sum
    FIN_INNER_B,     // ||r||^2, rho1 = <r~, r>, iterations = iter + 1; done = FULL / BREAK
    FIN_OUTER_B,     // ||r||^2, rho1 = <r~, r>
    FIN_PIPE_INIT,   // alpha = rho / <r~, w>, beta = 0, omega = 1 (no partials)
    FIN_PIPE_A,      // omega = <y, q> / ||y||^2; <r~, s>, <r~, z>; done = HALF on ||q||^2 < tol2
    FIN_PIPE_B       // rho, beta, next alpha, ||r||^2; iterations + 1; done = FULL / BREAK
};
// second stage of one system's reduction: sums `blocks` partials per value in
// block order, then applies `op` in one thread
struct FinArgs {
    int blocks;
    int op;
    const double *partials;
    double *result;    // FIN_STORE destination
    double *sc;        // scalar block of the level
    int *fl;           // flag block of the level
    const int *guard;  // skip when *guard != 0 (the producing kernel skipped too); may be null
    int iter;
    double tol2;
};
// one block per system; nvals values per system (1..3)
int launch_fin_batch(hipStream_t s, const FinArgs *f, int n, int nvals);

// ---------------------------------------------------------------------------
// stencil launches (dslash.hip).  A batch is a list of calls with the same
// precision, mode, reduction and output parity; one launch covers all of
// them.  Calls on one lattice are interleaved block by block so that the
// blocks that read the same links and clover run together on one XCD.
// ---------------------------------------------------------------------------
enum MultMode { M_HOPINV = 0, M_DHAT = 1, M_DFULL = 2, M_INVSRC = 3, M_HOP = 4, M_CLOV = 5 };
enum MultRed { R_NONE = 0, R_DOT = 1, R_DOTNORM = 2 };

// The FP64 stencil (140-196 VGPRs) runs 3 workgroups of 256 threads per CU
// when left alone; held to 2 (8 waves per CU) its L2 keeps more of the
// neighbours that the resident waves share, and MULT and D-hat run 10-11%
// faster at 32^3x64 and 48^3x96.  The FP32 and FP16 stencils have no cap
// unless the tuner finds one that pays on the lattice at hand.
constexpr int kDefaultWaveCap64 = 8;
inline int cap_class(int mode) { return mode == M_DHAT ? 1 : 0; }
inline bool valid_wave_cap(int w) { return w == 0 || (w >= 4 && w <= 16 && w % 4 == 0); }
inline int default_wave_cap(int prec) { return prec == P64 ? kDefaultWaveCap64 : 0; }
inline int wave_cap_for(const wc_lattice *lat, int prec, int mode = M_HOPINV) {
    if (lat->cap_force >= 0) return lat->cap_force;
    if (lat->wave_cap[prec] >= 0) return lat->wave_cap[prec];
    const int t = lat->cap_tuned[prec][cap_class(mode)];
    return t >= 0 ? t : default_wave_cap(prec);
}
// Dynamic LDS bytes per workgroup that leave room for exactly b = cap / (bs / 64)
// workgroups of bs threads on a CU (0 = no cap).  A workgroup's allocation
// must lie in (L / (b + 1), L / b] for L bytes of LDS per CU; the bytes are
// taken from the middle of that window, less the kernel's own few bytes of
// LDS, so that rounding up to the allocation granule keeps them inside it.
inline unsigned cap_lds_bytes(const wc_lattice *lat, int prec, int bs, int mode = M_HOPINV) {
    const int cap = wave_cap_for(lat, prec, mode);
    const int L = lat->lds_per_cu;
    if (cap <= 0 || L <= 0) return 0;
    int blocks = cap / (bs / 64);
    if (blocks < 1) blocks = 1;
    const int per = (L / blocks + L / (blocks + 1)) / 2 / 128 * 128 - 128;
    return per > 0 ? (unsigned)per : 0u;
}

struct MultCall {
    wc_lattice *lat;
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
    const int *done;     // skip this call when *done != 0
    int bs;              // threads per block of the launch (64, 128 or 256; 0 = 256)
};
// timing_lat (default: the first call's lattice) receives the timing record
int launch_mult_batch(hipStream_t s, const MultCall *calls, int n, wc_lattice *timing_lat = nullptr);
// one call on lat; a call without a block size takes the lattice's
inline int launch_mult(wc_lattice *lat, MultCall c) {
    c.lat = lat;
    if (!c.bs) c.bs = lattice_bs(lat, c.prec);
    return launch_mult_batch(lat->stream, &c, 1);
}
// time the stencil pair of the inner loop at each block size and keep the
// fastest for (lat, prec) (capi.cpp); us[3] and chosen may be null
int tune_block_size(wc_lattice *lat, int prec, double us[3], int *chosen);

// the inner loop of one system as a single cooperative launch (dslash.hip)
struct PersistCall {
    wc_lattice *lat;
    int prec;
    void *r, *rt, *p, *q, *t, *tmp, *x;
    double *part0, *part1;  // two partial buffers, at least kMaxRed x nblocks doubles each
    double *sc;
    int *fl;
    int maxit;
    unsigned long long *bar;  // nblocks + 2 words, zero before the first call
    unsigned int epoch;       // distinct and increasing per call on one bar
};
// longest a block of the one-launch loop waits at a grid barrier before the
// call gives up (seconds)
extern std::atomic<double> g_barrier_timeout_s;
int launch_inner_persistent(const PersistCall &c, hipStream_t s, bool *ran);

// ---------------------------------------------------------------------------
// vector kernels (blas.hip), batched the same way; one call per system
// ---------------------------------------------------------------------------
enum VecOp {
    V_NORM2,        // a: v (FP64)                       -> result[0] = ||v||^2, result[1] = 0
    V_SUB_NORM,     // a = b - c (FP64)                   -> result[0] = ||a||^2
    V_AXPY,         // a += coef b (FP64)
    V_INNER_INIT,   // a: src (FP64), b: r, c: r~, d: p, e: x   (Algorithm 2 set-up)
    V_INNER_A,      // a: r, b: q                         r -= alpha q
    V_INNER_B,      // a: x, b: r, c: p, d: t, e: r~      x += alpha p + omega s, r = s - omega t
    V_INNER_C,      // a: p, b: r, c: q                   p = r + beta (p - omega q)
    V_INNER_FIX,    // a: x, b: p                         x += alpha p
    V_INNER_FINAL,  // a: v (FP64), b: x                  v = ||src|| x
    V_OUTER_A,      // a: x, b: r, c: v, d: q             x += alpha v, r -= alpha q
    V_OUTER_B,      // a: x, b: r, c: v, d: t, e: r~      x += omega v, r -= omega t
    V_GAMMA5,       // a: FP64 two-parity field, in place
    V_COPY,         // a = b (FP64 single parity)
    V_ZERO,         // a = 0 (FP64 single parity)
    // pipelined BiCGStab (the inner-solver variant with two reduction phases)
    V_PIPE_INIT,    // a: src (FP64), b: r, c: r~, d: x, e: p, f: s, g: z, h: v   (set-up)
    V_PIPE_A,       // a: r, b: w, c: t, d: p, e: s, f: z, g: v, h: r~      (p, s, z updates)
    V_PIPE_B,       // a: x, b: p, c: r, d: s, e: w, f: z, g: t, h: v, j: r~ (x, r, w updates)
    V_PIPE_FIX      // a: x, b: p                         x += alpha p (alpha from its slot)
};

struct VecCall {
    int Vh;
    void *a, *b, *c, *d, *e, *f, *g, *h, *j;
    double *sc;        // scalar block of the system's level
    int *fl;           // flag block of the system's level
    double *partials;
    double *result;    // V_NORM2 / V_SUB_NORM destination
    double tol2;
    double coef;
    int iter;          // iteration index, when not taken from the device
    int guard;         // skip when fl[F_DONE] != 0
    int iter_dev;      // take the iteration index from fl[F_ITERS] (inner loop)
    int bs;            // threads per block of the launch (64, 128 or 256; 0 = 256)
};
// prec: storage precision of the inner vectors (the inner solution x is FP64
// for an FP64 loop and FP32 otherwise).  timing_lat (may be null) receives the
// timing record of the launch.
int launch_vec_batch(hipStream_t s, wc_lattice *timing_lat, int op, int prec, const VecCall *calls, int n);

// ---------------------------------------------------------------------------
// other launchers
// ---------------------------------------------------------------------------
int launch_pack_spinor(wc_lattice *lat, int prec, void *eo_out, const void *canon_in);
int launch_unpack_spinor(wc_lattice *lat, int prec, void *canon_out, const void *eo_in);
// converts U to the per-precision copies and posts the largest
// reconstruct-12 error into *err_bits (FP32 bits, atomic max)
int launch_load_links(wc_lattice *lat, const void *U, unsigned *err_bits);
int launch_links_recon8(wc_lattice *lat, unsigned *min_bits);
int launch_links_full32(wc_lattice *lat);  // links18 from the FP64 copy
// builds F and F^-1; *bad_blocks (device word, zeroed by the caller) receives the
// number of 6x6 blocks that are not positive definite
int launch_build_clover(wc_lattice *lat, double kappa, double csw, unsigned *bad_blocks);
int launch_link_grad(wc_lattice *lat, const void *lam_eo, const void *x_eo, void *G, void *Nbuf, double kappa,
                     double csw, bool clover);

// solver entry used by wc_solve and the batched solves (solver.cpp)
struct SolveSys {
    wc_lattice *lat;
    SysState *st;
    SysWork *work;
    const void *b_dev;
    void *x_dev;
    double kappa, csw;
    wc_solve_info info;
    int status;
};
// every system's SysState must be bound to `arena`; the work vectors of every
// system must exist (capi.cpp allocates them); all work runs on the first
// system's lattice stream.  Returns a HIP / argument error, else WC_OK with the
// per-system outcome in sys[k].status and sys[k].info.
int solve_systems(std::vector<SolveSys> &sys, Arena &arena, double tol, const wc_solve_params &P,
                  int x0_is_guess);
