/*
 * wc.h -- C ABI of the MI355X (gfx950) Wilson-clover quark-solver library.
 *
 * The library solves D x = b for the O(a)-improved Wilson ("clover") quark
 * operator of Boku, Ishikawa, Kuramashi and Meadows, arXiv:1709.08785:
 *
 *   D(n,m) = F(n) delta(n,m) - kappa H(n,m)                  (Sec. II-A, eq. 3)
 *   H psi(n) = sum_mu (1 - g_mu) U_mu(n) psi(n+mu)
 *            + (1 + g_mu) U_mu(n-mu)^dagger psi(n-mu)         (Sec. II-A, eq. 4)
 *
 * on a periodic 4-d lattice, through the even-odd (Schur) preconditioned
 * system D-hat_ee x_e = b-hat_e of Sec. II-B (eqs. 5-9) and the nested
 * (flexible) BiCGStab of Algorithms 1 and 2: an FP64 outer iteration whose
 * preconditioner is a low-precision (FP32, or FP16 storage with FP32
 * arithmetic) inner BiCGStab.
 *
 * Conventions (fixed by this library where the paper is silent):
 *   - gamma matrices in the Dirac representation:
 *       g_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z), g_t = diag(1, 1, -1, -1);
 *   - F(n) = 1 - kappa c_SW sum_{mu<nu} g_mu g_nu (x) Fhat_{mu nu}(n),
 *     Fhat = (Q - Q^dagger)/8 with Q the sum of the four counter-clockwise
 *     plaquettes at n (Sheikholeslami-Wohlert clover, no trace subtraction);
 *   - parity of site (x, y, z, t) is (x + y + z + t) mod 2, even = 0.
 *
 * Canonical layouts (device memory, complex128 = two doubles, C order), with
 * dims = {Lx, Ly, Lz, Lt}:
 *   links    U[mu][t][z][y][x][i][j], mu = x, y, z, t = 0..3; U_mu(n) is the
 *            3x3 matrix on the link n -> n + mu-hat;
 *   spinors  psi[t][z][y][x][alpha][a], spin alpha = 0..3, colour a = 0..2.
 *
 * Internal even-odd ("EO") layout: one parity of a spinor field holds V/2
 * sites, site n = x + Lx (y + Ly (z + Lz t)) stored at index i = n >> 1 of
 * its parity.  The parity is cut into tiles of 64 consecutive sites; a tile
 * holds its sites' data plane after plane, a plane being one group of 4 to
 * 16 bytes per site stored for all 64 sites contiguously, and the last tile
 * is padded.  wc_spinor_bytes() gives the
 * padded size of one parity in a given precision; a two-parity EO field
 * stores the even half first, then the odd half.  EO fields are meant to be
 * produced and read by wc_pack_spinor / wc_unpack_spinor.
 *
 * Ownership: every pointer passed in is owned by the caller.  Field pointers
 * are device pointers unless stated otherwise.  wc_load_links copies the
 * links into library-owned buffers, so the caller may free U afterwards.
 * All internal buffers are released by wc_destroy_lattice.
 *
 * Streams: every kernel runs on the stream given to wc_create_lattice (0 is
 * the null stream).  wc_apply_* calls are asynchronous on that stream.
 * wc_solve and wc_solve_batch return after the solve has finished.
 *
 * Devices: a lattice lives on the HIP device that is current when it is
 * created, and every later call on it must be made with that device
 * current; the library never switches devices.  Lattices given to one
 * wc_solve_multi call must live on the same device.
 *
 * Errors: every int-returning call returns WC_OK (0) or a negative wc_status.
 * Arguments are checked on the host before any GPU work (WC_EINVAL).  The
 * text of the last error of the calling thread is wc_last_error().  A
 * lattice handle must not be used from two threads at once.
 */
#ifndef WC_H
#define WC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wc_lattice wc_lattice;

enum wc_prec { WC_FP64 = 0, WC_FP32 = 1, WC_FP16 = 2 };

enum wc_status {
    WC_OK = 0,
    WC_EINVAL = -1,       /* bad argument (odd or zero extent, null pointer, bad enum) */
    WC_ENOMEM = -2,       /* device allocation failed */
    WC_EHIP = -3,         /* a HIP runtime call failed; see wc_last_error() */
    WC_ENOTREADY = -4,    /* no links loaded, or no clover term built */
    WC_ENOCONV = -5,      /* iteration cap reached before the tolerance */
    WC_EBREAKDOWN = -6    /* BiCGStab breakdown (zero or non-finite scalar) after restarts */
};

/* Solver parameters.  wc_solve_params_default() fills the defaults. */
typedef struct {
    int inner_prec;       /* WC_FP32 (default) or WC_FP16: storage precision of the inner
                             BiCGStab of Algorithm 2; WC_FP64 runs one plain FP64 BiCGStab
                             on D-hat_ee (no inner/outer nesting) */
    double inner_tol;     /* inner relative residual target (default 1e-6 FP32, 1e-3 FP16) */
    int inner_maxit;      /* inner iteration cap (default 5000; the iteration cap of WC_FP64) */
    int outer_maxit;      /* outer iteration cap (default 100) */
    int fixed_work;       /* >0: run exactly this many inner iterations per inner call, no
                             convergence test (the fixed-count timing mode of Sec. IV) */
    int check_every;      /* inner iterations queued between host convergence reads (default 8) */
    int adjoint;          /* != 0: solve D^dagger x = b instead, as g5 D^-1 g5 b (D is
                             gamma5-Hermitian: g5 D g5 = D^dagger); default 0 */
    int use_graph;        /* != 0 (default): record each chunk of check_every inner iterations
                             once as a HIP graph and replay it (not while kernel timing is on) */
    int outer;            /* outer iteration around the inner solver: WC_OUTER_BICGSTAB (default,
                             the flexible BiCGStab of Algorithm 1) or WC_OUTER_DC (defect
                             correction: x_e += M r_e, r_e recomputed in FP64 each step) */
    int inner_method;     /* WC_INNER_BICGSTAB (default, Algorithm 2) or WC_INNER_PIPELINED: the
                             pipelined BiCGStab of Cools and Vanroose (2017), the same iterates
                             with two reduction phases per iteration instead of four and
                             about 9 more vector passes; it also needs 4 more inner-precision
                             work vectors per system */
    int persistent;       /* != 0: a single-system solve runs each inner loop (Algorithm 2) as one
                             cooperative launch with grid-wide barriers between its phases, when
                             every workgroup of the lattice fits on the device at once (small
                             lattices: launch overhead dominates there); otherwise, for batches,
                             the pipelined loop or kernel timing, the launched loop runs.
                             Every wait at a grid barrier is bounded (wc_set_barrier_timeout):
                             a wait that runs out makes every workgroup leave the loop, and
                             the solve returns WC_EHIP.  Default 0. */
} wc_solve_params;

enum wc_outer { WC_OUTER_BICGSTAB = 0, WC_OUTER_DC = 1 };
enum wc_inner_method { WC_INNER_BICGSTAB = 0, WC_INNER_PIPELINED = 1 };

/* What a solve did.  Iteration counts follow Algorithms 1 and 2. */
typedef struct {
    int outer_iters;          /* outer (Algorithm 1) iterations, summed over restarts */
    int inner_iters_total;    /* inner (Algorithm 2) iterations summed over all inner calls */
    int inner_calls;          /* calls of the inner solver */
    int restarts;             /* outer restarts from the true residual */
    long dslash_count;        /* MULT applications (one D-hat_ee = 2 MULTs), any precision */
    int status;               /* same value as returned */
    double eo_rel_residual;   /* last recursive ||r_e|| / ||b-hat_e|| of the outer loop */
    double true_rel_residual; /* ||b - D x|| / ||b|| in FP64 on the full lattice */
    double seconds;           /* wall time of the solve (host clock, after the final sync) */
    int persistent_calls;     /* inner calls that ran as one cooperative launch (persistent) */
    int block_size;           /* threads per block of the solve's stencil and vector kernels */
} wc_solve_info;

void wc_solve_params_default(wc_solve_params *p);

/* Launch shape of the solver's per-site kernels (the counterpart of the site
   loop tiling of Sec. III-B).  Sites are stored in tiles of 64 (one tile per
   wavefront); a workgroup covers 1, 2 or 4 tiles, i.e. 64, 128 or 256
   threads.  Small lattices fill more compute units with small workgroups;
   large ones prefer large.  Unless pinned, the size is tuned per inner
   precision on the first solve of a lattice (wc_tune_block_size) and reused.
   Results do not depend on it beyond the rounding order of the reductions.

   wc_set_block_size: threads = 64, 128 or 256 pins the size for every
   precision; 0 returns to tuning.  WC_EINVAL for other values.
   wc_block_size: the size a solve with inner precision prec would use now
   (pinned, else tuned), or 0 when it is not yet tuned.
   wc_tune_block_size: times the inner loop's stencil pair (F^-1 H into the
   odd parity, then the D-hat half with its fused dot; Sec. II-B eq. 8) on
   zero vectors at 64, 128 and 256 threads and at XCD chunks of 8, 16, 32 and
   64 tiles (wc_set_xcd_chunk; only the pinned one when pinned) and keeps the
   fastest shape; 256 threads at chunk 32 are displaced only by a shape at
   least 3% faster, in the sweep and again in three alternating timings
   against it.  With a pinned block size, the chunk and caps are chosen
   for that size.  At that shape it then times the two kernels on their
   own under no cap and caps of 8 and 12 waves per CU (wc_set_wave_cap;
   skipped when pinned), and each kernel class keeps a cap only if it beats
   the precision's default by 3%, confirmed in the same way.  us_per_pair[3] (may be NULL) receives
   microseconds per pair for 64, 128, 256 at the chosen chunk under the
   default cap; *threads (may be NULL) the chosen block size.  With a tuning
   cache (wc_set_tune_cache) holding this case, the stored shape and caps are
   taken without timing; a tuning under a pinned block size or chunk neither
   reads nor writes the cache.
   Needs links and clover (WC_ENOTREADY).  Allocates three vectors of the
   precision for the duration of the call and synchronises the stream. */
int wc_set_block_size(wc_lattice *lat, int threads);
int wc_block_size(const wc_lattice *lat, int prec);
int wc_tune_block_size(wc_lattice *lat, int prec, double us_per_pair[3], int *threads);

/* The multi-system stencil of batched solves (wc_solve_batch, and systems of
   wc_solve_multi that share a lattice): many solutions per gauge field (Sec.
   II-A) apply the same operator, so the inner loop's MULTs (F^-1 H of eq. 9 and
   the second half of D-hat_ee, eq. 8) of all systems on one lattice run in one
   launch in which each thread takes one site for systems_per_thread systems:
   it computes the neighbour indices and rebuilds each link once, loads each
   clover block once, and applies them to every system's spinors.
   wc_set_multi_rhs: systems_per_thread = 2 or 4, 0 for one system per thread
   (each system's sites in workgroups of their own, the operator shared through
   the cache), or -1 (default) for 2 in FP32 and 4 in FP16, the faster setting
   of each precision on the 12-source batch.  WC_EINVAL for other values.
   Results agree with single solves to rounding.  wc_multi_rhs: systems per
   thread a batch in precision prec uses now (0 for FP64, which has no
   multi-system form), or -1 for a null lattice or bad precision. */
int wc_set_multi_rhs(wc_lattice *lat, int systems_per_thread);
int wc_multi_rhs(const wc_lattice *lat, int prec);

/* Order in which the stencils' workgroups visit the lattice.  Workgroups are
   handed to the device's 8 XCDs (each with its own L2) round-robin; the
   library remaps them so that each XCD takes chunks of `tiles` consecutive
   64-site tiles, the XCDs sweeping the lattice side by side (neighbours in y
   and z then fall in the XCD's own chunk).  tiles = 0 gives each XCD one
   contiguous slab instead.  Unless pinned, the chunk is tuned with the block
   size (wc_tune_block_size); before tuning it is 32.  Results do not depend
   on it.  wc_set_xcd_chunk: tiles in [0, 2^20] pins it for every precision,
   -1 returns to tuning; WC_EINVAL otherwise.  wc_xcd_chunk: the chunk a
   launch in precision prec uses now (-2 for a null lattice or bad prec). */
int wc_set_xcd_chunk(wc_lattice *lat, int tiles);
int wc_xcd_chunk(const wc_lattice *lat, int prec);

/* Occupancy cap of the one-system stencils (MULT, F^-1 H of Sec. II-B eq. 9,
   and the D-hat_ee halves of eq. 8, plus D of eqs. 3-4): at most waves_per_cu
   wavefronts of such a launch in precision prec share a compute unit.  The
   library applies it by reserving LDS that the kernels do not use, so results
   do not depend on it.  A cap that keeps fewer waves resident lets the L2
   keep more of the neighbour spinors those waves share: the FP64 stencil runs
   10-11% faster at 8 waves per CU than at the 12 its registers allow.
   Unless pinned, the cap is chosen per precision and per kernel class (the
   D-hat half, and every other stencil) by the launch-shape tuner
   (wc_tune_block_size) among no cap, 8 and 12 waves; before tuning it is 8
   for FP64 and none for FP32 and FP16.
   wc_set_wave_cap: 4, 8, 12 or 16 waves pins the cap of both classes, 0 pins
   no cap, -1 returns to tuning.  Changing it drops the tuned launch shape of
   that precision.  WC_EINVAL for other values or a bad precision.  Batches of
   several systems on one lattice take no cap.
   wc_wave_cap: the cap that launches in prec use now, for the D-hat half
   (dhat != 0) or the other stencils (dhat = 0); 0 = none, also when the
   device does not report its LDS size; -2 for a null lattice or bad prec. */
int wc_set_wave_cap(wc_lattice *lat, int prec, int waves_per_cu);
int wc_wave_cap(const wc_lattice *lat, int prec, int dhat);

/* Process-wide file in which the launch-shape tuner keeps its results, one
   line per device (architecture and compute units), lattice extents,
   precision, FP32 link form and pinned wave cap (wc_set_wave_cap); a later
   tuning of the same case, in this process or another, takes the stored
   shape instead of timing.  Tunings under a pinned block size or XCD chunk
   do not use the file.  path NULL or
   "" (the default) keeps no file.  A file that cannot be read or written only
   costs a new timing.  The path is copied. */
int wc_set_tune_cache(const char *path);

/* Longest time (seconds, > 0 finite, or 0 for "no waiting allowed") a
   workgroup of the one-launch inner loop (wc_solve_params.persistent) waits
   at a grid barrier before the call gives up with WC_EHIP.  Process-wide;
   default 2 s, far above a barrier's microseconds.  Returns WC_EINVAL for a
   negative or non-finite value. */
int wc_set_barrier_timeout(double seconds);

/* Create a lattice of extents dims = {Lx, Ly, Lz, Lt}; every extent even and >= 2
   (the even-odd split of Sec. II-B with periodic wrap needs even extents).
   stream is a hipStream_t (NULL = null stream).  *out receives the handle. */
int wc_create_lattice(const int dims[4], void *stream, wc_lattice **out);
void wc_destroy_lattice(wc_lattice *lat);
/* Rebind the stream used for all later work on this lattice. */
int wc_set_stream(wc_lattice *lat, void *stream);

/* Copy gauge links (canonical complex128 layout, device pointer) into the internal
   FP64, FP32 and FP16 copies.  FP32 and FP16 keep the first two columns of each
   matrix and rebuild the third as conj(col0 x col1) (SU(3) reconstruction,
   Sec. III-A); this is exact only for special-unitary links.  The call
   measures, in FP64, the largest |third column - conj(col0 x col1)| entry over
   all links (wc_link_su3_error; it synchronises the stream).  Above 1e-5 the
   links are not SU(3) to single precision: the lattice then switches the FP32
   stencil to full links (wc_set_link_recon 18) and refuses FP16 stencil work
   (WC_EINVAL); a later load of SU(3) links returns it to the form the caller
   last chose (12 by default).  Invalidates the clover term.  Links with a
   non-finite entry are refused with WC_EINVAL, and the lattice then has no
   links until a successful load. */
int wc_load_links(wc_lattice *lat, const void *U_dev);
/* The reconstruction error measured by the last wc_load_links (0 before any; -1
   for a null lattice). */
double wc_link_su3_error(const wc_lattice *lat);

/* Choose how the FP32 stencil stores links (Sec. III-A: each MULT reads every
   link once, so links are 44% of its bytes): recon = 12 (default, two columns,
   48 B), 8 (eight reals, 32 B: U01, U02, the smaller in modulus of U10 and
   U20, and the phases of U00 and of the other one; the remaining entries follow
   from unitarity and det U = 1, exact up to a few FP32 rounding steps) or 18
   (the full matrix, 72 B: for links that are not SU(3); 12 and 8 are refused
   with WC_EINVAL for such links).  FP64 always keeps full matrices; FP16 always
   keeps two columns (rebuilding from eight half-precision reals loses too many
   of its bits), so FP16 stencil work needs SU(3) links.  recon = 8 builds the
   extra copy from the loaded links and returns WC_EINVAL, leaving the setting
   unchanged, if some link has |U01|^2 + |U02|^2 < 1e-6 (unit links, for
   instance); WC_ENOTREADY before wc_load_links.  A later wc_load_links rebuilds
   the copy; if the new links fail the same check it returns WC_EINVAL and the
   lattice falls back to 12 (the links themselves are loaded).  Applies to every
   later FP32 apply and solve on this lattice; one batched solve needs the same
   setting on all its lattices. */
int wc_set_link_recon(wc_lattice *lat, int recon);
/* The current setting (12, 8 or 18); 0 for a null lattice. */
int wc_link_recon(const wc_lattice *lat);

/* Build the clover term F (Sec. II-A) from the loaded links in FP64, split into
   its two 6x6 Hermitian chiral blocks (Sec. III-A), invert them in FP64 (the
   inverses F_ee^-1, F_oo^-1 of Sec. II-B, eqs. 6-9), and keep FP64, FP32 and
   FP16 copies of F and F^-1.  kappa and csw must be finite and >= 0 (WC_EINVAL).
   There is no global bound on kappa csw: each 6x6 block is inverted by
   elimination without row exchanges, whose pivots are all real and positive
   exactly when the block is positive definite, and the call returns WC_EINVAL,
   naming the number of offending blocks, when some pivot is non-positive or
   not finite (the lattice then has no clover term until a successful build).
   Synchronises the stream (the count is read back).  WC_ENOTREADY before
   wc_load_links. */
int wc_build_clover(wc_lattice *lat, double kappa, double csw);

/* Bytes of one parity of a spinor field in the internal EO layout of precision prec. */
size_t wc_spinor_bytes(const wc_lattice *lat, int prec);

/* Canonical complex128 spinor -> two-parity EO field of precision prec, and back.
   FP32 rounds every real to nearest even.  FP16 works per site in FP32: the
   scale s is the largest magnitude of the site's 24 reals, each real times
   1/s is rounded to nearest even FP16 (subnormals kept; a zero site stores
   zeros and s = 0), and unpacking returns h * s.  Both are exact functions of
   the input, so a round trip is reproducible bit for bit. */
int wc_pack_spinor(wc_lattice *lat, void *eo_out, const void *canon_in, int prec);
int wc_unpack_spinor(wc_lattice *lat, void *canon_out, const void *eo_in, int prec);

/* out = D in on the whole lattice (eq. 3); canonical complex128 in and out.  The
   operator is applied in precision prec (WC_FP64 or WC_FP32) on internal copies. */
int wc_apply_D(wc_lattice *lat, void *out_dev, const void *in_dev, int prec);

/* MULT of Sec. II-B: out_p = H-tilde_{p,1-p} in_{1-p} = F_pp^-1 H_{p,1-p} in_{1-p}
   (eq. 9).  in and out are single-parity EO fields of precision prec; out_parity
   is 0 (even, H-tilde_eo) or 1 (odd, H-tilde_oe).  WC_EINVAL for WC_FP16 on links
   that are not SU(3), as for wc_apply_Dee_oo. */
int wc_apply_mult(wc_lattice *lat, void *out, const void *in, int out_parity, int prec);

/* The even-odd preconditioned operator D-hat_ee = 1 - kappa^2 H-tilde_eo H-tilde_oe
   (eq. 8, read with H-tilde_oe as the second factor) on single-parity EO fields
   of precision prec: out_e = D-hat_ee in_e.  Uses the kappa of the built clover. */
int wc_apply_Dee_oo(wc_lattice *lat, void *out_e, const void *in_e, int prec);

/* Batched forms of wc_apply_mult and wc_apply_Dee_oo: n fields (1 <= n <= 16)
   on this lattice, out[k] = MULT in[k] (eq. 9) resp. out_e[k] = D-hat_ee in_e[k]
   (eq. 8), in one launch per MULT (many solutions per gauge field, Sec. II-A).
   With the multi-system stencil on (wc_set_multi_rhs) and prec WC_FP32 or
   WC_FP16, each thread applies one site's links and clover blocks to several
   of the fields; otherwise the fields' workgroups are interleaved.  Arguments
   as for the single forms; out, in (out_e, in_e) are host arrays of n device
   pointers.  The D-hat_ee form keeps n single-parity temporaries of the
   precision in the lattice until it is destroyed. */
int wc_apply_mult_batch(wc_lattice *lat, int n, void *const *out, const void *const *in, int out_parity, int prec);
int wc_apply_Dee_oo_batch(wc_lattice *lat, int n, void *const *out_e, const void *const *in_e, int prec);

/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): wc_apply_Dee_oo with
   the same arguments, result and errors, whose odd-parity intermediate
   F_oo^-1 H_oe in_e lives in a fixed array of wc_noalloc_scratch_bytes()
   (128 MiB) that the library holds on each GPU it runs on until the process
   ends, instead of a buffer allocated on first use.  The call allocates
   nothing.  Returns WC_EINVAL, touching nothing, when one parity of a spinor
   field in precision prec (wc_spinor_bytes) is larger than the array.  Every
   call on one GPU shares that GPU's array: calls that overlap in time on one
   GPU (other streams, other host threads) race and must be ordered by the
   caller; each call overwrites the whole part of the array it reads.
   Asynchronous on the lattice's stream.  With event timing on
   (wc_set_timing) its launches are timed like any other, with HIP events
   created for them; leave timing off (the default) where no runtime object
   may be created. */
int wc_apply_Dee_oo_noalloc(wc_lattice *lat, void *out_e, const void *in_e, int prec);
size_t wc_noalloc_scratch_bytes(void);

/* Site-diagonal clover term of parity p: out_p = F_pp in_p (inverse = 0) or
   F_pp^-1 in_p (inverse = 1), F being the site-diagonal term of eq. 3 (Sec. II-A)
   and F_ee, F_oo its even and odd blocks in the even-odd form of Sec. II-B
   (eqs. 5-9).  in and out are single-parity EO fields of precision prec
   (wc_spinor_bytes each), device memory owned by the caller; they may be the
   same buffer.  Asynchronous on the lattice's stream.  WC_EINVAL for a null
   pointer, a bad precision or parity; WC_ENOTREADY without links and clover. */
int wc_apply_clover(wc_lattice *lat, void *out, const void *in, int parity, int inverse, int prec);

/* Solve D x = b (eq. 1) for canonical complex128 b, x (device pointers) with the
   nested BiCGStab of Algorithms 1 and 2 on the even-odd system (eqs. 5-9), until
   the true relative residual ||b - D x|| / ||b|| (FP64, full lattice) is below tol.
   Rebuilds the clover when (kappa, csw) differ from the built pair.  p may be NULL
   (defaults).  x is also the initial guess when x0_is_guess != 0 (else ignored).
   info may be NULL.  Returns WC_ENOCONV with the best iterate in x when the caps
   are reached, and WC_EINVAL for an FP16 inner solve on links that are not SU(3)
   (wc_load_links). */
int wc_solve(wc_lattice *lat, const void *b_dev, double kappa, double csw, double tol,
             const wc_solve_params *p, void *x_dev, int x0_is_guess, wc_solve_info *info);

/* Batched solves (many solutions per gauge field, Sec. II-A): n systems,
   1 <= n <= 16, solved together.  Every phase of the two BiCGStab loops is one
   launch over all systems that are still iterating; each system keeps its own
   scalars, convergence flag and caps, so the results equal n separate wc_solve
   calls up to rounding.
   wc_solve_batch: n right-hand sides b_dev[k] -> x_dev[k] on one lattice (canonical
   complex128 device pointers).  Blocks of the n systems that read the same links and
   clover run back to back on one XCD, so those operands are fetched from HBM about
   once for all n.
   wc_solve_multi: system k on lattice lats[k] (lattices of different sizes allowed;
   systems on one lattice must share kappa and csw), all work on lats[0]'s stream:
   work queued earlier on the other lattices' streams is waited for (an event per
   stream), and clover rebuilds for a new (kappa, csw) also run on lats[0]'s
   stream.  The call has finished all its work when it returns.
   info (n entries) may be NULL.  Returns WC_OK when every system met tol, else the
   first failing system's status; x0 guesses are not taken. */
int wc_solve_batch(wc_lattice *lat, int n, const void *const *b_dev, void *const *x_dev, double kappa,
                   double csw, double tol, const wc_solve_params *p, wc_solve_info *info);
int wc_solve_multi(int n, wc_lattice *const *lats, const void *const *b_dev, void *const *x_dev,
                   const double *kappa, const double *csw, double tol, const wc_solve_params *p,
                   wc_solve_info *info);

/* Gradient of a real loss through a solve, with respect to the links.  With
   x = D^-1 b and lam = D^-dagger g (g = dL/dRe x + i dL/dIm x, the adjoint solve),
   dL = -Re<lam, (dD) x> for dD = dF - kappa dH (eqs. 3-4, and the clover term of
   Sec. II-A).  Writes gradU (canonical link layout, complex128, device) with
   dL = Re sum conj(gradU_ab) dU_ab over all links: the hopping outer products
   kappa [lam(n) ((1 - g_mu) x(n+mu))^dag + ((1 + g_mu) x(n)) lam(n+mu)^dag] (traced
   over spin), plus, when include_clover != 0, the clover force pushed through the
   four leaves of every plane.  lam and x are canonical complex128 spinors.  Needs
   wc_load_links; FP64 throughout.  The gradient with respect to b is lam itself. */
int wc_link_grad(wc_lattice *lat, const void *lam_dev, const void *x_dev, double kappa, double csw,
                 int include_clover, void *gradU_dev);

/* Per-kernel timing with HIP events on the lattice's stream.  While enabled, every
   launch of the hot kernels is bracketed by an event pair; wc_kernel_stats()
   synchronises and reports, for kernel slot k (0 <= k < wc_kernel_slots()), its
   name, launch count, total milliseconds and total algorithmic bytes. */
int wc_set_timing(wc_lattice *lat, int enable);
int wc_kernel_slots(void);
int wc_kernel_stats(wc_lattice *lat, int slot, const char **name, long *launches,
                    double *total_ms, double *total_bytes);
int wc_reset_kernel_stats(wc_lattice *lat);

/* Text of the last error on the calling thread ("" if none). */
const char *wc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WC_H */
