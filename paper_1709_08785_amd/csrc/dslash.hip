// The hopping stencil with spin projection and its clover epilogues (MULT of
// Sec. II-B, eq. 9, and the Schur operator D-hat_ee of eq. 8).
//
// One thread per output site of one parity.  For each of the 8 directions the
// neighbour spinor (opposite parity) is projected to a two-spin half spinor,
// multiplied by U_mu(n) (forward) or U_mu(n - mu)^dagger (backward), and
// expanded back into the accumulator (eq. 4).  In the Dirac representation:
//   (1 - g_k) psi = (h, -i s_k h),  h = psi_u + i s_k psi_d     (k = x, y, z)
//   (1 + g_k) psi = (h',  i s_k h'), h' = psi_u - i s_k psi_d
//   (1 - g_t) psi = (0, 2 psi_d),    (1 + g_t) psi = (2 psi_u, 0)
// so each direction costs two 3x3 complex matrix-vector products.
// Neighbour spinors are ordinary cached loads (each is read by 8 output sites);
// links and clover blocks are read exactly once per launch and use
// non-temporal loads so they do not evict the spinor working set.
//
// Workgroups are handed to the 8 XCDs round-robin, and each XCD has its own
// L2.  The block index is remapped so that XCD k sweeps one contiguous slab of
// the lattice: the y, z and t neighbours a block needs were then loaded by
// blocks of the same XCD shortly before, and hit in that XCD's L2.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "reduce.hpp"

namespace {

struct MultKArgs {
    Geom g;
    int out_par;
    void *out;
    const void *in;
    const void *center;
    const void *aux;
    const char *links;   // base of the 8 link slabs of this precision
    size_t link_slab;    // bytes per (mu, parity) slab
    const void *clov;    // clover slab (F or F^-1) of the output parity
    double coef;
    RedTarget red;
    const int *done;
    int nblk;            // blocks of this system
};

struct MultBatch {
    BatchHdr h;
    MultKArgs d[kMaxSys];
};

// g = U h (dag = false) or U^dagger h (dag = true), two spin components
template <class R, bool DAG>
__device__ __forceinline__ void su3_mul2(const Mat3<R> &U, const cx<R> (&h)[2][3], cx<R> (&g)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; s++) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<R> acc = {R(0), R(0)};
#pragma unroll
            for (int b = 0; b < 3; b++) {
                if (DAG)
                    cmacc(acc, U.m[3 * b + a], h[s][b]);
                else
                    cmac(acc, U.m[3 * a + b], h[s][b]);
            }
            g[s][a] = acc;
        }
    }
}

// accumulate (1 -+ g_mu) U psi for direction mu; FWD selects the forward hop.
// SC: psi holds stored values whose site scale is sc (FP16 storage); the
// scale then rides on the accumulation, where every update is an FMA anyway.
template <class R, int MU, bool FWD, bool SC>
__device__ __forceinline__ void hop_term(const Spinor<R> &p, const Mat3<R> &U, Spinor<R> &acc, R sc) {
    cx<R> h[2][3], g[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const cx<R> p0 = p.c[a], p1 = p.c[3 + a], p2 = p.c[6 + a], p3 = p.c[9 + a];
        if (MU == 0) {
            h[0][a] = FWD ? p0 + mul_i(p3) : p0 - mul_i(p3);
            h[1][a] = FWD ? p1 + mul_i(p2) : p1 - mul_i(p2);
        } else if (MU == 1) {
            h[0][a] = FWD ? p0 + p3 : p0 - p3;
            h[1][a] = FWD ? p1 - p2 : p1 + p2;
        } else if (MU == 2) {
            h[0][a] = FWD ? p0 + mul_i(p2) : p0 - mul_i(p2);
            h[1][a] = FWD ? p1 - mul_i(p3) : p1 + mul_i(p3);
        } else {
            h[0][a] = FWD ? p2 + p2 : p0 + p0;
            h[1][a] = FWD ? p3 + p3 : p1 + p1;
        }
    }
    su3_mul2<R, !FWD>(U, h, g);
    auto S = [&](cx<R> v) { return SC ? sc * v : v; };
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const cx<R> g0 = g[0][a], g1 = g[1][a];
        if (MU == 3) {
            if (FWD) {
                acc.c[6 + a] = acc.c[6 + a] + S(g0);
                acc.c[9 + a] = acc.c[9 + a] + S(g1);
            } else {
                acc.c[a] = acc.c[a] + S(g0);
                acc.c[3 + a] = acc.c[3 + a] + S(g1);
            }
            continue;
        }
        acc.c[a] = acc.c[a] + S(g0);
        acc.c[3 + a] = acc.c[3 + a] + S(g1);
        if (MU == 0) {
            acc.c[6 + a] = acc.c[6 + a] + S(FWD ? mul_mi(g1) : mul_i(g1));
            acc.c[9 + a] = acc.c[9 + a] + S(FWD ? mul_mi(g0) : mul_i(g0));
        } else if (MU == 1) {
            acc.c[6 + a] = FWD ? acc.c[6 + a] - S(g1) : acc.c[6 + a] + S(g1);
            acc.c[9 + a] = FWD ? acc.c[9 + a] + S(g0) : acc.c[9 + a] - S(g0);
        } else {
            acc.c[6 + a] = acc.c[6 + a] + S(FWD ? mul_mi(g0) : mul_i(g0));
            acc.c[9 + a] = acc.c[9 + a] + S(FWD ? mul_i(g1) : mul_mi(g1));
        }
    }
}

// one neighbour: load its spinor and add its hop; FP16 storage leaves the
// site scale to the accumulation (hop_term, SC)
template <int P, int MU, bool FWD>
__device__ __forceinline__ void hop_one(const void *in, int Vh, int n, const Mat3<typename Real<P>::T> &U,
                                        Spinor<typename Real<P>::T> &acc) {
    using R = typename Real<P>::T;
    if constexpr (P == P16) {
        float sc;
        const Spinor<R> psi = SpinorIO<P16>::load_raw(in, Vh, n, sc);
        hop_term<R, MU, FWD, true>(psi, U, acc, sc);
    } else {
        hop_term<R, MU, FWD, false>(SpinorIO<P>::load(in, Vh, n), U, acc, R(1));
    }
}

template <int P, int MU, bool NT, int LR>
__device__ __forceinline__ void hop_dir(const MultKArgs &a, const SiteCoord &c, int i,
                                        Spinor<typename Real<P>::T> &acc) {
    using R = typename Real<P>::T;
    const int Vh = a.g.Vh;
    if constexpr (P == P16) {
        // FP16 storage: every load of both hops is issued before the first
        // conversion.  Its loads are small (half the bytes of FP32), and with
        // one hop's loads in flight at a time the waves waited on latency;
        // two hops' loads in flight took the MULT from 86.6-87.9 to 83.9-84.7
        // us at 32^3x64, with results bit for bit the same.
        const int nf = eo_neighbour(a.g, c, MU, +1);
        const int nb = eo_neighbour(a.g, c, MU, -1);
        const char *lf = a.links + (size_t)(2 * MU + a.out_par) * a.link_slab;
        const char *lk = a.links + (size_t)(2 * MU + 1 - a.out_par) * a.link_slab;
        const uint4 fa = ld_op<NT>(tp<uint4, 24>(lf, i, 0));
        const uint2 fb = ld_op<NT>(tp<uint2, 24>(lf, i, 16));
        const uint4 ba = ld_op<NT>(tp<uint4, 24>(lk, nb, 0));
        const uint2 bb = ld_op<NT>(tp<uint2, 24>(lk, nb, 16));
        uint4 sf[3], sb[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            sf[k] = *tp<uint4, 52>(a.in, nf, 16 * k);
            sb[k] = *tp<uint4, 52>(a.in, nb, 16 * k);
        }
        const float scf = *tp<float, 52>(a.in, nf, 48), scb = *tp<float, 52>(a.in, nb, 48);
        hop_term<R, MU, true, true>(SpinorIO<P16>::decode(sf), LinkIO<P16>::decode(fa, fb), acc, scf);
        hop_term<R, MU, false, true>(SpinorIO<P16>::decode(sb), LinkIO<P16>::decode(ba, bb), acc, scb);
        return;
    }
    if constexpr (P == P32 && LR == 8) {
        // reconstruct-8 links: both hops' links and spinors are loaded before
        // either hop is computed, so the loads overlap the rebuild of the
        // links (MULT 144.2 -> 140.3 us, D-hat half 154.8 -> 147.3 us at
        // 32^3x64, bit for bit the same).  The two-column and full forms
        // gain nothing from it and keep the one-hop order.
        const int nf = eo_neighbour(a.g, c, MU, +1);
        const int nb = eo_neighbour(a.g, c, MU, -1);
        const Mat3<R> Uf = LinkLoad<P, LR>::template load<NT>(a.links + (size_t)(2 * MU + a.out_par) * a.link_slab, Vh, i);
        const Mat3<R> Ub =
            LinkLoad<P, LR>::template load<NT>(a.links + (size_t)(2 * MU + 1 - a.out_par) * a.link_slab, Vh, nb);
        const Spinor<R> pf = SpinorIO<P32>::load(a.in, Vh, nf);
        const Spinor<R> pb = SpinorIO<P32>::load(a.in, Vh, nb);
        hop_term<R, MU, true, false>(pf, Uf, acc, R(1));
        hop_term<R, MU, false, false>(pb, Ub, acc, R(1));
        return;
    }
    {
        const int nf = eo_neighbour(a.g, c, MU, +1);
        const Mat3<R> U = LinkLoad<P, LR>::template load<NT>(a.links + (size_t)(2 * MU + a.out_par) * a.link_slab, Vh, i);
        hop_one<P, MU, true>(a.in, Vh, nf, U, acc);
    }
    {
        const int nb = eo_neighbour(a.g, c, MU, -1);
        const Mat3<R> U =
            LinkLoad<P, LR>::template load<NT>(a.links + (size_t)(2 * MU + 1 - a.out_par) * a.link_slab, Vh, nb);
        hop_one<P, MU, false>(a.in, Vh, nb, U, acc);
    }
}

// NT: links and clover read once per launch (one system) use non-temporal
// loads; a launch that serves several systems on one lattice reads them
// through the cache so that the blocks of the other systems hit in L2.
// The one-system FP16 MULT and D-hat instances are held to four waves per
// SIMD (128 VGPRs; they use about 103 with both hops' loads in flight, hop_dir).
// Five waves at 96 VGPRs helped the form with one hop's loads in flight
// (MULT 88.2 -> 85.5 us at 32^3x64), but with two hops' loads it spills and
// runs at 100.7 us; four waves with two hops' loads run at 83.9-84.7 us.
// The reconstruct-8 FP32 instances, with both hops' loads in flight, are held
// to four waves per SIMD in the same way (118-122 VGPRs).
template <int P, int MODE, int RED, bool NT, int LR>
constexpr int stencil_waves() {
    return ((P == P16 || (P == P32 && LR == 8)) && NT && (MODE == M_HOPINV || MODE == M_DHAT)) ? 4 : 1;
}
template <int P, int MODE, int RED, bool NT, int LR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(stencil_waves<P, MODE, RED, NT, LR>())))
void k_mult(MultBatch B) {
    using R = typename Real<P>::T;
    int s, lb;
    batch_locate(B.h, xcd_block(blockIdx.x, gridDim.x, B.h.chunk), s, lb);
    const MultKArgs &a = B.d[s];
    if (a.done && *a.done) return;
    const int i = lb * (int)blockDim.x + threadIdx.x;  // 64, 128 or 256 sites per block
    const bool active = i < a.g.Vh;
    const int Vh = a.g.Vh;
    Spinor<R> out;
    // the fused reduction's operand: the centre vector itself when aux is the
    // centre (read once), else loaded after the output is stored
    Spinor<R> ax;
    if (active) {
        Spinor<R> acc;
#pragma unroll
        for (int k = 0; k < 12; k++) acc.c[k] = {R(0), R(0)};
        if (MODE != M_CLOV) {
            const SiteCoord c = eo_coords(a.g, i, a.out_par);
            hop_dir<P, 0, NT, LR>(a, c, i, acc);
            hop_dir<P, 1, NT, LR>(a, c, i, acc);
            hop_dir<P, 2, NT, LR>(a, c, i, acc);
            hop_dir<P, 3, NT, LR>(a, c, i, acc);
        }
        const R coef = (R)a.coef;
        if (MODE == M_HOPINV) {
            clover_apply<P, R, NT>(a.clov, Vh, i, acc, out);
        } else if (MODE == M_DHAT) {
            Spinor<R> t;
            clover_apply<P, R, NT>(a.clov, Vh, i, acc, t);
            const Spinor<R> cen = SpinorIO<P>::template load<true>(a.center, Vh, i);
            if (RED != R_NONE && a.aux == a.center) ax = cen;
#pragma unroll
            for (int k = 0; k < 12; k++) out.c[k] = cen.c[k] + coef * t.c[k];
        } else if (MODE == M_DFULL) {
            const Spinor<R> cen = SpinorIO<P>::template load<true>(a.center, Vh, i);
            clover_apply<P, R, NT>(a.clov, Vh, i, cen, out);
#pragma unroll
            for (int k = 0; k < 12; k++) out.c[k] = out.c[k] + coef * acc.c[k];
        } else if (MODE == M_INVSRC) {
            Spinor<R> s = SpinorIO<P>::template load<true>(a.center, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) s.c[k] = s.c[k] + coef * acc.c[k];
            clover_apply<P, R, NT>(a.clov, Vh, i, s, out);
        } else if (MODE == M_CLOV) {
            const Spinor<R> cen = SpinorIO<P>::template load<true>(a.center, Vh, i);
            clover_apply<P, R, NT>(a.clov, Vh, i, cen, out);
        } else {
            out = acc;
        }
        SpinorIO<P>::template store<P == P64>(a.out, Vh, i, out);
    }
    if (RED != R_NONE) {
        constexpr int N = (RED == R_DOT) ? 2 : 3;
        double v[N];
#pragma unroll
        for (int k = 0; k < N; k++) v[k] = 0.0;
        if (active) {
            if (!(MODE == M_DHAT && a.aux == a.center)) ax = SpinorIO<P>::template load<true>(a.aux, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const double ar = ax.c[k].re, ai = ax.c[k].im, orr = out.c[k].re, oi = out.c[k].im;
                v[0] += ar * orr + ai * oi;
                v[1] += ar * oi - ai * orr;
                if (N == 3) v[N - 1] += orr * orr + oi * oi;
            }
        }
        block_partials<N>(v, a.red.partials, a.nblk, lb);
    }
}

// lds: dynamic LDS bytes that cap the workgroups per CU of the one-system
// (non-temporal) instance; the kernels use none of it
template <int P, int MODE, int RED, int LR>
void launch_nt(const MultBatch &B, int blocks, int bs, unsigned lds, hipStream_t s) {
    if (B.h.interleave)
        hipLaunchKernelGGL((k_mult<P, MODE, RED, false, LR>), dim3(blocks), dim3(bs), 0, s, B);
    else
        hipLaunchKernelGGL((k_mult<P, MODE, RED, true, LR>), dim3(blocks), dim3(bs), lds, s, B);
}

// reconstruct-8 and full-link instances exist for the FP32 stencil only
template <int P, int MODE, int RED>
void launch_one(const MultBatch &B, int blocks, int bs, unsigned lds, hipStream_t s, int lr) {
    if constexpr (P == P32) {
        if (lr == 8) {
            launch_nt<P, MODE, RED, 8>(B, blocks, bs, lds, s);
            return;
        }
        if (lr == 18) {
            launch_nt<P, MODE, RED, 18>(B, blocks, bs, lds, s);
            return;
        }
    }
    launch_nt<P, MODE, RED, 12>(B, blocks, bs, lds, s);
}

template <int P>
void dispatch_mode(const MultBatch &B, int mode, int red, int blocks, int bs, unsigned lds, hipStream_t s, int lr) {
    switch (mode) {
    case M_HOPINV: launch_one<P, M_HOPINV, R_NONE>(B, blocks, bs, lds, s, lr); break;
    case M_DHAT:
        if (red == R_DOT) launch_one<P, M_DHAT, R_DOT>(B, blocks, bs, lds, s, lr);
        else if (red == R_DOTNORM) launch_one<P, M_DHAT, R_DOTNORM>(B, blocks, bs, lds, s, lr);
        else launch_one<P, M_DHAT, R_NONE>(B, blocks, bs, lds, s, lr);
        break;
    case M_DFULL: launch_one<P, M_DFULL, R_NONE>(B, blocks, bs, lds, s, lr); break;
    case M_INVSRC: launch_one<P, M_INVSRC, R_NONE>(B, blocks, bs, lds, s, lr); break;
    case M_HOP: launch_one<P, M_HOP, R_NONE>(B, blocks, bs, lds, s, lr); break;
    case M_CLOV: launch_one<P, M_CLOV, R_NONE>(B, blocks, bs, lds, s, lr); break;
    }
}

// algorithmic bytes of one call (per output site: inputs and outputs at the
// stored precision, each link once, one clover pair).  The spinor part is per
// call; the link and clover part is per lattice, since calls of one batch on
// the same lattice read the same operator.
double mult_spinor_bytes(int prec, int mode, int red, bool aux_is_centre, int Vh) {
    const double S = (double)spinor_site_bytes(prec) * Vh;
    double b = 2 * S;                                                    // input (once) + output
    if (mode == M_DHAT || mode == M_DFULL || mode == M_INVSRC) b += S;  // centre vector
    if (red != R_NONE && !aux_is_centre) b += S;                         // aux vector, unless the centre
    return b;
}
double mult_operator_bytes(int prec, int mode, int lr, int Vh) {
    double b = 0;
    const int lb = lr == 8 ? 32 : lr == 18 ? 72 : link_site_bytes(prec);
    if (mode != M_CLOV) b += 8 * (double)lb * Vh;
    if (mode != M_HOP) b += (double)clover_site_bytes(prec) * Vh;
    return b;
}


// ---------------------------------------------------------------------------
// Several right-hand sides on one lattice (many solutions per gauge field,
// Sec. II-A): one thread takes one output site for G systems at once.  The
// neighbour indices, each link (with its third column rebuilt) and each
// clover block are computed or loaded once and applied to all G spinors, so
// the per-site work that does not depend on the source is shared, and the
// operator is read from memory once per site for every system of the launch.
// A wavefront covers the 64 sites of one tile for one group of G systems, and
// the waves of all groups of a tile form one workgroup (so they run on one
// compute unit), so their link and clover loads after the first hit in cache.
// Reductions are per wave: each wave folds its G systems' sums and writes one
// partial per system and tile, which the finalize stage sums in tile order.
// ---------------------------------------------------------------------------
struct MrhsSys {
    void *out;
    const void *in;
    const void *center;
    const void *aux;
    double *partials;  // [N][ntiles] of this system
    const int *done;
};

struct MrhsArgs {
    Geom g;
    int out_par;
    const char *links;
    size_t link_slab;
    const void *clov;
    double coef;
    int nsys;     // systems of the launch
    int ngroups;  // groups of G systems: ceil(nsys / G)
    int ntiles;   // 64-site tiles of one parity
    int chunk;    // tiles per XCD chunk of the block remap (0: one slab per XCD)
    MrhsSys s[kMaxSys];
};

// one stored 6x6 block; FP16 blocks without their site scale
template <int P>
__device__ __forceinline__ Herm6<typename Real<P>::T> clover_block(const void *slab, int Vh, int i, int b) {
    if constexpr (P == P16) return CloverIO<P16>::template load_scaled<false>(slab, Vh, i, b, 1.0f);
    else return CloverIO<P>::template load<false>(slab, Vh, i, b);
}

// out_j = M_blk(w_j) applied blockwise as in clover_apply, for G spinors, each
// 6x6 block loaded once: on entry acc[j] holds the hopping sum, on exit the
// clover result
template <int P, int G, class R>
__device__ __forceinline__ void clover_apply_multi(const void *slab, int Vh, int i, Spinor<R> (&acc)[G],
                                                   const bool (&live)[G]) {
    // acc.up <- wp = up + dn, acc.dn <- M1 (up - dn)
    {
        const Herm6<R> M1 = clover_block<P>(slab, Vh, i, 0);
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (!live[j]) continue;
            cx<R> wm[6], ym[6];
#pragma unroll
            for (int k = 0; k < 6; k++) {
                wm[k] = acc[j].c[k] - acc[j].c[k + 6];
                acc[j].c[k] = acc[j].c[k] + acc[j].c[k + 6];
            }
            herm6_apply(M1, wm, ym);
#pragma unroll
            for (int k = 0; k < 6; k++) acc[j].c[k + 6] = ym[k];
        }
    }
    const Herm6<R> M2 = clover_block<P>(slab, Vh, i, 1);
    R s = R(1);
    if constexpr (P == P16) s = CloverIO<P16>::scale(slab, i);
#pragma unroll
    for (int j = 0; j < G; j++) {
        if (!live[j]) continue;
        cx<R> yp[6];
        herm6_apply(M2, acc[j].c, yp);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const cx<R> ym = acc[j].c[k + 6];
            acc[j].c[k] = s * (yp[k] + ym);
            acc[j].c[k + 6] = s * (yp[k] - ym);
        }
    }
}

template <int P, int MU, int LR, int G>
__device__ __forceinline__ void hop_dir_multi(const MrhsArgs &A, const SiteCoord &c, int i, int q,
                                              Spinor<typename Real<P>::T> (&acc)[G], const bool (&live)[G]) {
    using R = typename Real<P>::T;
    const int Vh = A.g.Vh;
    {
        const int nf = eo_neighbour(A.g, c, MU, +1);
        const Mat3<R> U = LinkLoad<P, LR>::template load<false>(A.links + (size_t)(2 * MU + A.out_par) * A.link_slab, Vh, i);
#pragma unroll
        for (int j = 0; j < G; j++)
            if (live[j]) hop_one<P, MU, true>(A.s[q * G + j].in, Vh, nf, U, acc[j]);
    }
    {
        const int nb = eo_neighbour(A.g, c, MU, -1);
        const Mat3<R> U =
            LinkLoad<P, LR>::template load<false>(A.links + (size_t)(2 * MU + 1 - A.out_par) * A.link_slab, Vh, nb);
#pragma unroll
        for (int j = 0; j < G; j++)
            if (live[j]) hop_one<P, MU, false>(A.s[q * G + j].in, Vh, nb, U, acc[j]);
    }
}

// One workgroup per 64-site tile, one wavefront per group of G systems, so the
// waves that share a tile's links and clover blocks run on one compute unit;
// the tiles are handed to the XCDs in the lattice's chunks, as for the
// one-system stencil.
constexpr int kMrhsMaxGroups = 8;  // 16 systems at 2 per thread
template <int P, int MODE, int RED, int LR, int G>
__global__ __launch_bounds__(64 * kMrhsMaxGroups) void k_mult_mrhs(MrhsArgs A) {
    using R = typename Real<P>::T;
    const int tile = xcd_block(blockIdx.x, gridDim.x, A.chunk);
    const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform across the wave
    if (tile >= A.ntiles || q >= A.ngroups) return;  // whole waves only
    bool live[G];
    bool any = false;
#pragma unroll
    for (int j = 0; j < G; j++) {
        const int s = q * G + j;
        live[j] = s < A.nsys && !(A.s[s].done && *A.s[s].done);
        any = any || live[j];
    }
    if (!any) return;  // every system of this wave has stopped
    const int Vh = A.g.Vh;
    const int i = tile * 64 + (int)(threadIdx.x & 63);
    const bool active = i < Vh;
    constexpr int NR = (RED == R_DOTNORM) ? 3 : 2;  // values of the fused reduction
    double red[G][NR];
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int k = 0; k < NR; k++) red[j][k] = 0.0;
    Spinor<R> acc[G];
#pragma unroll
    for (int j = 0; j < G; j++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[j].c[k] = {R(0), R(0)};
    if (active) {
        const SiteCoord c = eo_coords(A.g, i, A.out_par);
        hop_dir_multi<P, 0, LR, G>(A, c, i, q, acc, live);
        hop_dir_multi<P, 1, LR, G>(A, c, i, q, acc, live);
        hop_dir_multi<P, 2, LR, G>(A, c, i, q, acc, live);
        hop_dir_multi<P, 3, LR, G>(A, c, i, q, acc, live);
        clover_apply_multi<P, G>(A.clov, Vh, i, acc, live);
        const R coef = (R)A.coef;
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (!live[j]) continue;
            const MrhsSys &S = A.s[q * G + j];
            if (MODE == M_DHAT) {
                // the centre, and the reduction's operand beside it (the centre
                // itself when aux is the centre)
                const Spinor<R> cen = SpinorIO<P>::template load<true>(S.center, Vh, i);
                Spinor<R> ax;
                if (RED != R_NONE) ax = (S.aux == S.center) ? cen : SpinorIO<P>::template load<true>(S.aux, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) acc[j].c[k] = cen.c[k] + coef * acc[j].c[k];
                SpinorIO<P>::template store<false>(S.out, Vh, i, acc[j]);
                if (RED != R_NONE) {
#pragma unroll
                    for (int k = 0; k < 12; k++) {
                        const double ar = ax.c[k].re, ai = ax.c[k].im, orr = acc[j].c[k].re, oi = acc[j].c[k].im;
                        red[j][0] += ar * orr + ai * oi;
                        red[j][1] += ar * oi - ai * orr;
                        if (NR == 3) red[j][NR - 1] += orr * orr + oi * oi;
                    }
                }
            } else {
                SpinorIO<P>::template store<false>(S.out, Vh, i, acc[j]);
            }
        }
    }
    if (RED != R_NONE) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (!live[j]) continue;
            wave_fold<NR>(red[j]);
            if ((threadIdx.x & 63) == 0) {
                double *part = A.s[q * G + j].partials;
#pragma unroll
                for (int k = 0; k < NR; k++) part[(size_t)k * A.ntiles + tile] = red[j][k];
            }
        }
    }
}

template <int P, int MODE, int RED, int LR, int G>
void launch_mrhs_g(const MrhsArgs &A, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_mult_mrhs<P, MODE, RED, LR, G>), dim3(blocks), dim3(64 * A.ngroups), 0, s, A);
}

template <int P, int MODE, int RED, int LR> void launch_mrhs_lr(const MrhsArgs &A, int blocks, hipStream_t s, int G) {
    if (G == 2) launch_mrhs_g<P, MODE, RED, LR, 2>(A, blocks, s);
    else launch_mrhs_g<P, MODE, RED, LR, 4>(A, blocks, s);
}

template <int P, int MODE, int RED> void launch_mrhs_mode(const MrhsArgs &A, int blocks, hipStream_t s, int lr, int G) {
    if constexpr (P == P32) {
        if (lr == 8) return launch_mrhs_lr<P, MODE, RED, 8>(A, blocks, s, G);
        if (lr == 18) return launch_mrhs_lr<P, MODE, RED, 18>(A, blocks, s, G);
    }
    launch_mrhs_lr<P, MODE, RED, 12>(A, blocks, s, G);
}

template <int P> void dispatch_mrhs(const MrhsArgs &A, int mode, int red, int blocks, hipStream_t s, int lr, int G) {
    if (mode == M_HOPINV) launch_mrhs_mode<P, M_HOPINV, R_NONE>(A, blocks, s, lr, G);
    else if (red == R_DOT) launch_mrhs_mode<P, M_DHAT, R_DOT>(A, blocks, s, lr, G);
    else if (red == R_DOTNORM) launch_mrhs_mode<P, M_DHAT, R_DOTNORM>(A, blocks, s, lr, G);
    else launch_mrhs_mode<P, M_DHAT, R_NONE>(A, blocks, s, lr, G);
}

// ---------------------------------------------------------------------------
// The whole inner loop (Algorithm 2) in one cooperative launch, for lattices
// small enough that every workgroup is resident at once.  Each phase of an
// iteration ends in a grid-wide barrier instead of a kernel boundary; every
// block then sums the reduction partials itself, in the same order as the
// finalize kernel of the launched path, so all blocks take the same
// decisions and leave the loop together.  The per-site arithmetic is that of
// the stencil and vector kernels, and the scalars and flags are left exactly
// as the launched path leaves them, so the host finishes the call the same
// way.  Partials alternate between two buffers: a buffer is written again
// only after a barrier that follows its last read.
// ---------------------------------------------------------------------------
struct PersistArgs {
    Geom g;
    const char *links;
    size_t link_slab;
    const void *clov_e, *clov_o;  // F_ee^-1, F_oo^-1
    void *r, *rt, *p, *q, *t, *tmp, *x;
    double *part[2];              // [kMaxRed][nblk] each
    double *sc;
    int *fl;
    double kappa2;
    int maxit;
    int nblk;
    unsigned long long *bar;  // the kernel's own barrier words (OWN instances)
    unsigned long long tag0;  // call number << 32; barrier k of the call has tag tag0 + k
    unsigned long long epoch; // written to the abort word when a wait runs out
    long long limit;          // wall-clock ticks a wait may take
};

__device__ __forceinline__ int rho_slot_p(int iter) { return (iter & 1) ? S_RHO1 : S_RHO0; }

// from this many blocks up the kernel's own barrier beats the runtime's
constexpr int kOwnBarrierMinBlocks = 16;

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier of the one-launch loop.  The runtime's barrier fences
// every wave of every block, which costs about 0.13 us per block; here every
// wave only waits for its own stores to reach L2, and one wave per block
// writes the L2 back (release) and, on the way out, invalidates the caches
// (acquire) before its block reads again.  Each block posts its arrival in a
// word of its own (no contended atomics); one wave of block 0 gathers them
// and posts the release.  Tags grow from barrier to barrier and from call to
// call (the host clears the words when its call counter wraps).  Every
// wait is bounded in wall-clock time: a wait that runs out posts the abort
// word, every other waiter sees it, and the function returns false in every
// block, so the kernel always ends.
template <bool OWN> __device__ __forceinline__ bool grid_barrier(const PersistArgs &A, unsigned long long &tag, int lb) {
    __shared__ int ok;
    ++tag;
    if constexpr (!OWN) {
        cooperative_groups::this_grid().sync();
        return true;
    }
    unsigned long long *w = A.bar;
    unsigned long long *rel = w + A.nblk, *abort = w + A.nblk + 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        st_agent(&w[lb], tag);
    }
    const long long t0 = wall_clock64();
    if (lb == 0 && threadIdx.x < 64) {
        int all = 0;
        for (;;) {
            int mine = 1;
            for (int j = threadIdx.x; j < A.nblk; j += 64) mine &= ld_agent(&w[j]) >= tag;
            all = __all(mine);
            if (all || ld_agent(abort) == A.epoch || wall_clock64() - t0 > A.limit) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (threadIdx.x == 0) {
            __threadfence();
            if (all) st_agent(rel, tag);
            else st_agent(abort, A.epoch);
        }
    }
    if (threadIdx.x == 0) {
        int good = 1;
        while (ld_agent(rel) < tag) {
            if (ld_agent(abort) == A.epoch || wall_clock64() - t0 > A.limit) {
                st_agent(abort, A.epoch);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        ok = good;
    }
    __syncthreads();
    return ok;
}

// a value every lane holds alike, read from lane 0 so the compiler knows it
// is uniform (branches on it stay scalar, pointers chosen by it stay in SGPRs)
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// every block: the N sums of the partials, in the finalize kernel's order
template <int N> __device__ __forceinline__ void sum_partials(const double *part, int nblk, double (&out)[N]) {
    __shared__ double sh[N][kWaves];
    __shared__ double tot[N];
    double a[N];
#pragma unroll
    for (int k = 0; k < N; k++) a[k] = 0.0;
    for (int j = threadIdx.x; j < nblk; j += kBlock) {
#pragma unroll
        for (int k = 0; k < N; k++) a[k] += part[(size_t)k * nblk + j];
    }
    block_fold<N>(a, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) tot[k] = a[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) out[k] = uniform(tot[k]);
    __syncthreads();
}

// out = F^-1 H in (one parity), the MULT of the launched path
template <int P, int LR>
__device__ __forceinline__ Spinor<typename Real<P>::T> mult_site(const PersistArgs &A, const void *in, int out_par,
                                                                     const void *clov, int i) {
    using R = typename Real<P>::T;
    MultKArgs a;
    a.g = A.g;
    a.out_par = out_par;
    a.in = in;
    a.links = A.links;
    a.link_slab = A.link_slab;
    Spinor<R> acc, out;
#pragma unroll
    for (int k = 0; k < 12; k++) acc.c[k] = {R(0), R(0)};
    const SiteCoord c = eo_coords(A.g, i, out_par);
    hop_dir<P, 0, false, LR>(a, c, i, acc);
    hop_dir<P, 1, false, LR>(a, c, i, acc);
    hop_dir<P, 2, false, LR>(a, c, i, acc);
    hop_dir<P, 3, false, LR>(a, c, i, acc);
    clover_apply<P, R, false>(clov, A.g.Vh, i, acc, out);
    return out;
}

template <class R> __device__ __forceinline__ cx<R> to_r(cx<double> a) { return {(R)a.re, (R)a.im}; }

// The loop runs as four stages per iteration, each opening with the one
// stencil instance of the kernel:
//   0: tmp = F_oo^-1 H_oe p               2: tmp = F_oo^-1 H_oe s
//   1: q = p - kappa^2 F_ee^-1 H_eo tmp   3: t = s - kappa^2 F_ee^-1 H_eo tmp
// followed by the vector updates and reductions of that half-iteration.  A
// single instance keeps the register allocation that of one stencil launch;
// the scalars every thread needs (rho, alpha) stay in registers, the ones
// only the final write-out needs sit in LDS.
template <int P, int LR, bool OWN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(P == P64 ? 1 : 2))) void k_inner_persistent(PersistArgs A) {
    using R = typename Real<P>::T;
    constexpr int XP = P == P64 ? P64 : P32;
    using RX = typename Real<XP>::T;
    enum { K_RQ = 0, K_SS = 2, K_ST = 3, K_TT = 5, K_RR = 6, K_N = 7 };
    __shared__ double kept[K_N];  // last values, for the write-out by block 0
    const int Vh = A.g.Vh;
    const int lb = xcd_block(blockIdx.x, gridDim.x);  // neighbouring sites share an XCD's L2
    const int i = lb * kBlock + threadIdx.x;
    const bool active = i < Vh;
    const double tol2 = A.sc[S_TOL2];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K_N; k++) kept[k] = 0.0;
    }
    cx<double> rho = ld_c(A.sc, S_RHO0), al = {0.0, 0.0};
    int it = 0, stage = 0, done = DONE_NO, stopph = 0;
    unsigned long long tag = A.tag0;
    bool timed_out = false;
    while (it < A.maxit) {
        const bool mult = !(stage & 1);
        const bool second = stage >= 2;
        const void *v = second ? A.r : A.p;  // p, or s (held in r)
        Spinor<R> h;
        if (active) h = mult_site<P, LR>(A, mult ? v : A.tmp, mult ? 1 : 0, mult ? A.clov_o : A.clov_e, i);
        if (mult) {
            if (active) SpinorIO<P>::store(A.tmp, Vh, i, h);
            if (!grid_barrier<OWN>(A, tag, lb)) {
                timed_out = true;
                break;
            }
            stage++;
            continue;
        }
        // D-hat v = v - kappa^2 h into q or t, with <r~, q> or <s, t>, ||t||^2
        Spinor<R> out;
        {
            double d[3] = {0.0, 0.0, 0.0};
            if (active) {
                const Spinor<R> cen = SpinorIO<P>::load(v, Vh, i);
                const R coef = (R)(-A.kappa2);
#pragma unroll
                for (int k = 0; k < 12; k++) out.c[k] = cen.c[k] + coef * h.c[k];
                SpinorIO<P>::store(second ? A.t : A.q, Vh, i, out);
                const Spinor<R> ax = second ? cen : SpinorIO<P>::load(A.rt, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    const double ar = ax.c[k].re, ai = ax.c[k].im, orr = out.c[k].re, oi = out.c[k].im;
                    d[0] += ar * orr + ai * oi;
                    d[1] += ar * oi - ai * orr;
                    d[2] += orr * orr + oi * oi;
                }
            }
            if (second) {
                block_partials<3>(d, A.part[0], A.nblk, lb);
            } else {
                double d2[2] = {d[0], d[1]};
                block_partials<2>(d2, A.part[0], A.nblk, lb);
            }
            // the updates below use q or t as stored (FP16 storage rounds)
            if constexpr (P == P16) {
                if (active) out = SpinorIO<P>::load(second ? A.t : A.q, Vh, i);
            }
        }
        if (!grid_barrier<OWN>(A, tag, lb)) {
            timed_out = true;
            break;
        }
        if (!second) {
            double sm[2];
            sum_partials<2>(A.part[0], A.nblk, sm);
            const cx<double> rq = {sm[0], sm[1]};
            al = cdiv(rho, rq);
            // s = r - alpha q (in r) with ||s||^2; the half-step check
            double n[1] = {0.0};
            if (active) {
                const cx<R> alpha = to_r<R>(al);
                Spinor<R> rv = SpinorIO<P>::load(A.r, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) rv.c[k] = rv.c[k] - alpha * out.c[k];
                SpinorIO<P>::store(A.r, Vh, i, rv);
#pragma unroll
                for (int k = 0; k < 12; k++) n[0] += norm2(rv.c[k]);
            }
            block_partials<1>(n, A.part[1], A.nblk, lb);
            if (!grid_barrier<OWN>(A, tag, lb)) {
                timed_out = true;
                break;
            }
            sum_partials<1>(A.part[1], A.nblk, n);
            if (threadIdx.x == 0) {
                kept[K_RQ] = rq.re;
                kept[K_RQ + 1] = rq.im;
                kept[K_SS] = n[0];
            }
            if (!(isfinite(al.re) && isfinite(al.im)) || !isfinite(n[0])) {
                done = DONE_BREAK;
                stopph = 1;
                break;
            }
            if (n[0] < tol2) {
                done = DONE_HALF;
                stopph = 1;
                break;
            }
            stage = 2;
            continue;
        }
        double sm[3];
        sum_partials<3>(A.part[0], A.nblk, sm);
        const cx<double> st = {sm[0], sm[1]};
        const double tt = sm[2];
        // x += alpha p + omega s; r = s - omega t with ||r||^2, <r~, r>
        const cx<double> om = {st.re / tt, -st.im / tt};
        double v3[3] = {0.0, 0.0, 0.0};
        if (active) {
            const cx<RX> alx = to_r<RX>(al), omx = to_r<RX>(om);
            const cx<R> omega = to_r<R>(om);
            Spinor<R> sv = SpinorIO<P>::load(A.r, Vh, i);
            const Spinor<R> pv = SpinorIO<P>::load(A.p, Vh, i);
            Spinor<RX> xv = SpinorIO<XP>::load(A.x, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<RX> pk = {(RX)pv.c[k].re, (RX)pv.c[k].im}, sk = {(RX)sv.c[k].re, (RX)sv.c[k].im};
                xv.c[k] = xv.c[k] + alx * pk + omx * sk;
            }
            SpinorIO<XP>::store(A.x, Vh, i, xv);
#pragma unroll
            for (int k = 0; k < 12; k++) sv.c[k] = sv.c[k] - omega * out.c[k];
            SpinorIO<P>::store(A.r, Vh, i, sv);
            const Spinor<R> rtv = SpinorIO<P>::load(A.rt, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v3[0] += norm2(sv.c[k]);
                const double ar = rtv.c[k].re, ai = rtv.c[k].im, br = sv.c[k].re, bi = sv.c[k].im;
                v3[1] += ar * br + ai * bi;
                v3[2] += ar * bi - ai * br;
            }
        }
        block_partials<3>(v3, A.part[1], A.nblk, lb);
        if (!grid_barrier<OWN>(A, tag, lb)) {
            timed_out = true;
            break;
        }
        sum_partials<3>(A.part[1], A.nblk, v3);
        const double rr = v3[0];
        const cx<double> rho1 = {v3[1], v3[2]};
        if (threadIdx.x == 0) {
            kept[K_ST] = st.re;
            kept[K_ST + 1] = st.im;
            kept[K_TT] = tt;
            kept[K_RR] = rr;
        }
        const bool bad = !(tt > 0.0) || !(isfinite(om.re) && isfinite(om.im)) || !isfinite(rr) ||
                         (rho1.re == 0.0 && rho1.im == 0.0);
        if (bad || rr < tol2) {
            done = (rr < tol2) ? DONE_FULL : DONE_BREAK;
            stopph = 2;
            // the scalars of a full step, as the launched path leaves them
            if (lb == 0 && threadIdx.x == 0) {
                const int nxt = rho_slot_p(it + 1);
                A.sc[nxt] = rho1.re;
                A.sc[nxt + 1] = rho1.im;
            }
            it++;
            break;
        }
        // p = r + beta (p - omega q)
        if (active) {
            const cx<R> beta = to_r<R>(cdiv(rho1, rho) * cdiv(al, om)), omega = to_r<R>(om);
            Spinor<R> pv = SpinorIO<P>::load(A.p, Vh, i);
            const Spinor<R> rv = SpinorIO<P>::load(A.r, Vh, i);
            const Spinor<R> qv = SpinorIO<P>::load(A.q, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) pv.c[k] = rv.c[k] + beta * (pv.c[k] - omega * qv.c[k]);
            SpinorIO<P>::store(A.p, Vh, i, pv);
        }
        rho = rho1;
        if (!grid_barrier<OWN>(A, tag, lb)) {
            timed_out = true;
            break;
        }
        stage = 0;
        it++;
    }
    if (timed_out) {
        done = DONE_BREAK;
        stopph = 3;
    }
    // leave the scalars and flags as the launched path would
    if (lb == 0 && threadIdx.x == 0) {
        double *sc = A.sc;
        if (stopph != 2) {
            const int cur = rho_slot_p(it);
            sc[cur] = rho.re;
            sc[cur + 1] = rho.im;
        }
        sc[S_RQ] = kept[K_RQ];
        sc[S_RQ + 1] = kept[K_RQ + 1];
        sc[S_SS] = kept[K_SS];
        sc[S_ST] = kept[K_ST];
        sc[S_ST + 1] = kept[K_ST + 1];
        sc[S_TT] = kept[K_TT];
        sc[S_RR] = kept[K_RR];
        A.fl[F_DONE] = done;
        A.fl[F_ITERS] = it;
        A.fl[F_STOPPH] = stopph;
    }
}

}  // namespace

// Several calls on one lattice through the multi-system stencil: G systems per
// thread, the operator loaded once per site for all of them.
static int launch_mult_mrhs(hipStream_t s, const MultCall *calls, int n, wc_lattice *tl, int G) {
    const MultCall &c0 = calls[0];
    wc_lattice *lat = c0.lat;
    const int lr = c0.prec == P32 ? lat->recon : 12;
    MrhsArgs A;
    A.g = lat->g;
    A.out_par = c0.out_par;
    A.links = (const char *)link_base(lat, c0.prec);
    A.link_slab = link_slab_for(lat, c0.prec);
    A.clov = (const char *)lat->clovinv[c0.prec] + (size_t)c0.out_par * clover_slab_bytes(c0.prec, lat->Vh);
    A.coef = c0.coef;
    A.nsys = n;
    A.ngroups = (n + G - 1) / G;
    A.ntiles = blocks_of(lat->Vh, 64);
    A.chunk = lattice_chunk(lat, c0.prec);
    double bytes = mult_operator_bytes(c0.prec, c0.mode, lr, lat->Vh);
    for (int k = 0; k < n; k++) {
        const MultCall &c = calls[k];
        if (c.coef != c0.coef) return wc_fail(WC_EINVAL, "multi-system stencil calls must share the coefficient");
        A.s[k] = MrhsSys{c.out, c.in, c.center, c.aux, c.red_to.partials, c.done};
        bytes += mult_spinor_bytes(c.prec, c.mode, c.red, c.aux == c.center, lat->Vh);
        lat->dslash_count++;
    }
    if (A.ngroups > kMrhsMaxGroups) return wc_fail(WC_EINVAL, "too many systems per multi-system launch");
    const int blocks = A.ntiles;
    int slot = c0.mode == M_HOPINV ? KS_MULT_HOPINV_P64 + c0.prec : KS_MULT_DHAT_P64 + c0.prec;
    TimedLaunch t;
    if (tl->timing) {
        timing_begin(tl, slot, bytes, t);
        t.iter = tl->tag_iter;
        t.phase = tl->tag_phase;
        TimedPart op{{}, mult_operator_bytes(c0.prec, c0.mode, lr, lat->Vh)};
        for (int k = 0; k < n; k++) {
            const MultCall &c = calls[k];
            t.parts.push_back(TimedPart{{c.done}, mult_spinor_bytes(c.prec, c.mode, c.red, c.aux == c.center,
                                                                      lat->Vh)});
            op.owners.push_back(c.done);
        }
        t.parts.push_back(op);
    }
    if (c0.prec == P32) dispatch_mrhs<P32>(A, c0.mode, c0.red, blocks, s, lr, G);
    else dispatch_mrhs<P16>(A, c0.mode, c0.red, blocks, s, 12, G);
    WC_HIP(hipGetLastError());
    if (tl->timing) timing_end(tl, t);
    if (c0.red != R_NONE) {
        FinArgs f[kMaxSys];
        for (int k = 0; k < n; k++) {
            f[k] = FinArgs{};
            f[k].blocks = A.ntiles;  // one partial per 64-site tile
            f[k].op = FIN_STORE;
            f[k].partials = calls[k].red_to.partials;
            f[k].result = calls[k].red_to.result;
            f[k].guard = calls[k].done;
        }
        return launch_fin_batch(s, f, n, c0.red == R_DOT ? 2 : 3);
    }
    return WC_OK;
}

int launch_mult_batch(hipStream_t s, const MultCall *calls, int n, wc_lattice *timing_lat) {
    if (n <= 0) return WC_OK;
    if (n > kMaxSys) return wc_fail(WC_EINVAL, "too many systems in one batch");
    const MultCall &c0 = calls[0];
    {
        // several systems on one lattice in an inner-precision stencil: the
        // multi-system form, when the lattice has it switched on
        bool same = n > 1 && mrhs_for(c0.lat, c0.prec) > 0 && (c0.prec == P32 || c0.prec == P16) &&
                    (c0.mode == M_HOPINV || c0.mode == M_DHAT);
        for (int k = 1; same && k < n; k++)
            same = calls[k].lat == c0.lat && calls[k].prec == c0.prec && calls[k].mode == c0.mode &&
                   calls[k].red == c0.red && calls[k].out_par == c0.out_par && calls[k].coef == c0.coef;
        if (same) return launch_mult_mrhs(s, calls, n, timing_lat ? timing_lat : c0.lat, mrhs_for(c0.lat, c0.prec));
    }
    const int bs = launch_bs(c0.bs);
    if (!valid_block_size(bs)) return wc_fail(WC_EINVAL, "block size must be 64, 128 or 256");
    MultBatch B;
    B.h.S = n;
    B.h.off[0] = 0;
    bool same = true;
    double bytes = 0;
    const int lr = c0.prec == P32 ? c0.lat->recon : 12;  // link form of the FP32 stencil
    for (int k = 0; k < n; k++) {
        const MultCall &c = calls[k];
        wc_lattice *lat = c.lat;
        if (c.prec != c0.prec || c.mode != c0.mode || c.red != c0.red || c.out_par != c0.out_par)
            return wc_fail(WC_EINVAL, "batched stencil calls must share precision, mode, reduction and parity");
        if (launch_bs(c.bs) != bs) return wc_fail(WC_EINVAL, "batched stencil calls must share the block size");
        same = same && (lat == c0.lat);
        MultKArgs &a = B.d[k];
        a.g = lat->g;
        a.out_par = c.out_par;
        a.out = c.out;
        a.in = c.in;
        a.center = c.center;
        a.aux = c.aux;
        if ((c.prec == P32 ? lat->recon : 12) != lr)
            return wc_fail(WC_EINVAL, "batched stencil calls must share the link reconstruction");
        a.links = (const char *)link_base(lat, c.prec);
        a.link_slab = link_slab_for(lat, c.prec);
        const bool use_inv = (c.mode == M_HOPINV || c.mode == M_DHAT || c.mode == M_INVSRC ||
                              (c.mode == M_CLOV && c.inverse));
        const char *cb = (const char *)(use_inv ? lat->clovinv[c.prec] : lat->clov[c.prec]);
        a.clov = cb + (size_t)c.out_par * clover_slab_bytes(c.prec, lat->Vh);
        a.coef = c.coef;
        a.red = c.red_to;
        a.done = c.done;
        a.nblk = blocks_of(lat->Vh, bs);
        B.h.off[k + 1] = B.h.off[k] + a.nblk;
        bytes += mult_spinor_bytes(c.prec, c.mode, c.red, c.aux == c.center, lat->Vh);
        bool seen = false;
        for (int j = 0; j < k; j++) seen = seen || (calls[j].lat == lat);
        if (!seen) bytes += mult_operator_bytes(c.prec, c.mode, lr, lat->Vh);
        if (c.mode != M_CLOV) lat->dslash_count++;
    }
    B.h.interleave = (same && n > 1) ? 1 : 0;
    // the lattice's chunk of sites per XCD, in blocks of this launch (with the
    // systems of one lattice interleaved block by block, every system's blocks)
    {
        const int tiles = lattice_chunk(c0.lat, c0.prec);
        B.h.chunk = tiles <= 0 ? 0 : std::max(1, tiles / (bs / 64)) * (B.h.interleave ? n : 1);
    }
    const int blocks = B.h.off[n];
    wc_lattice *tl = timing_lat ? timing_lat : c0.lat;
    int slot = KS_MULT_OTHER;
    if (c0.mode == M_HOPINV) slot = KS_MULT_HOPINV_P64 + c0.prec;
    if (c0.mode == M_DHAT) slot = KS_MULT_DHAT_P64 + c0.prec;
    TimedLaunch t;
    if (tl->timing) {
        timing_begin(tl, slot, bytes, t);
        // split by system, and the operator by the systems that share it
        t.iter = tl->tag_iter;
        t.phase = tl->tag_phase;
        for (int k = 0; k < n; k++) {
            const MultCall &c = calls[k];
            t.parts.push_back(TimedPart{{c.done}, mult_spinor_bytes(c.prec, c.mode, c.red, c.aux == c.center,
                                                                      c.lat->Vh)});
            bool seen = false;
            for (int j = 0; j < k; j++) seen = seen || (calls[j].lat == c.lat);
            if (seen) continue;
            TimedPart op{{}, mult_operator_bytes(c.prec, c.mode, lr, c.lat->Vh)};
            for (int j = k; j < n; j++)
                if (calls[j].lat == c.lat) op.owners.push_back(calls[j].done);
            t.parts.push_back(op);
        }
    }
    const unsigned lds = B.h.interleave ? 0u : cap_lds_bytes(c0.lat, c0.prec, bs, c0.mode);
    if (c0.prec == P64) dispatch_mode<P64>(B, c0.mode, c0.red, blocks, bs, lds, s, 12);
    else if (c0.prec == P32) dispatch_mode<P32>(B, c0.mode, c0.red, blocks, bs, lds, s, lr);
    else dispatch_mode<P16>(B, c0.mode, c0.red, blocks, bs, lds, s, 12);
    WC_HIP(hipGetLastError());
    if (tl->timing) timing_end(tl, t);
    if (c0.red != R_NONE && c0.mode == M_DHAT) {
        FinArgs f[kMaxSys];
        for (int k = 0; k < n; k++) {
            f[k] = FinArgs{};
            f[k].blocks = blocks_of(calls[k].lat->Vh, bs);
            f[k].op = FIN_STORE;
            f[k].partials = calls[k].red_to.partials;
            f[k].result = calls[k].red_to.result;
            f[k].guard = calls[k].done;
        }
        return launch_fin_batch(s, f, n, c0.red == R_DOT ? 2 : 3);
    }
    return WC_OK;
}

std::atomic<double> g_barrier_timeout_s{2.0};

// The inner loop as one cooperative launch; *ran = false (and WC_OK) when the
// lattice is too large for all its workgroups to be resident at once, so the
// caller uses the launched loop instead.
int launch_inner_persistent(const PersistCall &c, hipStream_t s, bool *ran) {
    *ran = false;
    wc_lattice *lat = c.lat;
    const int lr = c.prec == P32 ? lat->recon : 12;
    PersistArgs A;
    A.g = lat->g;
    A.links = (const char *)link_base(lat, c.prec);
    A.link_slab = link_slab_for(lat, c.prec);
    const char *ci = (const char *)lat->clovinv[c.prec];
    A.clov_e = ci;
    A.clov_o = ci + clover_slab_bytes(c.prec, lat->Vh);
    A.r = c.r;
    A.rt = c.rt;
    A.p = c.p;
    A.q = c.q;
    A.t = c.t;
    A.tmp = c.tmp;
    A.x = c.x;
    A.part[0] = c.part0;
    A.part[1] = c.part1;
    A.sc = c.sc;
    A.fl = c.fl;
    A.kappa2 = lat->kappa * lat->kappa;
    A.maxit = c.maxit;
    A.nblk = blocks_of(lat->Vh, kBlock);  // its own 256-thread layout
    // the runtime's barrier is the cheaper one for a handful of blocks only
    A.bar = A.nblk >= kOwnBarrierMinBlocks ? c.bar : nullptr;
    A.epoch = c.epoch;
    A.tag0 = (unsigned long long)c.epoch << 32;
    const bool own = A.bar != nullptr;
    const void *fn = c.prec == P64 ? (own ? (const void *)k_inner_persistent<P64, 12, true>
                                          : (const void *)k_inner_persistent<P64, 12, false>)
                     : c.prec == P16 ? (own ? (const void *)k_inner_persistent<P16, 12, true>
                                            : (const void *)k_inner_persistent<P16, 12, false>)
                     : lr == 8 ? (own ? (const void *)k_inner_persistent<P32, 8, true>
                                      : (const void *)k_inner_persistent<P32, 8, false>)
                     : lr == 18 ? (own ? (const void *)k_inner_persistent<P32, 18, true>
                                       : (const void *)k_inner_persistent<P32, 18, false>)
                                : (own ? (const void *)k_inner_persistent<P32, 12, true>
                                       : (const void *)k_inner_persistent<P32, 12, false>);
    int dev = 0, cus = 0, per_cu = 0, coop = 0, clock_khz = 0;
    WC_HIP(hipGetDevice(&dev));
    WC_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
    A.limit = (long long)(g_barrier_timeout_s.load() * 1e3 * clock_khz);
    WC_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    WC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    WC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0));
    if (!coop || (long)per_cu * cus < A.nblk) return WC_OK;
    void *args[] = {&A};
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(A.nblk), dim3(kBlock), args, 0, s);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();  // not resident all at once after all: use the launched loop
        return WC_OK;
    }
    if (e != hipSuccess) return wc_fail(WC_EHIP, std::string("cooperative launch: ") + hipGetErrorString(e));
    *ran = true;
    return WC_OK;
}
