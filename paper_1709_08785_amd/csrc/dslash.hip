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

template <int P, int MU, bool NT, bool R8>
__device__ __forceinline__ void hop_dir(const MultKArgs &a, const SiteCoord &c, int i,
                                        Spinor<typename Real<P>::T> &acc) {
    using R = typename Real<P>::T;
    const int Vh = a.g.Vh;
    {
        const int nf = eo_neighbour(a.g, c, MU, +1);
        const Mat3<R> U = LinkLoad<P, R8>::template load<NT>(a.links + (size_t)(2 * MU + a.out_par) * a.link_slab, Vh, i);
        hop_one<P, MU, true>(a.in, Vh, nf, U, acc);
    }
    {
        const int nb = eo_neighbour(a.g, c, MU, -1);
        const Mat3<R> U =
            LinkLoad<P, R8>::template load<NT>(a.links + (size_t)(2 * MU + 1 - a.out_par) * a.link_slab, Vh, nb);
        hop_one<P, MU, false>(a.in, Vh, nb, U, acc);
    }
}

// logical block of hardware block b: XCD (b mod 8) takes the slab
// [(b mod 8) per, (b mod 8 + 1) per); a ragged tail keeps its own index
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3;
    return (b < (per << 3)) ? (b & 7) * per + (b >> 3) : b;
}

// NT: links and clover read once per launch (one system) use non-temporal
// loads; a launch that serves several systems on one lattice reads them
// through the cache so that the blocks of the other systems hit in L2
template <int P, int MODE, int RED, bool NT, bool R8>
__global__ __launch_bounds__(kBlock) void k_mult(MultBatch B) {
    using R = typename Real<P>::T;
    int s, lb;
    batch_locate(B.h, xcd_block(blockIdx.x, gridDim.x), s, lb);
    const MultKArgs &a = B.d[s];
    if (a.done && *a.done) return;
    const int i = lb * kBlock + threadIdx.x;
    const bool active = i < a.g.Vh;
    const int Vh = a.g.Vh;
    Spinor<R> out;
    if (active) {
        Spinor<R> acc;
#pragma unroll
        for (int k = 0; k < 12; k++) acc.c[k] = {R(0), R(0)};
        if (MODE != M_CLOV) {
            const SiteCoord c = eo_coords(a.g, i, a.out_par);
            hop_dir<P, 0, NT, R8>(a, c, i, acc);
            hop_dir<P, 1, NT, R8>(a, c, i, acc);
            hop_dir<P, 2, NT, R8>(a, c, i, acc);
            hop_dir<P, 3, NT, R8>(a, c, i, acc);
        }
        const R coef = (R)a.coef;
        if (MODE == M_HOPINV) {
            clover_apply<P, R, NT>(a.clov, Vh, i, acc, out);
        } else if (MODE == M_DHAT) {
            Spinor<R> t;
            clover_apply<P, R, NT>(a.clov, Vh, i, acc, t);
            const Spinor<R> cen = SpinorIO<P>::template load<true>(a.center, Vh, i);
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
            const Spinor<R> ax = SpinorIO<P>::template load<true>(a.aux, Vh, i);
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

template <int P, int MODE, int RED, bool R8> void launch_nt(const MultBatch &B, int blocks, hipStream_t s) {
    if (B.h.interleave)
        hipLaunchKernelGGL((k_mult<P, MODE, RED, false, R8>), dim3(blocks), dim3(kBlock), 0, s, B);
    else
        hipLaunchKernelGGL((k_mult<P, MODE, RED, true, R8>), dim3(blocks), dim3(kBlock), 0, s, B);
}

// reconstruct-8 instances exist for the FP32 stencil only
template <int P, int MODE, int RED> void launch_one(const MultBatch &B, int blocks, hipStream_t s, bool r8) {
    if constexpr (P == P32) {
        if (r8) {
            launch_nt<P, MODE, RED, true>(B, blocks, s);
            return;
        }
    }
    launch_nt<P, MODE, RED, false>(B, blocks, s);
}

template <int P> void dispatch_mode(const MultBatch &B, int mode, int red, int blocks, hipStream_t s, bool r8) {
    switch (mode) {
    case M_HOPINV: launch_one<P, M_HOPINV, R_NONE>(B, blocks, s, r8); break;
    case M_DHAT:
        if (red == R_DOT) launch_one<P, M_DHAT, R_DOT>(B, blocks, s, r8);
        else if (red == R_DOTNORM) launch_one<P, M_DHAT, R_DOTNORM>(B, blocks, s, r8);
        else launch_one<P, M_DHAT, R_NONE>(B, blocks, s, r8);
        break;
    case M_DFULL: launch_one<P, M_DFULL, R_NONE>(B, blocks, s, r8); break;
    case M_INVSRC: launch_one<P, M_INVSRC, R_NONE>(B, blocks, s, r8); break;
    case M_HOP: launch_one<P, M_HOP, R_NONE>(B, blocks, s, r8); break;
    case M_CLOV: launch_one<P, M_CLOV, R_NONE>(B, blocks, s, r8); break;
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
double mult_operator_bytes(int prec, int mode, bool r8, int Vh) {
    double b = 0;
    if (mode != M_CLOV) b += 8 * (double)(r8 ? 32 : link_site_bytes(prec)) * Vh;
    if (mode != M_HOP) b += (double)clover_site_bytes(prec) * Vh;
    return b;
}

}  // namespace

int launch_mult_batch(hipStream_t s, const MultCall *calls, int n, wc_lattice *timing_lat) {
    if (n <= 0) return WC_OK;
    if (n > kMaxSys) return wc_fail(WC_EINVAL, "too many systems in one batch");
    const MultCall &c0 = calls[0];
    MultBatch B;
    B.h.S = n;
    B.h.off[0] = 0;
    bool same = true;
    double bytes = 0;
    const bool r8 = c0.prec == P32 && c0.lat->recon == 8;
    for (int k = 0; k < n; k++) {
        const MultCall &c = calls[k];
        wc_lattice *lat = c.lat;
        if (c.prec != c0.prec || c.mode != c0.mode || c.red != c0.red || c.out_par != c0.out_par)
            return wc_fail(WC_EINVAL, "batched stencil calls must share precision, mode, reduction and parity");
        same = same && (lat == c0.lat);
        MultKArgs &a = B.d[k];
        a.g = lat->g;
        a.out_par = c.out_par;
        a.out = c.out;
        a.in = c.in;
        a.center = c.center;
        a.aux = c.aux;
        if ((c.prec == P32 && lat->recon == 8) != r8)
            return wc_fail(WC_EINVAL, "batched stencil calls must share the link reconstruction");
        a.links = (const char *)(r8 ? lat->links8 : lat->links[c.prec]);
        a.link_slab = r8 ? link8_slab_bytes(lat->Vh) : link_slab_bytes(c.prec, lat->Vh);
        const bool use_inv = (c.mode == M_HOPINV || c.mode == M_DHAT || c.mode == M_INVSRC ||
                              (c.mode == M_CLOV && c.inverse));
        const char *cb = (const char *)(use_inv ? lat->clovinv[c.prec] : lat->clov[c.prec]);
        a.clov = cb + (size_t)c.out_par * clover_slab_bytes(c.prec, lat->Vh);
        a.coef = c.coef;
        a.red = c.red_to;
        a.done = c.done;
        a.nblk = lat->nblocks;
        B.h.off[k + 1] = B.h.off[k] + lat->nblocks;
        bytes += mult_spinor_bytes(c.prec, c.mode, c.red, c.aux == c.center, lat->Vh);
        bool seen = false;
        for (int j = 0; j < k; j++) seen = seen || (calls[j].lat == lat);
        if (!seen) bytes += mult_operator_bytes(c.prec, c.mode, r8, lat->Vh);
        if (c.mode != M_CLOV) lat->dslash_count++;
    }
    B.h.interleave = (same && n > 1) ? 1 : 0;
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
            TimedPart op{{}, mult_operator_bytes(c.prec, c.mode, r8, c.lat->Vh)};
            for (int j = k; j < n; j++)
                if (calls[j].lat == c.lat) op.owners.push_back(calls[j].done);
            t.parts.push_back(op);
        }
    }
    if (c0.prec == P64) dispatch_mode<P64>(B, c0.mode, c0.red, blocks, s, false);
    else if (c0.prec == P32) dispatch_mode<P32>(B, c0.mode, c0.red, blocks, s, r8);
    else dispatch_mode<P16>(B, c0.mode, c0.red, blocks, s, r8);
    WC_HIP(hipGetLastError());
    if (tl->timing) timing_end(tl, t);
    if (c0.red != R_NONE && c0.mode == M_DHAT) {
        FinArgs f[kMaxSys];
        for (int k = 0; k < n; k++) {
            f[k] = FinArgs{};
            f[k].blocks = calls[k].lat->nblocks;
            f[k].op = FIN_STORE;
            f[k].partials = calls[k].red_to.partials;
            f[k].result = calls[k].red_to.result;
            f[k].guard = calls[k].done;
        }
        return launch_fin_batch(s, f, n, c0.red == R_DOT ? 2 : 3);
    }
    return WC_OK;
}
