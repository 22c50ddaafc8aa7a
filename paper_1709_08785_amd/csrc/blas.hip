// BLAS-1 with fused global reductions, and the vector updates of the two
// BiCGStab loops (Algorithms 1 and 2), one thread per site.
//
// The BiCGStab coefficients never travel through the host: every update
// kernel recomputes alpha = rho0 / <r~, q>, omega = <t, s> / ||t||^2 and
// beta = (rho1 / rho0) (alpha / omega) from the device scalar block written
// by the preceding reductions.  rho alternates between two slots, so the
// value that becomes rho1 never overwrites the rho0 still in use.  The
// finalize stage of a reduction also raises the level's done flag; every
// later kernel of the level returns at once when the flag is set, so the
// host may queue several iterations between convergence reads.
#include "reduce.hpp"

namespace {

__device__ __forceinline__ int rho_slot(int iter) { return (iter & 1) ? S_RHO1 : S_RHO0; }

__device__ __forceinline__ bool finite_c(cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

// ------------------------------------------------------------------ FP64 helpers
// ||v||^2 into result[0], and 0 into result[1] (so the pair reads as a complex number)
__global__ __launch_bounds__(kBlock) void k_norm2_p64(int Vh, const void *v, RedTarget to) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double a[2] = {0.0, 0.0};
    if (i < Vh) {
        const Spinor<double> s = SpinorIO<P64>::load(v, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) a[0] += norm2(s.c[k]);
    }
    block_partials<2>(a, to.partials);
}

__global__ __launch_bounds__(kBlock) void k_sub_norm_p64(int Vh, void *r, const void *x, const void *y, RedTarget to) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double a[1] = {0.0};
    if (i < Vh) {
        const Spinor<double> s = SpinorIO<P64>::load(x, Vh, i);
        const Spinor<double> t = SpinorIO<P64>::load(y, Vh, i);
        Spinor<double> o;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            o.c[k] = s.c[k] - t.c[k];
            a[0] += norm2(o.c[k]);
        }
        SpinorIO<P64>::store(r, Vh, i, o);
    }
    block_partials<1>(a, to.partials);
}

__global__ __launch_bounds__(kBlock) void k_axpy_p64(int Vh, void *y, const void *x, double alpha) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Vh) return;
    Spinor<double> a = SpinorIO<P64>::load(y, Vh, i);
    const Spinor<double> b = SpinorIO<P64>::load(x, Vh, i);
#pragma unroll
    for (int k = 0; k < 12; k++) a.c[k] = a.c[k] + alpha * b.c[k];
    SpinorIO<P64>::store(y, Vh, i, a);
}

__global__ __launch_bounds__(kBlock) void k_zero(size_t n16, uint4 *p) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ Algorithm 2
// b = src / ||src||; x = 0; r = r~ = p = b; rho0 = <r~, r>
template <int P, int XP>
__global__ __launch_bounds__(kBlock) void k_inner_init(int Vh, const void *src, void *r, void *rt, void *p, void *x,
                                                       const double *sc, double *partials) {
    using R = typename Real<P>::T;
    using RX = typename Real<XP>::T;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double a[1] = {0.0};
    if (i < Vh) {
        const double inv = 1.0 / sqrt(sc[S_NORM]);
        const Spinor<double> s = SpinorIO<P64>::load(src, Vh, i);
        Spinor<R> b;
#pragma unroll
        for (int k = 0; k < 12; k++) b.c[k] = {(R)(inv * s.c[k].re), (R)(inv * s.c[k].im)};
        SpinorIO<P>::store(r, Vh, i, b);
        SpinorIO<P>::store(rt, Vh, i, b);
        SpinorIO<P>::store(p, Vh, i, b);
        Spinor<RX> z;
#pragma unroll
        for (int k = 0; k < 12; k++) z.c[k] = {RX(0), RX(0)};
        SpinorIO<XP>::store(x, Vh, i, z);
        const Spinor<R> bs = SpinorIO<P>::load(r, Vh, i);  // the stored (rounded) value
#pragma unroll
        for (int k = 0; k < 12; k++) a[0] += norm2(bs.c[k]);
    }
    block_partials<1>(a, partials);
}

// alpha = rho0 / <r~, q>;  s = r - alpha q (in place in r);  ||s||^2
template <int P>
__global__ __launch_bounds__(kBlock) void k_inner_a(int Vh, void *r, const void *q, const double *sc, const int *fl,
                                                    int iter, double *partials) {
    using R = typename Real<P>::T;
    if (fl[F_DONE]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const cx<double> al = cdiv(ld_c(sc, rho_slot(iter)), ld_c(sc, S_RQ));
    const cx<R> alpha = {(R)al.re, (R)al.im};
    double a[1] = {0.0};
    if (i < Vh) {
        Spinor<R> rv = SpinorIO<P>::load(r, Vh, i);
        const Spinor<R> qv = SpinorIO<P>::load(q, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) rv.c[k] = rv.c[k] - alpha * qv.c[k];
        SpinorIO<P>::store(r, Vh, i, rv);
#pragma unroll
        for (int k = 0; k < 12; k++) a[0] += norm2(rv.c[k]);
    }
    block_partials<1>(a, partials);
}

// omega = <t, s> / ||t||^2;  x += alpha p + omega s;  r = s - omega t;  ||r||^2, rho1 = <r~, r>
template <int P, int XP>
__global__ __launch_bounds__(kBlock) void k_inner_b(int Vh, void *x, void *r, const void *p, const void *t,
                                                    const void *rt, const double *sc, const int *fl, int iter,
                                                    double *partials) {
    using R = typename Real<P>::T;
    using RX = typename Real<XP>::T;
    if (fl[F_DONE]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const cx<double> al = cdiv(ld_c(sc, rho_slot(iter)), ld_c(sc, S_RQ));
    const double tt = sc[S_TT];
    const cx<double> om = {sc[S_ST] / tt, -sc[S_ST + 1] / tt};
    const cx<RX> alx = {(RX)al.re, (RX)al.im}, omx = {(RX)om.re, (RX)om.im};
    const cx<R> omega = {(R)om.re, (R)om.im};
    double a[3] = {0.0, 0.0, 0.0};
    if (i < Vh) {
        Spinor<R> sv = SpinorIO<P>::load(r, Vh, i);
        const Spinor<R> pv = SpinorIO<P>::load(p, Vh, i);
        Spinor<RX> xv = SpinorIO<XP>::load(x, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const cx<RX> pk = {(RX)pv.c[k].re, (RX)pv.c[k].im}, sk = {(RX)sv.c[k].re, (RX)sv.c[k].im};
            xv.c[k] = xv.c[k] + alx * pk + omx * sk;
        }
        SpinorIO<XP>::store(x, Vh, i, xv);
        const Spinor<R> tv = SpinorIO<P>::load(t, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) sv.c[k] = sv.c[k] - omega * tv.c[k];
        SpinorIO<P>::store(r, Vh, i, sv);
        const Spinor<R> rtv = SpinorIO<P>::load(rt, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            a[0] += norm2(sv.c[k]);
            const double ar = rtv.c[k].re, ai = rtv.c[k].im, br = sv.c[k].re, bi = sv.c[k].im;
            a[1] += ar * br + ai * bi;
            a[2] += ar * bi - ai * br;
        }
    }
    block_partials<3>(a, partials);
}

// beta = (rho1 / rho0) (alpha / omega);  p = r + beta (p - omega q)
template <int P>
__global__ __launch_bounds__(kBlock) void k_inner_c(int Vh, void *p, const void *r, const void *q, const double *sc,
                                                    const int *fl, int iter) {
    using R = typename Real<P>::T;
    if (fl && fl[F_DONE]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Vh) return;
    const cx<double> rho0 = ld_c(sc, rho_slot(iter)), rho1 = ld_c(sc, rho_slot(iter + 1));
    const cx<double> al = cdiv(rho0, ld_c(sc, S_RQ));
    const double tt = sc[S_TT];
    const cx<double> om = {sc[S_ST] / tt, -sc[S_ST + 1] / tt};
    const cx<double> be = cdiv(rho1, rho0) * cdiv(al, om);
    const cx<R> beta = {(R)be.re, (R)be.im}, omega = {(R)om.re, (R)om.im};
    Spinor<R> pv = SpinorIO<P>::load(p, Vh, i);
    const Spinor<R> rv = SpinorIO<P>::load(r, Vh, i);
    const Spinor<R> qv = SpinorIO<P>::load(q, Vh, i);
#pragma unroll
    for (int k = 0; k < 12; k++) pv.c[k] = rv.c[k] + beta * (pv.c[k] - omega * qv.c[k]);
    SpinorIO<P>::store(p, Vh, i, pv);
}

// x += alpha p (the update skipped when the half step already converged)
template <int P, int XP>
__global__ __launch_bounds__(kBlock) void k_inner_fix(int Vh, void *x, const void *p, const double *sc, int iter) {
    using R = typename Real<P>::T;
    using RX = typename Real<XP>::T;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Vh) return;
    const cx<double> al = cdiv(ld_c(sc, rho_slot(iter)), ld_c(sc, S_RQ));
    const cx<RX> alx = {(RX)al.re, (RX)al.im};
    Spinor<RX> xv = SpinorIO<XP>::load(x, Vh, i);
    const Spinor<R> pv = SpinorIO<P>::load(p, Vh, i);
#pragma unroll
    for (int k = 0; k < 12; k++) xv.c[k] = xv.c[k] + alx * cx<RX>{(RX)pv.c[k].re, (RX)pv.c[k].im};
    SpinorIO<XP>::store(x, Vh, i, xv);
}

// v = ||src|| x  (Algorithm 2, last step), into FP64
template <int XP>
__global__ __launch_bounds__(kBlock) void k_inner_final(int Vh, void *v, const void *x, const double *sc) {
    using RX = typename Real<XP>::T;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Vh) return;
    const double nrm = sqrt(sc[S_NORM]);
    const Spinor<RX> xv = SpinorIO<XP>::load(x, Vh, i);
    Spinor<double> o;
#pragma unroll
    for (int k = 0; k < 12; k++) o.c[k] = {nrm * (double)xv.c[k].re, nrm * (double)xv.c[k].im};
    SpinorIO<P64>::store(v, Vh, i, o);
}

// ------------------------------------------------------------------ Algorithm 1 (FP64)
// alpha = rho0 / <r~, q>;  x += alpha v;  r -= alpha q;  ||r||^2
__global__ __launch_bounds__(kBlock) void k_outer_a(int Vh, void *x, void *r, const void *v, const void *q,
                                                    const double *sc, int iter, double *partials) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const cx<double> al = cdiv(ld_c(sc, rho_slot(iter)), ld_c(sc, S_RQ));
    double a[1] = {0.0};
    if (i < Vh) {
        Spinor<double> xv = SpinorIO<P64>::load(x, Vh, i);
        Spinor<double> rv = SpinorIO<P64>::load(r, Vh, i);
        const Spinor<double> vv = SpinorIO<P64>::load(v, Vh, i);
        const Spinor<double> qv = SpinorIO<P64>::load(q, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xv.c[k] = xv.c[k] + al * vv.c[k];
            rv.c[k] = rv.c[k] - al * qv.c[k];
            a[0] += norm2(rv.c[k]);
        }
        SpinorIO<P64>::store(x, Vh, i, xv);
        SpinorIO<P64>::store(r, Vh, i, rv);
    }
    block_partials<1>(a, partials);
}

// omega = <t, r> / ||t||^2;  x += omega v;  r -= omega t;  ||r||^2, rho1 = <r~, r>
__global__ __launch_bounds__(kBlock) void k_outer_b(int Vh, void *x, void *r, const void *v, const void *t,
                                                    const void *rt, const double *sc, double *partials) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double tt = sc[S_TT];
    const cx<double> om = {sc[S_ST] / tt, -sc[S_ST + 1] / tt};
    double a[3] = {0.0, 0.0, 0.0};
    if (i < Vh) {
        Spinor<double> xv = SpinorIO<P64>::load(x, Vh, i);
        Spinor<double> rv = SpinorIO<P64>::load(r, Vh, i);
        const Spinor<double> vv = SpinorIO<P64>::load(v, Vh, i);
        const Spinor<double> tv = SpinorIO<P64>::load(t, Vh, i);
        const Spinor<double> rtv = SpinorIO<P64>::load(rt, Vh, i);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xv.c[k] = xv.c[k] + om * vv.c[k];
            rv.c[k] = rv.c[k] - om * tv.c[k];
            a[0] += norm2(rv.c[k]);
            const double ar = rtv.c[k].re, ai = rtv.c[k].im, br = rv.c[k].re, bi = rv.c[k].im;
            a[1] += ar * br + ai * bi;
            a[2] += ar * bi - ai * br;
        }
        SpinorIO<P64>::store(x, Vh, i, xv);
        SpinorIO<P64>::store(r, Vh, i, rv);
    }
    block_partials<3>(a, partials);
}

// ------------------------------------------------------------------ reduction stage 2
template <int N> __global__ __launch_bounds__(kBlock) void k_finalize(FinArgs f) {
    if (f.guard && *f.guard) return;
    __shared__ double sh[N][kWaves];
    double a[N];
#pragma unroll
    for (int k = 0; k < N; k++) a[k] = 0.0;
    for (int j = threadIdx.x; j < f.blocks; j += kBlock) {
#pragma unroll
        for (int k = 0; k < N; k++) a[k] += f.partials[(size_t)k * f.blocks + j];
    }
    block_fold<N>(a, sh);
    if (threadIdx.x != 0) return;
    double *sc = f.sc;
    int *fl = f.fl;
    switch (f.op) {
    case FIN_STORE:
        for (int k = 0; k < N; k++) f.result[k] = a[k];
        break;
    case FIN_INIT:
        sc[S_RHO0] = a[0];
        sc[S_RHO0 + 1] = 0.0;
        fl[F_DONE] = DONE_NO;
        fl[F_ITERS] = 0;
        break;
    case FIN_INNER_A: {
        const cx<double> al = cdiv(ld_c(sc, rho_slot(f.iter)), ld_c(sc, S_RQ));
        sc[S_SS] = a[0];
        if (!finite_c(al) || !isfinite(a[0])) fl[F_DONE] = DONE_BREAK;
        else if (a[0] < f.tol2) fl[F_DONE] = DONE_HALF;
        break;
    }
    case FIN_INNER_B: {
        const int nxt = rho_slot(f.iter + 1);
        const double tt = sc[S_TT];
        const cx<double> om = {sc[S_ST] / tt, -sc[S_ST + 1] / tt};
        sc[S_RR] = a[0];
        sc[nxt] = a[1];
        sc[nxt + 1] = a[2];
        fl[F_ITERS] = f.iter + 1;
        if (!(tt > 0.0) || !finite_c(om) || !isfinite(a[0]) || (a[1] == 0.0 && a[2] == 0.0))
            fl[F_DONE] = (a[0] < f.tol2) ? DONE_FULL : DONE_BREAK;
        else if (a[0] < f.tol2)
            fl[F_DONE] = DONE_FULL;
        break;
    }
    case FIN_OUTER_B: {
        const int nxt = rho_slot(f.iter + 1);
        sc[S_RR] = a[0];
        sc[nxt] = a[1];
        sc[nxt + 1] = a[2];
        break;
    }
    }
}

inline int nblk(int Vh) { return (Vh + kBlock - 1) / kBlock; }

template <class F> int timed_blas(wc_lattice *lat, double bytes, F &&launch) {
    TimedLaunch t;
    if (lat->timing) timing_begin(lat, KS_BLAS, bytes, t);
    launch();
    WC_HIP(hipGetLastError());
    if (lat->timing) timing_end(lat, t);
    return WC_OK;
}

inline double S(int prec, int Vh) { return (double)spinor_bytes(prec, Vh); }

}  // namespace

int launch_finalize(wc_lattice *lat, const FinArgs &f) {
    switch (f.n) {
    case 1: hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kBlock), 0, lat->stream, f); break;
    case 2: hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kBlock), 0, lat->stream, f); break;
    default: hipLaunchKernelGGL(k_finalize<3>, dim3(1), dim3(kBlock), 0, lat->stream, f); break;
    }
    WC_HIP(hipGetLastError());
    return WC_OK;
}

static FinArgs fin(wc_lattice *lat, int n, int op, int lvl, double *result, const int *guard, int iter) {
    FinArgs f{};
    f.n = n;
    f.blocks = nblk(lat->Vh);
    f.op = op;
    f.partials = lat->partials;
    f.result = result;
    f.sc = lat->level_scalars(lvl);
    f.fl = lat->level_flags(lvl);
    f.guard = guard;
    f.iter = iter;
    f.tol2 = lat->host_tol2[lvl];
    return f;
}

int launch_norm2_p64(wc_lattice *lat, const void *v, RedTarget to) {
    int rc = timed_blas(lat, S(P64, lat->Vh), [&] {
        hipLaunchKernelGGL(k_norm2_p64, dim3(nblk(lat->Vh)), dim3(kBlock), 0, lat->stream, lat->Vh, v, to);
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 2, FIN_STORE, 0, to.result, nullptr, 0));
}

int launch_sub_norm_p64(wc_lattice *lat, void *r, const void *a, const void *b, RedTarget to) {
    int rc = timed_blas(lat, 3 * S(P64, lat->Vh), [&] {
        hipLaunchKernelGGL(k_sub_norm_p64, dim3(nblk(lat->Vh)), dim3(kBlock), 0, lat->stream, lat->Vh, r, a, b, to);
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 1, FIN_STORE, 0, to.result, nullptr, 0));
}

int launch_axpy_p64(wc_lattice *lat, void *y, const void *x, double a) {
    return timed_blas(lat, 3 * S(P64, lat->Vh), [&] {
        hipLaunchKernelGGL(k_axpy_p64, dim3(nblk(lat->Vh)), dim3(kBlock), 0, lat->stream, lat->Vh, y, x, a);
    });
}

int launch_copy(wc_lattice *lat, void *dst, const void *src, size_t bytes) {
    WC_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, lat->stream));
    return WC_OK;
}

int launch_zero(wc_lattice *lat, void *dst, size_t bytes) {
    // sizes here are multiples of 16 bytes (every field is a whole number of uint4)
    const size_t n16 = bytes / 16;
    const unsigned blocks = (unsigned)((n16 + kBlock - 1) / kBlock);
    if (blocks == 0) return WC_OK;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(kBlock), 0, lat->stream, n16, (uint4 *)dst);
    WC_HIP(hipGetLastError());
    return WC_OK;
}

#define WC_PREC_SWITCH(prec, BODY)      \
    do {                                \
        if ((prec) == P64) {            \
            constexpr int PP = P64;     \
            BODY;                       \
        } else if ((prec) == P32) {     \
            constexpr int PP = P32;     \
            BODY;                       \
        } else {                        \
            constexpr int PP = P16;     \
            BODY;                       \
        }                               \
    } while (0)

#define WC_XPREC_SWITCH(xprec, BODY)    \
    do {                                \
        if ((xprec) == P64) {           \
            constexpr int XX = P64;     \
            BODY;                       \
        } else {                        \
            constexpr int XX = P32;     \
            BODY;                       \
        }                               \
    } while (0)

int launch_inner_init(wc_lattice *lat, int prec, int xprec, const void *src64, void *r, void *rt, void *p, void *x,
                      int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    double *part = lat->partials;
    int rc = timed_blas(lat, S(P64, Vh) + 3 * S(prec, Vh) + S(xprec, Vh), [&] {
        WC_PREC_SWITCH(prec, WC_XPREC_SWITCH(xprec, hipLaunchKernelGGL((k_inner_init<PP, XX>), dim3(nblk(Vh)),
                                                                        dim3(kBlock), 0, lat->stream, Vh, src64, r,
                                                                        rt, p, x, sc, part)));
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 1, FIN_INIT, lvl, nullptr, nullptr, 0));
}

int launch_inner_a(wc_lattice *lat, int prec, void *r, const void *q, int iter, int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    const int *fl = lat->level_flags(lvl);
    double *part = lat->partials;
    int rc = timed_blas(lat, 3 * S(prec, Vh), [&] {
        WC_PREC_SWITCH(prec, hipLaunchKernelGGL((k_inner_a<PP>), dim3(nblk(Vh)), dim3(kBlock), 0, lat->stream, Vh,
                                                r, q, sc, fl, iter, part));
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 1, FIN_INNER_A, lvl, nullptr, fl, iter));
}

int launch_inner_b(wc_lattice *lat, int prec, int xprec, void *x, void *r, const void *p, const void *t,
                   const void *rt, int iter, int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    const int *fl = lat->level_flags(lvl);
    double *part = lat->partials;
    int rc = timed_blas(lat, 5 * S(prec, Vh) + 2 * S(xprec, Vh), [&] {
        WC_PREC_SWITCH(prec, WC_XPREC_SWITCH(xprec, hipLaunchKernelGGL((k_inner_b<PP, XX>), dim3(nblk(Vh)),
                                                                        dim3(kBlock), 0, lat->stream, Vh, x, r, p, t,
                                                                        rt, sc, fl, iter, part)));
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 3, FIN_INNER_B, lvl, nullptr, fl, iter));
}

int launch_inner_c(wc_lattice *lat, int prec, void *p, const void *r, const void *q, int iter, int lvl, bool guard) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    const int *fl = guard ? lat->level_flags(lvl) : nullptr;
    return timed_blas(lat, 4 * S(prec, Vh), [&] {
        WC_PREC_SWITCH(prec, hipLaunchKernelGGL((k_inner_c<PP>), dim3(nblk(Vh)), dim3(kBlock), 0, lat->stream, Vh,
                                                p, r, q, sc, fl, iter));
    });
}

int launch_inner_fix(wc_lattice *lat, int prec, int xprec, void *x, const void *p, int iter, int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    return timed_blas(lat, S(prec, Vh) + 2 * S(xprec, Vh), [&] {
        WC_PREC_SWITCH(prec, WC_XPREC_SWITCH(xprec, hipLaunchKernelGGL((k_inner_fix<PP, XX>), dim3(nblk(Vh)),
                                                                        dim3(kBlock), 0, lat->stream, Vh, x, p, sc,
                                                                        iter)));
    });
}

int launch_inner_final(wc_lattice *lat, int xprec, void *v64, const void *x, int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    return timed_blas(lat, S(xprec, Vh) + S(P64, Vh), [&] {
        WC_XPREC_SWITCH(xprec, hipLaunchKernelGGL((k_inner_final<XX>), dim3(nblk(Vh)), dim3(kBlock), 0, lat->stream,
                                                  Vh, v64, x, sc));
    });
}

int launch_outer_a(wc_lattice *lat, void *x, void *r, const void *v, const void *q, int iter, int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    double *part = lat->partials;
    int rc = timed_blas(lat, 6 * S(P64, Vh), [&] {
        hipLaunchKernelGGL(k_outer_a, dim3(nblk(Vh)), dim3(kBlock), 0, lat->stream, Vh, x, r, v, q, sc, iter, part);
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 1, FIN_STORE, lvl, lat->level_scalars(lvl) + S_RR, nullptr, iter));
}

int launch_outer_b(wc_lattice *lat, void *x, void *r, const void *v, const void *t, const void *rt, int iter,
                   int lvl) {
    const int Vh = lat->Vh;
    const double *sc = lat->level_scalars(lvl);
    double *part = lat->partials;
    int rc = timed_blas(lat, 7 * S(P64, Vh), [&] {
        hipLaunchKernelGGL(k_outer_b, dim3(nblk(Vh)), dim3(kBlock), 0, lat->stream, Vh, x, r, v, t, rt, sc, part);
    });
    if (rc) return rc;
    return launch_finalize(lat, fin(lat, 3, FIN_OUTER_B, lvl, nullptr, nullptr, iter));
}
