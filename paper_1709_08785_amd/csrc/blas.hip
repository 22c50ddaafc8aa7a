// BLAS-1 with fused global reductions, and the vector updates of the two
// BiCGStab loops (Algorithms 1 and 2), one thread per site, batched over
// systems: one launch serves every active system of a solve.
//
// The BiCGStab coefficients never travel through the host: every update
// kernel recomputes alpha = rho0 / <r~, q>, omega = <t, s> / ||t||^2 and
// beta = (rho1 / rho0) (alpha / omega) from its system's device scalar block,
// written by the preceding reductions.  rho alternates between two slots, so
// the value that becomes rho1 never overwrites the rho0 still in use.  The
// finalize stage of a reduction also raises the system's done flag; every
// later kernel of the loop skips a system whose flag is set, so the host may
// queue several iterations between convergence reads.
#include "reduce.hpp"

namespace {

// vector operands are streamed: each is touched once per launch
constexpr bool kVNT = true;

__device__ __forceinline__ int rho_slot(int iter) { return (iter & 1) ? S_RHO1 : S_RHO0; }

__device__ __forceinline__ bool finite_c(cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

struct VecBatch {
    BatchHdr h;
    VecCall c[kMaxSys];
};

template <class R> __device__ __forceinline__ cx<R> to(cx<double> a) { return {(R)a.re, (R)a.im}; }

// number of reduced values of each op (0: no reduction)
__host__ __device__ constexpr int red_count(int op) {
    return op == V_NORM2 ? 2
         : (op == V_SUB_NORM || op == V_INNER_INIT || op == V_INNER_A || op == V_OUTER_A || op == V_PIPE_INIT) ? 1
         : (op == V_INNER_B || op == V_OUTER_B) ? 3
         : op == V_PIPE_A ? 8
         : op == V_PIPE_B ? 5
         : 0;
}

static_assert(red_count(V_PIPE_A) <= kMaxRed && red_count(V_PIPE_B) <= kMaxRed, "partials too small");

// a += conj(x) y as (re, im) into two accumulators
template <class T> __device__ __forceinline__ void dot_acc(double &re, double &im, cx<T> x, cx<T> y) {
    const double xr = x.re, xi = x.im, yr = y.re, yi = y.im;
    re += xr * yr + xi * yi;
    im += xr * yi - xi * yr;
}

template <int OP, int P, int XP> __global__ __launch_bounds__(kBlock) void k_vec(VecBatch B) {
    using R = typename Real<P>::T;
    using RX = typename Real<XP>::T;
    constexpr int N = red_count(OP);
    constexpr int NA = N > 0 ? N : 1;
    int s, lb;
    batch_locate(B.h, blockIdx.x, s, lb);
    const VecCall &c = B.c[s];
    if (c.guard && c.fl[F_DONE]) return;
    const int Vh = c.Vh;
    // inner-loop kernels take the iteration index from the device, so a
    // captured chunk of iterations replays unchanged; the p update runs after
    // the iteration count has been advanced
    const int iter = c.iter_dev ? c.fl[F_ITERS] - (OP == V_INNER_C ? 1 : 0) : c.iter;
    const int i = lb * (int)blockDim.x + threadIdx.x;  // 64, 128 or 256 sites per block
    const bool active = i < Vh;
    double a[NA];
#pragma unroll
    for (int k = 0; k < NA; k++) a[k] = 0.0;

    if (OP == V_NORM2) {
        if (active) {
            const Spinor<double> v = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) a[0] += norm2(v.c[k]);
        }
    } else if (OP == V_SUB_NORM) {
        if (active) {
            const Spinor<double> x = SpinorIO<P64>::template load<kVNT>(c.b, Vh, i);
            const Spinor<double> y = SpinorIO<P64>::template load<kVNT>(c.c, Vh, i);
            Spinor<double> o;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                o.c[k] = x.c[k] - y.c[k];
                a[0] += norm2(o.c[k]);
            }
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, o);
        }
    } else if (OP == V_AXPY) {
        if (active) {
            Spinor<double> y = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
            const Spinor<double> x = SpinorIO<P64>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) y.c[k] = y.c[k] + c.coef * x.c[k];
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, y);
        }
    } else if (OP == V_COPY) {
        if (active) SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, SpinorIO<P64>::template load<kVNT>(c.b, Vh, i));
    } else if (OP == V_ZERO) {
        if (active) {
            Spinor<double> z;
#pragma unroll
            for (int k = 0; k < 12; k++) z.c[k] = {0.0, 0.0};
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, z);
        }
    } else if (OP == V_GAMMA5) {
        // g5 = -[[0, 1], [1, 0]] in upper/lower spin blocks, both parity slabs
        if (active) {
            for (int par = 0; par < 2; par++) {
                char *v = (char *)c.a + (size_t)par * spinor_bytes(P64, Vh);
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    double2 *pu = tp<double2, 192>(v, i, 16 * k), *pd = tp<double2, 192>(v, i, 16 * (k + 6));
                    const double2 up = *pu, dn = *pd;
                    *pu = make_double2(-dn.x, -dn.y);
                    *pd = make_double2(-up.x, -up.y);
                }
            }
        }
    } else if (OP == V_INNER_INIT) {
        // b = src / ||src||; x = 0; r = r~ = p = b; rho0 = <r~, r> of the stored values
        if (active) {
            const double nrm2 = c.sc[S_NORM];
            const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
            const Spinor<double> v = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
            Spinor<R> b;
#pragma unroll
            for (int k = 0; k < 12; k++) b.c[k] = {(R)(inv * v.c[k].re), (R)(inv * v.c[k].im)};
            SpinorIO<P>::template store<kVNT>(c.b, Vh, i, b);
            SpinorIO<P>::template store<kVNT>(c.c, Vh, i, b);
            SpinorIO<P>::template store<kVNT>(c.d, Vh, i, b);
            Spinor<RX> z;
#pragma unroll
            for (int k = 0; k < 12; k++) z.c[k] = {RX(0), RX(0)};
            SpinorIO<XP>::template store<kVNT>(c.e, Vh, i, z);
            const Spinor<R> bs = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) a[0] += norm2(bs.c[k]);
        }
    } else if (OP == V_INNER_A) {
        // alpha = rho0 / <r~, q>;  s = r - alpha q (in place in r);  ||s||^2
        const cx<R> alpha = to<R>(cdiv(ld_c(c.sc, rho_slot(iter)), ld_c(c.sc, S_RQ)));
        if (active) {
            Spinor<R> rv = SpinorIO<P>::template load<kVNT>(c.a, Vh, i);
            const Spinor<R> qv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) rv.c[k] = rv.c[k] - alpha * qv.c[k];
            SpinorIO<P>::template store<kVNT>(c.a, Vh, i, rv);
#pragma unroll
            for (int k = 0; k < 12; k++) a[0] += norm2(rv.c[k]);
        }
    } else if (OP == V_INNER_B) {
        // omega = <t, s> / ||t||^2;  x += alpha p + omega s;  r = s - omega t;  ||r||^2, <r~, r>
        const cx<double> al = cdiv(ld_c(c.sc, rho_slot(iter)), ld_c(c.sc, S_RQ));
        const double tt = c.sc[S_TT];
        const cx<double> om = {c.sc[S_ST] / tt, -c.sc[S_ST + 1] / tt};
        const cx<RX> alx = to<RX>(al), omx = to<RX>(om);
        const cx<R> omega = to<R>(om);
        if (active) {
            Spinor<R> sv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
            const Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.c, Vh, i);
            Spinor<RX> xv = SpinorIO<XP>::template load<kVNT>(c.a, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<RX> pk = {(RX)pv.c[k].re, (RX)pv.c[k].im}, sk = {(RX)sv.c[k].re, (RX)sv.c[k].im};
                xv.c[k] = xv.c[k] + alx * pk + omx * sk;
            }
            SpinorIO<XP>::template store<kVNT>(c.a, Vh, i, xv);
            const Spinor<R> tv = SpinorIO<P>::template load<kVNT>(c.d, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) sv.c[k] = sv.c[k] - omega * tv.c[k];
            SpinorIO<P>::template store<kVNT>(c.b, Vh, i, sv);
            const Spinor<R> rtv = SpinorIO<P>::template load<kVNT>(c.e, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                a[0] += norm2(sv.c[k]);
                const double ar = rtv.c[k].re, ai = rtv.c[k].im, br = sv.c[k].re, bi = sv.c[k].im;
                a[1 % NA] += ar * br + ai * bi;
                a[2 % NA] += ar * bi - ai * br;
            }
        }
    } else if (OP == V_INNER_C) {
        // beta = (rho1 / rho0) (alpha / omega);  p = r + beta (p - omega q)
        if (active) {
            const cx<double> rho0 = ld_c(c.sc, rho_slot(iter)), rho1 = ld_c(c.sc, rho_slot(iter + 1));
            const cx<double> al = cdiv(rho0, ld_c(c.sc, S_RQ));
            const double tt = c.sc[S_TT];
            const cx<double> om = {c.sc[S_ST] / tt, -c.sc[S_ST + 1] / tt};
            const cx<R> beta = to<R>(cdiv(rho1, rho0) * cdiv(al, om)), omega = to<R>(om);
            Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.a, Vh, i);
            const Spinor<R> rv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
            const Spinor<R> qv = SpinorIO<P>::template load<kVNT>(c.c, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) pv.c[k] = rv.c[k] + beta * (pv.c[k] - omega * qv.c[k]);
            SpinorIO<P>::template store<kVNT>(c.a, Vh, i, pv);
        }
    } else if (OP == V_INNER_FIX) {
        // x += alpha p (the update skipped when the half step already converged)
        if (active) {
            const cx<RX> alx = to<RX>(cdiv(ld_c(c.sc, rho_slot(iter)), ld_c(c.sc, S_RQ)));
            Spinor<RX> xv = SpinorIO<XP>::template load<kVNT>(c.a, Vh, i);
            const Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) xv.c[k] = xv.c[k] + alx * cx<RX>{(RX)pv.c[k].re, (RX)pv.c[k].im};
            SpinorIO<XP>::template store<kVNT>(c.a, Vh, i, xv);
        }
    } else if (OP == V_INNER_FINAL) {
        // v = ||src|| x into FP64 (Algorithm 2, last step)
        if (active) {
            const double nrm = sqrt(c.sc[S_NORM]);
            const Spinor<RX> xv = SpinorIO<XP>::template load<kVNT>(c.b, Vh, i);
            Spinor<double> o;
#pragma unroll
            for (int k = 0; k < 12; k++) o.c[k] = {nrm * (double)xv.c[k].re, nrm * (double)xv.c[k].im};
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, o);
        }
    } else if (OP == V_OUTER_A) {
        // alpha = rho0 / <r~, q>;  x += alpha v;  r -= alpha q;  ||r||^2
        const cx<double> al = cdiv(ld_c(c.sc, rho_slot(iter)), ld_c(c.sc, S_RQ));
        if (active) {
            Spinor<double> xv = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
            Spinor<double> rv = SpinorIO<P64>::template load<kVNT>(c.b, Vh, i);
            const Spinor<double> vv = SpinorIO<P64>::template load<kVNT>(c.c, Vh, i);
            const Spinor<double> qv = SpinorIO<P64>::template load<kVNT>(c.d, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                xv.c[k] = xv.c[k] + al * vv.c[k];
                rv.c[k] = rv.c[k] - al * qv.c[k];
                a[0] += norm2(rv.c[k]);
            }
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, xv);
            SpinorIO<P64>::template store<kVNT>(c.b, Vh, i, rv);
        }
    } else if (OP == V_OUTER_B) {
        // omega = <t, r> / ||t||^2;  x += omega v;  r -= omega t;  ||r||^2, <r~, r>
        const double tt = c.sc[S_TT];
        const cx<double> om = {c.sc[S_ST] / tt, -c.sc[S_ST + 1] / tt};
        if (active) {
            Spinor<double> xv = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
            Spinor<double> rv = SpinorIO<P64>::template load<kVNT>(c.b, Vh, i);
            const Spinor<double> vv = SpinorIO<P64>::template load<kVNT>(c.c, Vh, i);
            const Spinor<double> tv = SpinorIO<P64>::template load<kVNT>(c.d, Vh, i);
            const Spinor<double> rtv = SpinorIO<P64>::template load<kVNT>(c.e, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                xv.c[k] = xv.c[k] + om * vv.c[k];
                rv.c[k] = rv.c[k] - om * tv.c[k];
                a[0] += norm2(rv.c[k]);
                const double ar = rtv.c[k].re, ai = rtv.c[k].im, br = rv.c[k].re, bi = rv.c[k].im;
                a[1 % NA] += ar * br + ai * bi;
                a[2 % NA] += ar * bi - ai * br;
            }
            SpinorIO<P64>::template store<kVNT>(c.a, Vh, i, xv);
            SpinorIO<P64>::template store<kVNT>(c.b, Vh, i, rv);
        }
    }
    if (OP == V_PIPE_INIT) {
        // b = src / ||src||; r = r~ = b; x = 0; p = s = z = v = 0 (the recurrences
        // start with beta = 0, so the zeros only keep them finite); rho = <r~, r>
        if (active) {
            const double nrm2 = c.sc[S_NORM];
            const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
            const Spinor<double> v = SpinorIO<P64>::template load<kVNT>(c.a, Vh, i);
            Spinor<R> b, z;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                b.c[k] = {(R)(inv * v.c[k].re), (R)(inv * v.c[k].im)};
                z.c[k] = {R(0), R(0)};
            }
            SpinorIO<P>::template store<kVNT>(c.b, Vh, i, b);
            SpinorIO<P>::template store<kVNT>(c.c, Vh, i, b);
            SpinorIO<P>::template store<kVNT>(c.e, Vh, i, z);
            SpinorIO<P>::template store<kVNT>(c.f, Vh, i, z);
            SpinorIO<P>::template store<kVNT>(c.g, Vh, i, z);
            SpinorIO<P>::template store<kVNT>(c.h, Vh, i, z);
            Spinor<RX> zx;
#pragma unroll
            for (int k = 0; k < 12; k++) zx.c[k] = {RX(0), RX(0)};
            SpinorIO<XP>::template store<kVNT>(c.d, Vh, i, zx);
            const Spinor<R> bs = SpinorIO<P>::load(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) a[0] += norm2(bs.c[k]);
        }
    } else if (OP == V_PIPE_A) {
        // p = r + beta (p - omega s); s = w + beta (s - omega z); z = t + beta (z - omega v)
        // with the new s, z: q = r - alpha s, y = w - alpha z, and the sums
        // <y, q>, ||y||^2, ||q||^2, <r~, s>, <r~, z> (q and y are not stored)
        const cx<R> al = to<R>(ld_c(c.sc, S_RQ)), om = to<R>(ld_c(c.sc, S_ST)), be = to<R>(ld_c(c.sc, S_RHO1));
        if (active) {
            const Spinor<R> s0 = SpinorIO<P>::template load<kVNT>(c.e, Vh, i);
            const Spinor<R> r = SpinorIO<P>::template load<kVNT>(c.a, Vh, i);
            {
                Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.d, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) pv.c[k] = r.c[k] + be * (pv.c[k] - om * s0.c[k]);
                SpinorIO<P>::template store<kVNT>(c.d, Vh, i, pv);
            }
            const Spinor<R> z0 = SpinorIO<P>::template load<kVNT>(c.f, Vh, i);
            const Spinor<R> w = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
            Spinor<R> sn;
#pragma unroll
            for (int k = 0; k < 12; k++) sn.c[k] = w.c[k] + be * (s0.c[k] - om * z0.c[k]);
            SpinorIO<P>::template store<kVNT>(c.e, Vh, i, sn);
            Spinor<R> zn;
            {
                const Spinor<R> t = SpinorIO<P>::template load<kVNT>(c.c, Vh, i);
                const Spinor<R> v = SpinorIO<P>::template load<kVNT>(c.g, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) zn.c[k] = t.c[k] + be * (z0.c[k] - om * v.c[k]);
            }
            SpinorIO<P>::template store<kVNT>(c.f, Vh, i, zn);
            const Spinor<R> rt = SpinorIO<P>::template load<kVNT>(c.h, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const cx<R> q = r.c[k] - al * sn.c[k], y = w.c[k] - al * zn.c[k];
                dot_acc(a[0 % NA], a[1 % NA], y, q);
                a[2 % NA] += norm2(y);
                a[3 % NA] += norm2(q);
                dot_acc(a[4 % NA], a[5 % NA], rt.c[k], sn.c[k]);
                dot_acc(a[6 % NA], a[7 % NA], rt.c[k], zn.c[k]);
            }
        }
    } else if (OP == V_PIPE_B) {
        // q = r - alpha s, y = w - alpha z; x += alpha p + omega q; r = q - omega y;
        // w = y - omega (t - alpha v); sums <r~, r>, <r~, w>, ||r||^2
        const cx<double> ald = ld_c(c.sc, S_RQ), omd = ld_c(c.sc, S_ST);
        const cx<R> al = to<R>(ald), om = to<R>(omd);
        const cx<RX> alx = to<RX>(ald), omx = to<RX>(omd);
        if (active) {
            const Spinor<R> r = SpinorIO<P>::template load<kVNT>(c.c, Vh, i);
            const Spinor<R> sv = SpinorIO<P>::template load<kVNT>(c.d, Vh, i);
            Spinor<R> q;
#pragma unroll
            for (int k = 0; k < 12; k++) q.c[k] = r.c[k] - al * sv.c[k];
            {
                Spinor<RX> xv = SpinorIO<XP>::template load<kVNT>(c.a, Vh, i);
                const Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    const cx<RX> pk = {(RX)pv.c[k].re, (RX)pv.c[k].im}, qk = {(RX)q.c[k].re, (RX)q.c[k].im};
                    xv.c[k] = xv.c[k] + alx * pk + omx * qk;
                }
                SpinorIO<XP>::template store<kVNT>(c.a, Vh, i, xv);
            }
            Spinor<R> y;
            {
                const Spinor<R> w = SpinorIO<P>::template load<kVNT>(c.e, Vh, i);
                const Spinor<R> zv = SpinorIO<P>::template load<kVNT>(c.f, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) y.c[k] = w.c[k] - al * zv.c[k];
            }
            Spinor<R> rn;
#pragma unroll
            for (int k = 0; k < 12; k++) rn.c[k] = q.c[k] - om * y.c[k];
            SpinorIO<P>::template store<kVNT>(c.c, Vh, i, rn);
            Spinor<R> wn;
            {
                const Spinor<R> t = SpinorIO<P>::template load<kVNT>(c.g, Vh, i);
                const Spinor<R> v = SpinorIO<P>::template load<kVNT>(c.h, Vh, i);
#pragma unroll
                for (int k = 0; k < 12; k++) wn.c[k] = y.c[k] - om * (t.c[k] - al * v.c[k]);
            }
            SpinorIO<P>::template store<kVNT>(c.e, Vh, i, wn);
            const Spinor<R> rt = SpinorIO<P>::template load<kVNT>(c.j, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                dot_acc(a[0 % NA], a[1 % NA], rt.c[k], rn.c[k]);
                dot_acc(a[2 % NA], a[3 % NA], rt.c[k], wn.c[k]);
                a[4 % NA] += norm2(rn.c[k]);
            }
        }
    } else if (OP == V_PIPE_FIX) {
        // x += alpha p with alpha from the pipelined loop's slot
        if (active) {
            const cx<RX> alx = to<RX>(ld_c(c.sc, S_RQ));
            Spinor<RX> xv = SpinorIO<XP>::template load<kVNT>(c.a, Vh, i);
            const Spinor<R> pv = SpinorIO<P>::template load<kVNT>(c.b, Vh, i);
#pragma unroll
            for (int k = 0; k < 12; k++) xv.c[k] = xv.c[k] + alx * cx<RX>{(RX)pv.c[k].re, (RX)pv.c[k].im};
            SpinorIO<XP>::template store<kVNT>(c.a, Vh, i, xv);
        }
    }
    if (N > 0) block_partials<NA>(a, c.partials, blocks_of(Vh, (int)blockDim.x), lb);
}

// ------------------------------------------------------------------ reduction stage 2
struct FinBatch {
    FinArgs f[kMaxSys];
};

template <int N> __global__ __launch_bounds__(kBlock) void k_finalize(FinBatch B) {
    const FinArgs &f = B.f[blockIdx.x];
    if (f.guard && *f.guard) return;
    __shared__ double sh[N][kWaves];
    double a[N];
#pragma unroll
    for (int k = 0; k < N; k++) a[k] = 0.0;
    // unrolled so that the loads of several partials are in flight at once;
    // the sums keep their order, so the result does not change
#pragma unroll 8
    for (int j = threadIdx.x; j < f.blocks; j += kBlock) {
#pragma unroll
        for (int k = 0; k < N; k++) a[k] += f.partials[(size_t)k * f.blocks + j];
    }
    block_fold<N>(a, sh);
    if (threadIdx.x != 0) return;
    double *sc = f.sc;
    int *fl = f.fl;
    const double a1 = a[1 % N], a2 = a[2 % N];
    switch (f.op) {
    case FIN_STORE:
        for (int k = 0; k < N; k++) f.result[k] = a[k];
        break;
    case FIN_INIT:
        sc[S_RHO0] = a[0];
        sc[S_RHO0 + 1] = 0.0;
        sc[S_TOL2] = f.tol2;
        fl[F_DONE] = DONE_NO;
        fl[F_ITERS] = 0;
        fl[F_STOPPH] = 0;
        break;
    case FIN_INNER_A: {
        const int it = fl[F_ITERS];
        const cx<double> al = cdiv(ld_c(sc, rho_slot(it)), ld_c(sc, S_RQ));
        sc[S_SS] = a[0];
        if (!finite_c(al) || !isfinite(a[0])) fl[F_DONE] = DONE_BREAK;
        else if (a[0] < sc[S_TOL2]) fl[F_DONE] = DONE_HALF;
        if (fl[F_DONE] != DONE_NO) fl[F_STOPPH] = 1;
        break;
    }
    case FIN_INNER_B: {
        const int it = fl[F_ITERS];
        const int nxt = rho_slot(it + 1);
        const double tt = sc[S_TT];
        const double tol2 = sc[S_TOL2];
        const cx<double> om = {sc[S_ST] / tt, -sc[S_ST + 1] / tt};
        sc[S_RR] = a[0];
        sc[nxt] = a1;
        sc[nxt + 1] = a2;
        fl[F_ITERS] = it + 1;
        if (!(tt > 0.0) || !finite_c(om) || !isfinite(a[0]) || (a1 == 0.0 && a2 == 0.0))
            fl[F_DONE] = (a[0] < tol2) ? DONE_FULL : DONE_BREAK;
        else if (a[0] < tol2)
            fl[F_DONE] = DONE_FULL;
        if (fl[F_DONE] != DONE_NO) fl[F_STOPPH] = 2;
        break;
    }
    case FIN_PIPE_INIT: {
        // alpha_0 = rho / <r~, w> (the D-hat reduction left <r~, w> in S_RQ)
        const cx<double> al = cdiv(ld_c(sc, S_RHO0), ld_c(sc, S_RQ));
        sc[S_RQ] = al.re;
        sc[S_RQ + 1] = al.im;
        sc[S_ST] = 1.0;
        sc[S_ST + 1] = 0.0;
        sc[S_RHO1] = 0.0;
        sc[S_RHO1 + 1] = 0.0;
        if (!finite_c(al)) {
            fl[F_DONE] = DONE_BREAK;
            fl[F_STOPPH] = 1;
        }
        break;
    }
    case FIN_PIPE_A: {
        const double yy = a[2 % N], qq = a[3 % N];
        const cx<double> om = {a[0] / yy, a[1 % N] / yy};
        sc[S_ST] = om.re;
        sc[S_ST + 1] = om.im;
        sc[S_AUX] = a[4 % N];
        sc[S_AUX + 1] = a[5 % N];
        sc[S_AUX + 2] = a[6 % N];
        sc[S_AUX + 3] = a[7 % N];
        sc[S_SS] = qq;
        sc[S_TT] = yy;
        if (isfinite(qq) && qq < sc[S_TOL2]) fl[F_DONE] = DONE_HALF;
        else if (!(yy > 0.0) || !finite_c(om) || !isfinite(qq)) fl[F_DONE] = DONE_BREAK;
        if (fl[F_DONE] != DONE_NO) fl[F_STOPPH] = 1;
        break;
    }
    case FIN_PIPE_B: {
        const int it = fl[F_ITERS];
        const cx<double> rho1 = {a[0], a[1 % N]}, rw = {a[2 % N], a[3 % N]};
        const double rr = a[4 % N];
        const cx<double> al = ld_c(sc, S_RQ), om = ld_c(sc, S_ST), rho0 = ld_c(sc, S_RHO0);
        const cx<double> be = cdiv(al, om) * cdiv(rho1, rho0);
        const cx<double> den = rw + be * ld_c(sc, S_AUX) - be * om * ld_c(sc, S_AUX + 2);
        const cx<double> aln = cdiv(rho1, den);
        sc[S_RHO0] = rho1.re;
        sc[S_RHO0 + 1] = rho1.im;
        sc[S_RHO1] = be.re;
        sc[S_RHO1 + 1] = be.im;
        sc[S_RQ] = aln.re;
        sc[S_RQ + 1] = aln.im;
        sc[S_RR] = rr;
        fl[F_ITERS] = it + 1;
        const double tol2 = sc[S_TOL2];
        if (!finite_c(be) || !finite_c(aln) || !isfinite(rr) || (rho1.re == 0.0 && rho1.im == 0.0))
            fl[F_DONE] = (rr < tol2) ? DONE_FULL : DONE_BREAK;
        else if (rr < tol2)
            fl[F_DONE] = DONE_FULL;
        if (fl[F_DONE] != DONE_NO) fl[F_STOPPH] = 2;
        break;
    }
    case FIN_OUTER_B: {
        const int nxt = rho_slot(f.iter + 1);
        sc[S_RR] = a[0];
        sc[nxt] = a1;
        sc[nxt + 1] = a2;
        break;
    }
    }
}

// algorithmic bytes of one op on one system (vectors read and written)
double vec_bytes(int op, int prec, int xprec, int Vh) {
    const double S = (double)spinor_site_bytes(prec) * Vh, X = (double)spinor_site_bytes(xprec) * Vh,
                 D = (double)spinor_site_bytes(P64) * Vh;
    switch (op) {
    case V_NORM2: return D;
    case V_SUB_NORM: return 3 * D;
    case V_AXPY: return 3 * D;
    case V_COPY: return 2 * D;
    case V_ZERO: return D;
    case V_GAMMA5: return 4 * D;
    case V_INNER_INIT: return D + 3 * S + X;
    case V_INNER_A: return 3 * S;
    case V_INNER_B: return 5 * S + 2 * X;
    case V_INNER_C: return 4 * S;
    case V_INNER_FIX: return S + 2 * X;
    case V_INNER_FINAL: return X + D;
    case V_OUTER_A: return 6 * D;
    case V_PIPE_INIT: return D + 6 * S + X;
    case V_PIPE_A: return 11 * S;
    case V_PIPE_B: return 10 * S + 2 * X;
    case V_PIPE_FIX: return S + 2 * X;
    case V_OUTER_B: return 7 * D;
    }
    return 0;
}

template <int OP, int P, int XP> void launch_op(hipStream_t s, const VecBatch &B, int blocks, int bs) {
    hipLaunchKernelGGL((k_vec<OP, P, XP>), dim3(blocks), dim3(bs), 0, s, B);
}

// the inner-loop ops exist for every storage precision; x is FP32 for the
// FP32 and FP16 inner loops and FP64 for the all-FP64 loop
template <int OP> void dispatch_inner(hipStream_t s, const VecBatch &B, int blocks, int bs, int prec) {
    if (prec == P64) launch_op<OP, P64, P64>(s, B, blocks, bs);
    else if (prec == P32) launch_op<OP, P32, P32>(s, B, blocks, bs);
    else launch_op<OP, P16, P32>(s, B, blocks, bs);
}

}  // namespace

int launch_fin_batch(hipStream_t s, const FinArgs *f, int n, int nvals) {
    if (n <= 0) return WC_OK;
    FinBatch B;
    for (int k = 0; k < n; k++) B.f[k] = f[k];
    switch (nvals) {
    case 1: hipLaunchKernelGGL(k_finalize<1>, dim3(n), dim3(kBlock), 0, s, B); break;
    case 2: hipLaunchKernelGGL(k_finalize<2>, dim3(n), dim3(kBlock), 0, s, B); break;
    case 3: hipLaunchKernelGGL(k_finalize<3>, dim3(n), dim3(kBlock), 0, s, B); break;
    case 5: hipLaunchKernelGGL(k_finalize<5>, dim3(n), dim3(kBlock), 0, s, B); break;
    case 8: hipLaunchKernelGGL(k_finalize<8>, dim3(n), dim3(kBlock), 0, s, B); break;
    default: return wc_fail(WC_EINVAL, "unsupported reduction width");
    }
    WC_HIP(hipGetLastError());
    return WC_OK;
}

int launch_vec_batch(hipStream_t s, wc_lattice *tlat, int op, int prec, const VecCall *calls, int n) {
    if (n <= 0) return WC_OK;
    if (n > kMaxSys) return wc_fail(WC_EINVAL, "too many systems in one batch");
    VecBatch B;
    B.h.S = n;
    B.h.interleave = 0;
    B.h.chunk = 0;
    B.h.off[0] = 0;
    const int xprec = prec == P64 ? P64 : P32;
    const int bs = launch_bs(calls[0].bs);
    if (!valid_block_size(bs)) return wc_fail(WC_EINVAL, "block size must be 64, 128 or 256");
    double bytes = 0;
    for (int k = 0; k < n; k++) {
        if (launch_bs(calls[k].bs) != bs) return wc_fail(WC_EINVAL, "batched vector calls must share the block size");
        B.c[k] = calls[k];
        B.h.off[k + 1] = B.h.off[k] + blocks_of(calls[k].Vh, bs);
        bytes += vec_bytes(op, prec, xprec, calls[k].Vh);
    }
    const int blocks = B.h.off[n];
    TimedLaunch t;
    if (tlat && tlat->timing) {
        timing_begin(tlat, KS_BLAS, bytes, t);
        t.iter = tlat->tag_iter;
        t.phase = tlat->tag_phase;
        for (int k = 0; k < n; k++)
            t.parts.push_back(TimedPart{{calls[k].guard ? calls[k].fl : nullptr},
                                        vec_bytes(op, prec, xprec, calls[k].Vh)});
    }
    switch (op) {
    case V_NORM2: launch_op<V_NORM2, P64, P64>(s, B, blocks, bs); break;
    case V_SUB_NORM: launch_op<V_SUB_NORM, P64, P64>(s, B, blocks, bs); break;
    case V_AXPY: launch_op<V_AXPY, P64, P64>(s, B, blocks, bs); break;
    case V_COPY: launch_op<V_COPY, P64, P64>(s, B, blocks, bs); break;
    case V_ZERO: launch_op<V_ZERO, P64, P64>(s, B, blocks, bs); break;
    case V_GAMMA5: launch_op<V_GAMMA5, P64, P64>(s, B, blocks, bs); break;
    case V_INNER_INIT: dispatch_inner<V_INNER_INIT>(s, B, blocks, bs, prec); break;
    case V_INNER_A: dispatch_inner<V_INNER_A>(s, B, blocks, bs, prec); break;
    case V_INNER_B: dispatch_inner<V_INNER_B>(s, B, blocks, bs, prec); break;
    case V_INNER_C: dispatch_inner<V_INNER_C>(s, B, blocks, bs, prec); break;
    case V_INNER_FIX: dispatch_inner<V_INNER_FIX>(s, B, blocks, bs, prec); break;
    case V_INNER_FINAL: dispatch_inner<V_INNER_FINAL>(s, B, blocks, bs, prec); break;
    case V_PIPE_INIT: dispatch_inner<V_PIPE_INIT>(s, B, blocks, bs, prec); break;
    case V_PIPE_A: dispatch_inner<V_PIPE_A>(s, B, blocks, bs, prec); break;
    case V_PIPE_B: dispatch_inner<V_PIPE_B>(s, B, blocks, bs, prec); break;
    case V_PIPE_FIX: dispatch_inner<V_PIPE_FIX>(s, B, blocks, bs, prec); break;
    case V_OUTER_A: launch_op<V_OUTER_A, P64, P64>(s, B, blocks, bs); break;
    case V_OUTER_B: launch_op<V_OUTER_B, P64, P64>(s, B, blocks, bs); break;
    default: return wc_fail(WC_EINVAL, "unknown vector op");
    }
    WC_HIP(hipGetLastError());
    if (tlat && tlat->timing) timing_end(tlat, t);

    // second stage of the reductions
    const int N = red_count(op);
    if (N == 0) return WC_OK;
    FinArgs f[kMaxSys];
    for (int k = 0; k < n; k++) {
        const VecCall &c = calls[k];
        FinArgs &a = f[k];
        a = FinArgs{};
        a.blocks = blocks_of(c.Vh, bs);
        a.partials = c.partials;
        a.result = c.result;
        a.sc = c.sc;
        a.fl = c.fl;
        a.guard = c.guard ? c.fl : nullptr;
        a.iter = c.iter;
        a.tol2 = c.tol2;
        a.op = (op == V_INNER_INIT || op == V_PIPE_INIT) ? FIN_INIT
             : (op == V_INNER_A)                          ? FIN_INNER_A
             : (op == V_INNER_B)                          ? FIN_INNER_B
             : (op == V_OUTER_B)                          ? FIN_OUTER_B
             : (op == V_PIPE_A)                           ? FIN_PIPE_A
             : (op == V_PIPE_B)                           ? FIN_PIPE_B
                                                          : FIN_STORE;
        if (op == V_OUTER_A) a.result = c.sc + S_RR;
    }
    return launch_fin_batch(s, f, n, N);
}
