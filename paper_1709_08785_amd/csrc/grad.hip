// Gradient of a solve with respect to the gauge links.
//
// For L = Re<eta, D^-1 b> (or any real loss with dL = Re<eta, dx>) the adjoint
// solve gives lam = D^-dagger eta = g5 D^-1 g5 eta (D is gamma5-Hermitian),
// and dL = -Re<lam, (dD) x> with dD = dF - kappa dH (eq. 3).  The gradient G
// of a link (torch convention: dL = Re sum conj(G_ab) dU_ab) has
//
//   hopping part (eq. 4), link U_mu(m):
//     G += kappa sum_alpha [ lam(m)_alpha ((1 - g_mu) x(m+mu))_alpha^dagger
//                          + ((1 + g_mu) x(m))_alpha lam(m+mu)_alpha^dagger ]
//   clover part: per site n and plane mu<nu,
//     M_ab = sum conj(lam_{alpha a}) (g_mu g_nu)_{alpha beta} x_{beta b},  N = M - M^dagger,
//     and a leaf f1 f2 f3 f4 of Q_{mu nu}(n) whose factor k is the link contributes
//     (kappa c_SW / 8) (B N^T A)^dagger (or B N^T A when the factor is daggered),
//     A = f1..f_{k-1}, B = f_{k+1}..f4.
//
// The clover part is a gather: one thread per link visits the 8 leaf slots of
// each of the 3 planes that contain it, so no two threads write the same
// link and the result is deterministic.
#include "reduce.hpp"

namespace {

using C = cx<double>;
using M3 = Mat3<double>;

__device__ __forceinline__ M3 mmul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) cmac(s, a.m[3 * i + k], b.m[3 * k + j]);
            c.m[3 * i + j] = s;
        }
    return c;
}
__device__ __forceinline__ M3 mdag(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.m[3 * i + j] = conjx(a.m[3 * j + i]);
    return c;
}
__device__ __forceinline__ M3 mtrans(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.m[3 * i + j] = a.m[3 * j + i];
    return c;
}
__device__ __forceinline__ M3 meye() {
    M3 c;
#pragma unroll
    for (int k = 0; k < 9; k++) c.m[k] = {(k % 4 == 0) ? 1.0 : 0.0, 0.0};
    return c;
}

// (1 - s g_mu) psi for s = +1, (1 + g_mu) psi for s = -1, Dirac representation
__device__ void one_minus_gamma(int mu, bool minus, const Spinor<double> &p, Spinor<double> &o) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const C p0 = p.c[a], p1 = p.c[3 + a], p2 = p.c[6 + a], p3 = p.c[9 + a];
        C o0, o1, o2, o3;
        if (mu == 0) {
            if (minus) { o0 = p0 + mul_i(p3); o1 = p1 + mul_i(p2); o2 = p2 - mul_i(p1); o3 = p3 - mul_i(p0); }
            else       { o0 = p0 - mul_i(p3); o1 = p1 - mul_i(p2); o2 = p2 + mul_i(p1); o3 = p3 + mul_i(p0); }
        } else if (mu == 1) {
            if (minus) { o0 = p0 + p3; o1 = p1 - p2; o2 = p2 - p1; o3 = p3 + p0; }
            else       { o0 = p0 - p3; o1 = p1 + p2; o2 = p2 + p1; o3 = p3 - p0; }
        } else if (mu == 2) {
            if (minus) { o0 = p0 + mul_i(p2); o1 = p1 - mul_i(p3); o2 = p2 - mul_i(p0); o3 = p3 + mul_i(p1); }
            else       { o0 = p0 - mul_i(p2); o1 = p1 + mul_i(p3); o2 = p2 + mul_i(p0); o3 = p3 - mul_i(p1); }
        } else {
            const C z = {0, 0};
            if (minus) { o0 = z; o1 = z; o2 = p2 + p2; o3 = p3 + p3; }
            else       { o0 = p0 + p0; o1 = p1 + p1; o2 = z; o3 = z; }
        }
        o.c[a] = o0;
        o.c[3 + a] = o1;
        o.c[6 + a] = o2;
        o.c[9 + a] = o3;
    }
}

// (g_mu g_nu) psi for plane p = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ void gamma_pair(int plane, const Spinor<double> &p, Spinor<double> &o) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const C p0 = p.c[a], p1 = p.c[3 + a], p2 = p.c[6 + a], p3 = p.c[9 + a];
        C o0, o1, o2, o3;
        switch (plane) {
        case 0: o0 = mul_i(p0); o1 = mul_mi(p1); o2 = mul_i(p2); o3 = mul_mi(p3); break;   // i s_z
        case 1: o0 = -p1; o1 = p0; o2 = -p3; o3 = p2; break;                               // -i s_y
        case 2: o0 = mul_i(p3); o1 = mul_i(p2); o2 = mul_i(p1); o3 = mul_i(p0); break;     // off-diag i s_x
        case 3: o0 = mul_i(p1); o1 = mul_i(p0); o2 = mul_i(p3); o3 = mul_i(p2); break;     // i s_x
        case 4: o0 = p3; o1 = -p2; o2 = p1; o3 = -p0; break;                               // off-diag i s_y
        default: o0 = mul_i(p2); o1 = mul_mi(p3); o2 = mul_i(p0); o3 = mul_mi(p1); break;  // off-diag i s_z
        }
        o.c[a] = o0;
        o.c[3 + a] = o1;
        o.c[6 + a] = o2;
        o.c[9 + a] = o3;
    }
}

__device__ __forceinline__ int plane_of(int mu, int nu) {
    // mu < nu
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}

// canonical gradient slot of link (mu, site n) -> 9 complex128
__device__ __forceinline__ double2 *gslot(double2 *G, const Geom &g, int mu, const SiteCoord &c) {
    const size_t n = (size_t)c.x + (size_t)g.L[0] * c.row;
    return G + ((size_t)mu * 2 * g.Vh + n) * 9;
}

// hopping part; overwrites G
__global__ __launch_bounds__(kBlock) void k_grad_hop(Geom g, const char *lam, const char *x, size_t sb, double2 *G,
                                                     double kappa) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int slab = blockIdx.y;  // 2 mu + parity
    if (i >= g.Vh) return;
    const int mu = slab >> 1, par = slab & 1;
    const SiteCoord c = eo_coords(g, i, par);
    const int np = eo_neighbour(g, c, mu, +1);
    const Spinor<double> lm = SpinorIO<P64>::load(lam + par * sb, g.Vh, i);
    const Spinor<double> lp = SpinorIO<P64>::load(lam + (1 - par) * sb, g.Vh, np);
    const Spinor<double> xm = SpinorIO<P64>::load(x + par * sb, g.Vh, i);
    const Spinor<double> xp = SpinorIO<P64>::load(x + (1 - par) * sb, g.Vh, np);
    Spinor<double> y, z;
    one_minus_gamma(mu, true, xp, y);
    one_minus_gamma(mu, false, xm, z);
    double2 *out = gslot(G, g, mu, c);
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            C s = {0, 0};
#pragma unroll
            for (int al = 0; al < 4; al++) {
                cmac(s, lm.c[3 * al + a], conjx(y.c[3 * al + b]));
                cmac(s, z.c[3 * al + a], conjx(lp.c[3 * al + b]));
            }
            out[3 * a + b] = make_double2(kappa * s.re, kappa * s.im);
        }
}

// N_{mu nu}(n) = M - M^dagger for the 6 planes, FP64 [plane][parity][9][Vh] double2
__global__ __launch_bounds__(kBlock) void k_grad_N(Geom g, const char *lam, const char *x, size_t sb, double2 *N) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    const Spinor<double> l = SpinorIO<P64>::load(lam + par * sb, g.Vh, i);
    const Spinor<double> xv = SpinorIO<P64>::load(x + par * sb, g.Vh, i);
    for (int p = 0; p < 6; p++) {
        Spinor<double> y;
        gamma_pair(p, xv, y);
        C M[9];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                C s = {0, 0};
#pragma unroll
                for (int al = 0; al < 4; al++) cmacc(s, l.c[3 * al + a], y.c[3 * al + b]);
                M[3 * a + b] = s;
            }
        double2 *o = N + (size_t)(2 * p + par) * 9 * g.Vh;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const C v = M[3 * a + b] - conjx(M[3 * b + a]);
                o[(size_t)(3 * a + b) * g.Vh + i] = make_double2(v.re, v.im);
            }
    }
}

// the four counter-clockwise leaves of Q_{mu nu}(n), factor by factor:
// {0: mu-link / 1: nu-link, root offset along mu, root offset along nu, daggered}
__constant__ int kLeafG[4][4][4] = {
    // U_mu(n) U_nu(n+mu) U_mu(n+nu)^dag U_nu(n)^dag
    {{0, 0, 0, 0}, {1, 1, 0, 0}, {0, 0, 1, 1}, {1, 0, 0, 1}},
    // U_nu(n) U_mu(n+nu-mu)^dag U_nu(n-mu)^dag U_mu(n-mu)
    {{1, 0, 0, 0}, {0, -1, 1, 1}, {1, -1, 0, 1}, {0, -1, 0, 0}},
    // U_mu(n-mu)^dag U_nu(n-mu-nu)^dag U_mu(n-mu-nu) U_nu(n-nu)
    {{0, -1, 0, 1}, {1, -1, -1, 1}, {0, -1, -1, 0}, {1, 0, -1, 0}},
    // U_nu(n-nu)^dag U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^dag
    {{1, 0, -1, 1}, {0, 0, -1, 0}, {1, 1, -1, 0}, {0, 0, 0, 1}},
};

// clover part; adds into G
__global__ __launch_bounds__(64) void k_grad_clover(Geom g, const double2 *l64, const double2 *N, double2 *G,
                                                    double fac) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int slab = blockIdx.y;  // 2 d + parity
    if (i >= g.Vh) return;
    const int d = slab >> 1, par = slab & 1;
    const SiteCoord c = eo_coords(g, i, par);
    const int cm[4] = {c.x, c.y, c.z, c.t};
    M3 acc;
#pragma unroll
    for (int k = 0; k < 9; k++) acc.m[k] = {0, 0};
    for (int e = 0; e < 4; e++) {
        if (e == d) continue;
        const int mu = d < e ? d : e, nu = d < e ? e : d;
        const int role = (d == mu) ? 0 : 1;
        const int p = plane_of(mu, nu);
        for (int lf = 0; lf < 4; lf++) {
            for (int k = 0; k < 4; k++) {
                if (kLeafG[lf][k][0] != role) continue;
                // leaf site n = m - offset of factor k
                int n[4] = {cm[0], cm[1], cm[2], cm[3]};
                n[mu] -= kLeafG[lf][k][1];
                n[nu] -= kLeafG[lf][k][2];
                M3 A = meye(), B = meye();
                for (int j = 0; j < 4; j++) {
                    if (j == k) continue;
                    int s[4] = {n[0], n[1], n[2], n[3]};
                    s[mu] += kLeafG[lf][j][1];
                    s[nu] += kLeafG[lf][j][2];
                    const int dir = kLeafG[lf][j][0] ? nu : mu;
                    M3 f = link64(l64, g, dir, site_ref(g, s[0], s[1], s[2], s[3]));
                    if (kLeafG[lf][j][3]) f = mdag(f);
                    if (j < k) A = mmul(A, f);
                    else B = mmul(B, f);
                }
                const SiteRef sn = site_ref(g, n[0], n[1], n[2], n[3]);
                M3 Nm;
                const double2 *np_ = N + (size_t)(2 * p + sn.par) * 9 * g.Vh;
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    const double2 v = np_[(size_t)q * g.Vh + sn.i];
                    Nm.m[q] = {v.x, v.y};
                }
                const M3 P = mmul(mmul(B, mtrans(Nm)), A);
                const M3 add = kLeafG[lf][k][3] ? P : mdag(P);
#pragma unroll
                for (int q = 0; q < 9; q++) acc.m[q] = acc.m[q] + add.m[q];
            }
        }
    }
    double2 *out = gslot(G, g, d, c);
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const double2 v = out[q];
        out[q] = make_double2(v.x + fac * acc.m[q].re, v.y + fac * acc.m[q].im);
    }
}

}  // namespace

int launch_link_grad(wc_lattice *lat, const void *lam_eo, const void *x_eo, void *G, void *Nbuf, double kappa,
                     double csw, bool clover) {
    const size_t sb = spinor_bytes(P64, lat->Vh);
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 8);
    hipLaunchKernelGGL(k_grad_hop, grid, dim3(kBlock), 0, lat->stream, lat->g, (const char *)lam_eo,
                       (const char *)x_eo, sb, (double2 *)G, kappa);
    WC_HIP(hipGetLastError());
    if (!clover) return WC_OK;
    dim3 gridN((lat->Vh + kBlock - 1) / kBlock, 2);
    hipLaunchKernelGGL(k_grad_N, gridN, dim3(kBlock), 0, lat->stream, lat->g, (const char *)lam_eo,
                       (const char *)x_eo, sb, (double2 *)Nbuf);
    WC_HIP(hipGetLastError());
    dim3 gridC((lat->Vh + 63) / 64, 8);
    hipLaunchKernelGGL(k_grad_clover, gridC, dim3(64), 0, lat->stream, lat->g, (const double2 *)lat->links[P64],
                       (const double2 *)Nbuf, (double2 *)G, kappa * csw / 8.0);
    WC_HIP(hipGetLastError());
    return WC_OK;
}
