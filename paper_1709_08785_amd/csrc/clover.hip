// Clover term (Sec. II-A; packed as two 6x6 Hermitian blocks as in Sec. III-A)
// and its inverse, built once per (links, kappa, c_SW) in FP64.
//
//   Q_{mu nu}(n) = sum of the four counter-clockwise plaquettes at n
//   Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dagger) / 8
//   F = 1 - kappa c_SW sum_{mu<nu} g_mu g_nu (x) Fhat_{mu nu}
//
// In the Dirac representation g_k g_l = diag(s_k s_l, s_k s_l) and
// g_k g_t = [[0, i s_k], [i s_k, 0]], so F = [[A, B], [B, A]] with
//   A = 1 - kappa c_SW [ i s_z (x) Fhat_xy - i s_y (x) Fhat_xz + i s_x (x) Fhat_yz ]
//   B = -kappa c_SW i [ s_x (x) Fhat_xt + s_y (x) Fhat_yt + s_z (x) Fhat_zt ].
// F commutes with g5 = -[[0, 1], [1, 0]]; on the g5 = +1 space (u, -u) it acts
// as A - B and on the g5 = -1 space (u, u) as A + B.  Stored per site are
// M1 = (A - B)/2 and M2 = (A + B)/2 (and the same for the inverses), which
// is what the Dirac-basis epilogue of the stencil consumes.
#include "reduce.hpp"

namespace {

using C = cx<double>;

struct M3 {
    C m[9];
};

__device__ __forceinline__ M3 m3mul(const M3 &a, const M3 &b) {
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

// a * b^dagger
__device__ __forceinline__ M3 m3mul_d(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) cmac(s, a.m[3 * i + k], conjx(b.m[3 * j + k]));
            c.m[3 * i + j] = s;
        }
    return c;
}

// a^dagger * b
__device__ __forceinline__ M3 m3dmul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            C s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) cmac(s, conjx(a.m[3 * k + i]), b.m[3 * k + j]);
            c.m[3 * i + j] = s;
        }
    return c;
}

struct LinkView {
    Geom g;
    const double2 *l64;  // tiled FP64 link slabs [mu][parity]

    __device__ M3 at(int mu, int x, int y, int z, int t) const {
        const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
        x = (x + L0) % L0;
        y = (y + L1) % L1;
        z = (z + L2) % L2;
        t = (t + L3) % L3;
        const int par = (x + y + z + t) & 1;
        const int n = x + L0 * (y + L1 * (z + L2 * t));
        const int i = n >> 1;
        const char *slab = (const char *)l64 + (size_t)(2 * mu + par) * link_slab_bytes(P64, g.Vh);
        M3 u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            double2 v = *tp<double2, 144>(slab, i, 16 * k);
            u.m[k] = {v.x, v.y};
        }
        return u;
    }
};

// Fhat_{mu nu}(n) = (Q - Q^dagger)/8 from the four counter-clockwise leaves
__device__ M3 fhat(const LinkView &lv, const int c[4], int mu, int nu) {
    int e[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    const int *a = e[mu], *b = e[nu];
    auto U = [&](int d, int sa, int sb) {
        return lv.at(d, c[0] + sa * a[0] + sb * b[0], c[1] + sa * a[1] + sb * b[1], c[2] + sa * a[2] + sb * b[2],
                     c[3] + sa * a[3] + sb * b[3]);
    };
    M3 q, t;
    // U_mu(n) U_nu(n+mu) U_mu(n+nu)^dag U_nu(n)^dag
    t = m3mul(U(mu, 0, 0), U(nu, 1, 0));
    t = m3mul_d(t, U(mu, 0, 1));
    q = m3mul_d(t, U(nu, 0, 0));
    // U_nu(n) U_mu(n+nu-mu)^dag U_nu(n-mu)^dag U_mu(n-mu)
    t = m3mul_d(U(nu, 0, 0), U(mu, -1, 1));
    t = m3mul_d(t, U(nu, -1, 0));
    t = m3mul(t, U(mu, -1, 0));
#pragma unroll
    for (int k = 0; k < 9; k++) q.m[k] = q.m[k] + t.m[k];
    // U_mu(n-mu)^dag U_nu(n-mu-nu)^dag U_mu(n-mu-nu) U_nu(n-nu)
    {
        M3 a1 = U(mu, -1, 0), b1 = U(nu, -1, -1);
        M3 ab;  // a1^dag b1^dag = (b1 a1)^dag
        M3 ba = m3mul(b1, a1);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) ab.m[3 * i + j] = conjx(ba.m[3 * j + i]);
        t = m3mul(ab, U(mu, -1, -1));
        t = m3mul(t, U(nu, 0, -1));
    }
#pragma unroll
    for (int k = 0; k < 9; k++) q.m[k] = q.m[k] + t.m[k];
    // U_nu(n-nu)^dag U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^dag
    t = m3dmul(U(nu, 0, -1), U(mu, 0, -1));
    t = m3mul(t, U(nu, 1, -1));
    t = m3mul_d(t, U(mu, 0, 0));
#pragma unroll
    for (int k = 0; k < 9; k++) q.m[k] = q.m[k] + t.m[k];
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const C a0 = q.m[3 * i + j], b0 = conjx(q.m[3 * j + i]);
            f.m[3 * i + j] = 0.125 * (a0 - b0);
        }
    return f;
}

// M += coef * (S (x) F), S a 2x2 complex spin matrix, F a 3x3 colour matrix
__device__ __forceinline__ void add_kron(C (&M)[6][6], C coef, const C (&S)[2][2], const M3 &F) {
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int sp = 0; sp < 2; sp++) {
            const C cs = coef * S[s][sp];
            if (cs.re == 0.0 && cs.im == 0.0) continue;
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) cmac(M[3 * s + a][3 * sp + b], cs, F.m[3 * a + b]);
        }
}

// 6x6 inverse by Gauss-Jordan elimination without row exchanges.  For a
// Hermitian matrix the pivots met on the way are the ratios of successive
// leading principal minors, so they are all real and positive exactly when the
// matrix is positive definite; the return value counts the pivots that are
// not (non-positive or non-finite real part), 0 for a positive definite block,
// for which elimination without exchanges is stable.
__device__ int inv6(const C (&A)[6][6], C (&Ai)[6][6]) {
    C a[6][12];
    int bad = 0;
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) {
            a[i][j] = A[i][j];
            a[i][6 + j] = (i == j) ? C{1, 0} : C{0, 0};
        }
    for (int col = 0; col < 6; col++) {
        const C d = a[col][col];
        if (!(d.re > 0.0) || !isfinite(d.re) || !isfinite(d.im)) bad++;
        const double dn = d.re * d.re + d.im * d.im;
        const C dinv = {d.re / dn, -d.im / dn};
        for (int j = 0; j < 12; j++) a[col][j] = a[col][j] * dinv;
        for (int r = 0; r < 6; r++) {
            if (r == col) continue;
            const C f = a[r][col];
            for (int j = 0; j < 12; j++) a[r][j] = a[r][j] - f * a[col][j];
        }
    }
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) Ai[i][j] = a[i][6 + j];
    return bad;
}

// pack the Hermitian part of M (times `scale`) into 6 reals + 15 complex
__device__ void pack_herm(const C (&M)[6][6], double scale, double (&f)[36]) {
    for (int k = 0; k < 6; k++) f[k] = scale * M[k][k].re;
    int k = 0;
    for (int i = 0; i < 6; i++)
        for (int j = i + 1; j < 6; j++) {
            // symmetrise: (M_ij + conj(M_ji)) / 2
            f[6 + 2 * k] = scale * 0.5 * (M[i][j].re + M[j][i].re);
            f[7 + 2 * k] = scale * 0.5 * (M[i][j].im - M[j][i].im);
            k++;
        }
}

struct CloverOut {
    char *f64, *i64;  // tiled slabs [parity], 576 B/site
    char *f32, *i32;  // 288 B/site
    char *f16, *i16;  // 148 B/site
};

__device__ void store_block_set(const CloverOut &o, bool inv, int par, int Vh, int i, const double (&f)[2][36]) {
    char *d64 = (inv ? o.i64 : o.f64) + (size_t)par * clover_slab_bytes(P64, Vh);
    char *d32 = (inv ? o.i32 : o.f32) + (size_t)par * clover_slab_bytes(P32, Vh);
    char *d16 = (inv ? o.i16 : o.f16) + (size_t)par * clover_slab_bytes(P16, Vh);
    double mx = 0.0;
    for (int b = 0; b < 2; b++) {
        for (int k = 0; k < 18; k++)
            *tp<double2, 576>(d64, i, 16 * (18 * b + k)) = make_double2(f[b][2 * k], f[b][2 * k + 1]);
        for (int k = 0; k < 9; k++)
            *tp<float4, 288>(d32, i, 16 * (9 * b + k)) = make_float4((float)f[b][4 * k], (float)f[b][4 * k + 1],
                                                                     (float)f[b][4 * k + 2], (float)f[b][4 * k + 3]);
        for (int k = 0; k < 36; k++) mx = fmax(mx, fabs(f[b][k]));
    }
    const float s = (float)mx;
    const float inv_s = s > 0.f ? 1.0f / s : 0.f;
    for (int b = 0; b < 2; b++) {
        uint32_t w[18];
        for (int k = 0; k < 18; k++) w[k] = f2h((float)f[b][2 * k] * inv_s, (float)f[b][2 * k + 1] * inv_s);
        for (int k = 0; k < 4; k++)
            *tp<uint4, 148>(d16, i, 72 * b + 16 * k) = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
        *tp<uint2, 148>(d16, i, 72 * b + 64) = make_uint2(w[16], w[17]);
    }
    *tp<float, 148>(d16, i, 144) = s;
}

// bad_blocks: device counter of the 6x6 blocks (two per site) that are not
// positive definite, incremented by the kernel
__global__ __launch_bounds__(64) void k_build_clover(Geom g, const double2 *l64, CloverOut o, double kappa,
                                                     double csw, unsigned *bad_blocks) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    const SiteCoord sc = eo_coords(g, i, par);
    const int c[4] = {sc.x, sc.y, sc.z, sc.t};
    LinkView lv{g, l64};

    const C I1 = {0, 1}, ONE = {1, 0}, ZERO = {0, 0};
    // i s_z, -i s_y, i s_x, and the Pauli matrices themselves
    const C isz[2][2] = {{I1, ZERO}, {ZERO, -I1}};
    const C misy[2][2] = {{ZERO, -ONE}, {ONE, ZERO}};
    const C isx[2][2] = {{ZERO, I1}, {I1, ZERO}};
    const C sx[2][2] = {{ZERO, ONE}, {ONE, ZERO}};
    const C sy[2][2] = {{ZERO, -I1}, {I1, ZERO}};
    const C sz[2][2] = {{ONE, ZERO}, {ZERO, -ONE}};

    C A[6][6], B[6][6];
    for (int r = 0; r < 6; r++)
        for (int s = 0; s < 6; s++) {
            A[r][s] = (r == s) ? ONE : ZERO;
            B[r][s] = ZERO;
        }
    const double kc = kappa * csw;
    const C mkc = {-kc, 0.0};
    add_kron(A, mkc, isz, fhat(lv, c, 0, 1));
    add_kron(A, mkc, misy, fhat(lv, c, 0, 2));
    add_kron(A, mkc, isx, fhat(lv, c, 1, 2));
    const C mikc = {0.0, -kc};
    add_kron(B, mikc, sx, fhat(lv, c, 0, 3));
    add_kron(B, mikc, sy, fhat(lv, c, 1, 3));
    add_kron(B, mikc, sz, fhat(lv, c, 2, 3));

    C M[6][6], Mi[6][6];
    double fF[2][36], fI[2][36];
    unsigned nbad = 0;
    // block 0: A - B (g5 = +1), block 1: A + B (g5 = -1); store halves
    for (int blk = 0; blk < 2; blk++) {
        const double sgn = blk == 0 ? -1.0 : 1.0;
        for (int r = 0; r < 6; r++)
            for (int s = 0; s < 6; s++) M[r][s] = A[r][s] + sgn * B[r][s];
        nbad += inv6(M, Mi) != 0;
        pack_herm(M, 0.5, fF[blk]);
        pack_herm(Mi, 0.5, fI[blk]);
    }
    store_block_set(o, false, par, g.Vh, i, fF);
    store_block_set(o, true, par, g.Vh, i, fI);
    if (nbad) atomicAdd(bad_blocks, nbad);
}

}  // namespace

int launch_build_clover(wc_lattice *lat, double kappa, double csw, unsigned *bad_blocks) {
    CloverOut o;
    o.f64 = (char *)lat->clov[P64];
    o.i64 = (char *)lat->clovinv[P64];
    o.f32 = (char *)lat->clov[P32];
    o.i32 = (char *)lat->clovinv[P32];
    o.f16 = (char *)lat->clov[P16];
    o.i16 = (char *)lat->clovinv[P16];
    dim3 grid((lat->Vh + 63) / 64, 2);
    hipLaunchKernelGGL(k_build_clover, grid, dim3(64), 0, lat->stream, lat->g, (const double2 *)lat->links[P64], o,
                       kappa, csw, bad_blocks);
    WC_HIP(hipGetLastError());
    return WC_OK;
}
