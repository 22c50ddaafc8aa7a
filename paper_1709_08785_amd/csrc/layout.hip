// Layout kernels: canonical complex128 fields <-> the site-tiled
// even-odd layout, and the per-precision copies of the gauge links.
#include "reduce.hpp"

namespace {

// |third column - conj(col0 x col1)| of one link, largest entry, in FP64: how
// far the link is from what the two-column forms rebuild
__device__ __forceinline__ float recon12_error(const double2 (&m)[9]) {
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
        // row r of conj(c0 x c1): conj(c0[r1] c1[r2] - c0[r2] c1[r1])
        const double2 a = m[3 * r1], b = m[3 * r2 + 1], c = m[3 * r2], d = m[3 * r1 + 1];
        const double re = (a.x * b.x - a.y * b.y) - (c.x * d.x - c.y * d.y);
        const double im = -((a.x * b.y + a.y * b.x) - (c.x * d.y + c.y * d.x));
        const double2 t = m[3 * r + 2];
        e = fmax(e, sqrt((t.x - re) * (t.x - re) + (t.y - im) * (t.y - im)));
    }
    return (float)e;
}

__global__ __launch_bounds__(kBlock) void k_load_links(Geom g, const double2 *U, double2 *l64, float4 *l32,
                                                       char *l16, unsigned *err_bits) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int slab = blockIdx.y;  // 2 mu + parity
    float err = 0.f;
    if (i < g.Vh) {
        const int mu = slab >> 1, par = slab & 1;
        const SiteCoord c = eo_coords(g, i, par);
        const size_t n = (size_t)c.x + (size_t)g.L[0] * c.row;
        const size_t V = (size_t)2 * g.Vh;
        const double2 *src = U + ((size_t)mu * V + n) * 9;
        double2 m[9];
    #pragma unroll
        for (int k = 0; k < 9; k++) m[k] = src[k];
        char *d64 = (char *)l64 + (size_t)slab * link_slab_bytes(P64, g.Vh);
    #pragma unroll
        for (int k = 0; k < 9; k++) *tp<double2, 144>(d64, i, 16 * k) = m[k];
        // columns 0 and 1: U00 U10 | U20 U01 | U11 U21
        char *d32 = (char *)l32 + (size_t)slab * link_slab_bytes(P32, g.Vh);
        *tp<float4, 48>(d32, i, 0) = make_float4((float)m[0].x, (float)m[0].y, (float)m[3].x, (float)m[3].y);
        *tp<float4, 48>(d32, i, 16) = make_float4((float)m[6].x, (float)m[6].y, (float)m[1].x, (float)m[1].y);
        *tp<float4, 48>(d32, i, 32) = make_float4((float)m[4].x, (float)m[4].y, (float)m[7].x, (float)m[7].y);
        char *b16 = l16 + (size_t)slab * link_slab_bytes(P16, g.Vh);
        uint4 u;
        u.x = f2h((float)m[0].x, (float)m[0].y);
        u.y = f2h((float)m[3].x, (float)m[3].y);
        u.z = f2h((float)m[6].x, (float)m[6].y);
        u.w = f2h((float)m[1].x, (float)m[1].y);
        *tp<uint4, 24>(b16, i, 0) = u;
        *tp<uint2, 24>(b16, i, 16) = make_uint2(f2h((float)m[4].x, (float)m[4].y), f2h((float)m[7].x, (float)m[7].y));
        bool finite = true;
    #pragma unroll
        for (int k = 0; k < 9; k++) finite = finite && isfinite(m[k].x) && isfinite(m[k].y);
        // a non-finite entry posts +inf, which orders above every finite error
        // (a NaN would be dropped by the max below)
        err = finite ? recon12_error(m) : INFINITY;
    }
    // non-negative floats order like their bits
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) err = fmaxf(err, __shfl_xor(err, off));
    if ((threadIdx.x & 63) == 0) atomicMax(err_bits, __float_as_uint(err));
}

// the full FP32 copy of the FP64 links (row-major, four float4 and a float2)
__global__ __launch_bounds__(kBlock) void k_links_full32(Geom g, const char *l64, char *l18) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int slab = blockIdx.y;  // 2 mu + parity
    if (i >= g.Vh) return;
    const char *src = l64 + (size_t)slab * link_slab_bytes(P64, g.Vh);
    double2 m[9];
#pragma unroll
    for (int k = 0; k < 9; k++) m[k] = *tp<double2, 144>(src, i, 16 * k);
    char *d = l18 + (size_t)slab * link18_slab_bytes(g.Vh);
#pragma unroll
    for (int k = 0; k < 4; k++)
        *tp<float4, 72>(d, i, 16 * k) = make_float4((float)m[2 * k].x, (float)m[2 * k].y, (float)m[2 * k + 1].x,
                                                    (float)m[2 * k + 1].y);
    *tp<float2, 72>(d, i, 64) = make_float2((float)m[8].x, (float)m[8].y);
}

// reconstruct-8 copy of the FP64 links and the smallest N = |U01|^2 + |U02|^2
// (as FP32 bits, which order like the non-negative values they encode)
__global__ __launch_bounds__(kBlock) void k_links_recon8(Geom g, const char *l64, char *l8, unsigned *min_bits) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int slab = blockIdx.y;  // 2 mu + parity
    float n32 = 3.0e38f;
    if (i < g.Vh) {
        const char *src = l64 + (size_t)slab * link_slab_bytes(P64, g.Vh);
        double2 m[9];
#pragma unroll
        for (int k = 0; k < 9; k++) m[k] = *tp<double2, 144>(src, i, 16 * k);
        const double2 a2 = m[1], a3 = m[2], b1 = m[3], c1 = m[6];
        const bool swap = (b1.x * b1.x + b1.y * b1.y) > (c1.x * c1.x + c1.y * c1.y);
        const double2 y = swap ? c1 : b1, z = swap ? b1 : c1;
        const double ta = atan2(m[0].y, m[0].x) / M_PI;
        double tz = atan2(z.y, z.x) / M_PI;
        if (tz < 0.0) tz += 2.0;  // [0, 2]: the sign bit is free for the flag
        char *d = l8 + (size_t)slab * link8_slab_bytes(g.Vh);
        const float4 p0 = make_float4((float)a2.x, (float)a2.y, (float)a3.x, (float)a3.y);
        *tp<float4, 32>(d, i, 0) = p0;
        const float tzf = (float)tz;
        *tp<float4, 32>(d, i, 16) = make_float4((float)y.x, (float)y.y, (float)ta, swap ? -tzf : tzf);
        n32 = p0.x * p0.x + p0.y * p0.y + p0.z * p0.z + p0.w * p0.w;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n32 = fminf(n32, __shfl_xor(n32, off));
    if ((threadIdx.x & 63) == 0) atomicMin(min_bits, __float_as_uint(n32));
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_pack(Geom g, char *eo, const double2 *canon, size_t slab_bytes) {
    using R = typename Real<P>::T;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    const SiteCoord c = eo_coords(g, i, par);
    const size_t n = (size_t)c.x + (size_t)g.L[0] * c.row;
    const double2 *src = canon + n * 12;
    Spinor<R> s;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 v = src[k];
        s.c[k] = {(R)v.x, (R)v.y};
    }
    SpinorIO<P>::store(eo + par * slab_bytes, g.Vh, i, s);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_unpack(Geom g, double2 *canon, const char *eo, size_t slab_bytes) {
    using R = typename Real<P>::T;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    const SiteCoord c = eo_coords(g, i, par);
    const size_t n = (size_t)c.x + (size_t)g.L[0] * c.row;
    const Spinor<R> s = SpinorIO<P>::load(eo + par * slab_bytes, g.Vh, i);
    double2 *dst = canon + n * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) dst[k] = make_double2((double)s.c[k].re, (double)s.c[k].im);
}

}  // namespace

int launch_load_links(wc_lattice *lat, const void *U, unsigned *err_bits) {
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 8);
    hipLaunchKernelGGL(k_load_links, grid, dim3(kBlock), 0, lat->stream, lat->g, (const double2 *)U,
                       (double2 *)lat->links[P64], (float4 *)lat->links[P32], (char *)lat->links[P16], err_bits);
    WC_HIP(hipGetLastError());
    return WC_OK;
}

int launch_links_full32(wc_lattice *lat) {
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 8);
    hipLaunchKernelGGL(k_links_full32, grid, dim3(kBlock), 0, lat->stream, lat->g, (const char *)lat->links[P64],
                       (char *)lat->links18);
    WC_HIP(hipGetLastError());
    return WC_OK;
}

int launch_links_recon8(wc_lattice *lat, unsigned *min_bits) {
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 8);
    hipLaunchKernelGGL(k_links_recon8, grid, dim3(kBlock), 0, lat->stream, lat->g, (const char *)lat->links[P64],
                       (char *)lat->links8, min_bits);
    WC_HIP(hipGetLastError());
    return WC_OK;
}

int launch_pack_spinor(wc_lattice *lat, int prec, void *eo_out, const void *canon_in) {
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 2);
    const size_t sb = spinor_bytes(prec, lat->Vh);
    if (prec == P64)
        hipLaunchKernelGGL(k_pack<P64>, grid, dim3(kBlock), 0, lat->stream, lat->g, (char *)eo_out,
                           (const double2 *)canon_in, sb);
    else if (prec == P32)
        hipLaunchKernelGGL(k_pack<P32>, grid, dim3(kBlock), 0, lat->stream, lat->g, (char *)eo_out,
                           (const double2 *)canon_in, sb);
    else
        hipLaunchKernelGGL(k_pack<P16>, grid, dim3(kBlock), 0, lat->stream, lat->g, (char *)eo_out,
                           (const double2 *)canon_in, sb);
    WC_HIP(hipGetLastError());
    return WC_OK;
}

int launch_unpack_spinor(wc_lattice *lat, int prec, void *canon_out, const void *eo_in) {
    dim3 grid((lat->Vh + kBlock - 1) / kBlock, 2);
    const size_t sb = spinor_bytes(prec, lat->Vh);
    if (prec == P64)
        hipLaunchKernelGGL(k_unpack<P64>, grid, dim3(kBlock), 0, lat->stream, lat->g, (double2 *)canon_out,
                           (const char *)eo_in, sb);
    else if (prec == P32)
        hipLaunchKernelGGL(k_unpack<P32>, grid, dim3(kBlock), 0, lat->stream, lat->g, (double2 *)canon_out,
                           (const char *)eo_in, sb);
    else
        hipLaunchKernelGGL(k_unpack<P16>, grid, dim3(kBlock), 0, lat->stream, lat->g, (double2 *)canon_out,
                           (const char *)eo_in, sb);
    WC_HIP(hipGetLastError());
    return WC_OK;
}
