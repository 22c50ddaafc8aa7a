// Device-side building blocks shared by the gfx950 kernels: complex arithmetic,
// even-odd geometry, and the structure-of-arrays accessors of each storage
// precision.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#define WC_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <class R> struct cx {
    R re, im;
};

template <class R> WC_HD cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <class R> WC_HD cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> WC_HD cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> WC_HD cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <class R> WC_HD cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> WC_HD cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> WC_HD cx<R> conjx(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class R> WC_HD cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a, -i * a
template <class R> WC_HD cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }
template <class R> WC_HD cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }
// fused multiply-add in the precision of R
WC_HD float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
WC_HD double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc += a * b, as a chain of four fused multiply-adds into the accumulator
// (written out: "acc + (a.re b.re - a.im b.im)" would cost a multiply, an FMA
// and an add per component, since the sum may not be reassociated)
template <class R> WC_HD void cmac(cx<R> &acc, cx<R> a, cx<R> b) {
    acc.re = fmar(a.re, b.re, acc.re);
    acc.re = fmar(-a.im, b.im, acc.re);
    acc.im = fmar(a.re, b.im, acc.im);
    acc.im = fmar(a.im, b.re, acc.im);
}
// acc += conj(a) * b, likewise
template <class R> WC_HD void cmacc(cx<R> &acc, cx<R> a, cx<R> b) {
    acc.re = fmar(a.re, b.re, acc.re);
    acc.re = fmar(a.im, b.im, acc.re);
    acc.im = fmar(a.re, b.im, acc.im);
    acc.im = fmar(-a.im, b.re, acc.im);
}
template <class R> WC_HD R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// even-odd geometry
//   site n = x + Lx (y + Ly (z + Lz t)), parity (x+y+z+t)&1, EO index n >> 1.
//   All extents are even, so each x-row holds Lx/2 sites of each parity and
//   EO index i of parity p decodes as xh = i % (Lx/2), row = i / (Lx/2).
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];      // Lx, Ly, Lz, Lt
    int Lxh;       // Lx / 2
    int Vh;        // sites per parity
};

struct SiteCoord {
    int x, y, z, t, row;  // row = y + Ly (z + Lz t)
};

WC_HD SiteCoord eo_coords(const Geom &g, int i, int parity) {
    SiteCoord c;
    int xh = i % g.Lxh;
    c.row = i / g.Lxh;
    c.y = c.row % g.L[1];
    int r2 = c.row / g.L[1];
    c.z = r2 % g.L[2];
    c.t = r2 / g.L[2];
    c.x = 2 * xh + ((parity + c.y + c.z + c.t) & 1);
    return c;
}

// EO index (within the opposite parity) of the neighbour n + s mu-hat, s = +-1
WC_HD int eo_neighbour(const Geom &g, const SiteCoord &c, int mu, int s) {
    if (mu == 0) {
        int x = c.x + s;
        x = (x == g.L[0]) ? 0 : (x < 0 ? g.L[0] - 1 : x);
        return (x >> 1) + g.Lxh * c.row;
    }
    int row;
    if (mu == 1) {
        int y = c.y + s;
        y = (y == g.L[1]) ? 0 : (y < 0 ? g.L[1] - 1 : y);
        row = c.row + (y - c.y);
    } else if (mu == 2) {
        int z = c.z + s;
        z = (z == g.L[2]) ? 0 : (z < 0 ? g.L[2] - 1 : z);
        row = c.row + (z - c.z) * g.L[1];
    } else {
        int t = c.t + s;
        t = (t == g.L[3]) ? 0 : (t < 0 ? g.L[3] - 1 : t);
        row = c.row + (t - c.t) * g.L[1] * g.L[2];
    }
    return (c.x >> 1) + g.Lxh * row;
}

// ---------------------------------------------------------------------------
// storage precisions
//   spinor  (12 complex per site)
//     FP64: 12 planes of double2                                  (192 B/site)
//     FP32:  6 planes of float4 (two complex per plane)           ( 96 B/site)
//     FP16:  3 planes of uint4 (eight halves = four complex per plane) plus a
//            float scale plane; value = scale * half               ( 52 B/site)
//   links (one (mu, parity) slab)
//     FP64: 9 planes of double2, row-major U[i][j]                (144 B/site)
//     FP32: 3 planes of float4: columns 0 and 1 (U00 U10 | U20 U01 | U11 U21);
//           column 2 = conj(col0 x col1)                          ( 48 B/site)
//     FP16: the same six complex as halves: 1 uint4 + 1 uint2 plane (24 B/site)
//   clover (two Hermitian 6x6 blocks per site, each 6 real diagonal entries
//           then the 15 complex entries above the diagonal, row by row)
//     FP64: 36 planes of double2                                  (576 B/site)
//     FP32: 18 planes of float4                                   (288 B/site)
//     FP16: per block 4 uint4 + 1 uint2 planes, then a float scale plane
//                                                                 (148 B/site)
//
// Site tiles.  A parity slab is cut into tiles of kTile consecutive EO sites;
// a tile holds every plane of its sites, plane after plane, each plane kTile
// consecutive entries.  One wavefront's load of a plane is then 64 adjacent
// entries, and all planes of its sites share a few KB of one DRAM region
// instead of being spread over slabs hundreds of MB apart.  A plane at byte
// offset OFF of the site record (the bytes of the planes before it) with
// entries of E bytes lives, for site i, at
//     slab + (i / kTile) * kTile * SB + OFF * kTile + (i % kTile) * E,
// SB being the bytes per site.  Slabs are padded to whole tiles.
// ---------------------------------------------------------------------------
enum { P64 = 0, P32 = 1, P16 = 2 };

template <int P> struct Real;
template <> struct Real<P64> { using T = double; };
template <> struct Real<P32> { using T = float; };
template <> struct Real<P16> { using T = float; };

constexpr int kTile = 64;

WC_HD int pad_sites(int Vh) { return (Vh + kTile - 1) / kTile * kTile; }

// logical block of hardware block b, which runs on XCD b mod 8.  The logical
// blocks are cut into windows of 8 chunks of kXcdChunk consecutive blocks,
// and XCD x takes chunk x of every window, in order: all XCDs sweep one
// front, y and z neighbours stay within an XCD's chunk (its L2), and a t
// neighbour that is read again two t-slices later is still in the
// memory-side cache.  Blocks past the last whole window are split into one
// slab per XCD; a ragged tail keeps its own index.
// chunk: blocks per chunk.  The stencil launches pass the lattice's chunk
// (tuned, in 64-site tiles, converted to blocks of the launch); the default
// kXcdChunk serves the one-launch inner loop, whose 256-site blocks then take
// 64 tiles per chunk.  chunk <= 0 gives one contiguous slab of blocks per XCD.
constexpr int kXcdChunk = 16;
WC_HD int xcd_block(int b, int nb, int chunk = kXcdChunk) {
    if (chunk <= 0) chunk = nb;  // a window larger than the launch: slabs only
    const int win = 8 * chunk;
    const int full = nb / win * win;
    if (b < full) {
        const int k = b >> 3;
        return ((k / chunk) * 8 + (b & 7)) * chunk + k % chunk;
    }
    const int rb = b - full, per = (nb - full) >> 3;
    return full + ((rb < (per << 3)) ? (rb & 7) * per + (rb >> 3) : rb);
}

// bytes per site of each field kind
WC_HD size_t spinor_site_bytes(int prec) { return prec == P64 ? 192 : prec == P32 ? 96 : 52; }
WC_HD size_t link_site_bytes(int prec) { return prec == P64 ? 144 : prec == P32 ? 48 : 24; }
WC_HD size_t clover_site_bytes(int prec) { return prec == P64 ? 576 : prec == P32 ? 288 : 148; }

// bytes of one (padded) parity slab of each field kind
WC_HD size_t spinor_bytes(int prec, int Vh) { return (size_t)pad_sites(Vh) * spinor_site_bytes(prec); }
WC_HD size_t link_slab_bytes(int prec, int Vh) { return (size_t)pad_sites(Vh) * link_site_bytes(prec); }
WC_HD size_t clover_slab_bytes(int prec, int Vh) { return (size_t)pad_sites(Vh) * clover_site_bytes(prec); }

// byte offset of entry i of the plane at record offset off (entries of eb bytes)
// in a tiled slab of sb bytes per site
WC_HD size_t tile_off(int i, size_t sb, size_t off, size_t eb) {
    const unsigned u = (unsigned)i;
    return (size_t)(u / kTile) * (kTile * sb) + off * kTile + (size_t)(u % kTile) * eb;
}
template <class E, int SB> __device__ __forceinline__ const E *tp(const void *slab, int i, int off) {
    return (const E *)((const char *)slab + tile_off(i, SB, (size_t)off, sizeof(E)));
}
template <class E, int SB> __device__ __forceinline__ E *tp(void *slab, int i, int off) {
    return (E *)((char *)slab + tile_off(i, SB, (size_t)off, sizeof(E)));
}

template <class R> struct Spinor {
    cx<R> c[12];  // index 3*alpha + colour
};

// ---- non-temporal loads: streamed operands that are read exactly once ----
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 ld_stream(const float4 *p) {
    nt_f4 v = __builtin_nontemporal_load((const nt_f4 *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_stream(const double2 *p) {
    nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_stream(const uint4 *p) {
    nt_u4 v = __builtin_nontemporal_load((const nt_u4 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_stream(const uint2 *p) {
    nt_u2 v = __builtin_nontemporal_load((const nt_u2 *)p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2 *p) {
    nt_f2 v = __builtin_nontemporal_load((const nt_f2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(float4 *p, float4 v) {
    __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, (nt_f4 *)p);
}
__device__ __forceinline__ void st_stream(double2 *p, double2 v) {
    __builtin_nontemporal_store(nt_d2{v.x, v.y}, (nt_d2 *)p);
}
__device__ __forceinline__ void st_stream(uint4 *p, uint4 v) {
    __builtin_nontemporal_store(nt_u4{v.x, v.y, v.z, v.w}, (nt_u4 *)p);
}
__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
template <bool NT, class T> __device__ __forceinline__ void st_op(T *p, T v) {
    if (NT) st_stream(p, v);
    else *p = v;
}
// operand load: non-temporal when NT (read once per launch), cached otherwise
// (operands that several systems of one batched launch read)
template <bool NT, class T> __device__ __forceinline__ T ld_op(const T *p) {
    if (NT) return ld_stream(p);
    return *p;
}

// ---- half <-> float ----
// an empty statement that hides a value's origin from the optimiser (no code)
__device__ __forceinline__ void keep(float2 &v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y));
}
__device__ __forceinline__ float2 h2f(uint32_t u) {
    __half2 h = *reinterpret_cast<__half2 *>(&u);
    return __half22float2(h);
}
__device__ __forceinline__ uint32_t f2h(float a, float b) {
    __half2 h = __floats2half2_rn(a, b);
    return *reinterpret_cast<uint32_t *>(&h);
}

// ---------------------------------------------------------------------------
// spinor load / store (one tiled parity slab; Vh is the slab's site count)
// ---------------------------------------------------------------------------
template <int P> struct SpinorIO;

template <> struct SpinorIO<P64> {
    using R = double;
    template <bool NT = false> __device__ static Spinor<R> load(const void *base, int Vh, int i) {
        Spinor<R> s;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = ld_op<NT>(tp<double2, 192>(base, i, 16 * k));
            s.c[k] = {v.x, v.y};
        }
        return s;
    }
    template <bool NT = false> __device__ static void store(void *base, int Vh, int i, const Spinor<R> &s) {
#pragma unroll
        for (int k = 0; k < 12; k++) st_op<NT>(tp<double2, 192>(base, i, 16 * k), make_double2(s.c[k].re, s.c[k].im));
    }
};

template <> struct SpinorIO<P32> {
    using R = float;
    template <bool NT = false> __device__ static Spinor<R> load(const void *base, int Vh, int i) {
        Spinor<R> s;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = ld_op<NT>(tp<float4, 96>(base, i, 16 * k));
            s.c[2 * k] = {v.x, v.y};
            s.c[2 * k + 1] = {v.z, v.w};
        }
        return s;
    }
    template <bool NT = false> __device__ static void store(void *base, int Vh, int i, const Spinor<R> &s) {
#pragma unroll
        for (int k = 0; k < 6; k++)
            st_op<NT>(tp<float4, 96>(base, i, 16 * k),
                      make_float4(s.c[2 * k].re, s.c[2 * k].im, s.c[2 * k + 1].re, s.c[2 * k + 1].im));
    }
};

// FP16 storage: planes of uint4 (3 * 16 B) followed by a float scale plane at 48
template <> struct SpinorIO<P16> {
    using R = float;
    // stored values without their site scale, from the three stored planes
    __device__ static Spinor<R> decode(const uint4 (&v)[3]) {
        Spinor<R> out;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float2 a = h2f(v[k].x), b = h2f(v[k].y), c = h2f(v[k].z), d = h2f(v[k].w);
            out.c[4 * k + 0] = {a.x, a.y};
            out.c[4 * k + 1] = {b.x, b.y};
            out.c[4 * k + 2] = {c.x, c.y};
            out.c[4 * k + 3] = {d.x, d.y};
        }
        return out;
    }
    // stored values without their site scale, and the scale
    __device__ static Spinor<R> load_raw(const void *base, int Vh, int i, float &s) {
        s = *tp<float, 52>(base, i, 48);
        Spinor<R> out;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint4 v = *tp<uint4, 52>(base, i, 16 * k);
            const float2 a = h2f(v.x), b = h2f(v.y), c = h2f(v.z), d = h2f(v.w);
            out.c[4 * k + 0] = {a.x, a.y};
            out.c[4 * k + 1] = {b.x, b.y};
            out.c[4 * k + 2] = {c.x, c.y};
            out.c[4 * k + 3] = {d.x, d.y};
        }
        return out;
    }
    template <bool NT = false> __device__ static Spinor<R> load(const void *base, int Vh, int i) {
        const float s = ld_op<NT>(tp<float, 52>(base, i, 48));
        Spinor<R> out;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = ld_op<NT>(tp<uint4, 52>(base, i, 16 * k));
            float2 a = h2f(v.x), b = h2f(v.y), c = h2f(v.z), d = h2f(v.w);
            out.c[4 * k + 0] = {s * a.x, s * a.y};
            out.c[4 * k + 1] = {s * b.x, s * b.y};
            out.c[4 * k + 2] = {s * c.x, s * c.y};
            out.c[4 * k + 3] = {s * d.x, s * d.y};
        }
        return out;
    }
    template <bool NT = false> __device__ static void store(void *base, int Vh, int i, const Spinor<R> &v) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v.c[k].re), fabsf(v.c[k].im)));
        float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 u;
            u.x = f2h(v.c[4 * k + 0].re * inv, v.c[4 * k + 0].im * inv);
            u.y = f2h(v.c[4 * k + 1].re * inv, v.c[4 * k + 1].im * inv);
            u.z = f2h(v.c[4 * k + 2].re * inv, v.c[4 * k + 2].im * inv);
            u.w = f2h(v.c[4 * k + 3].re * inv, v.c[4 * k + 3].im * inv);
            st_op<NT>(tp<uint4, 52>(base, i, 16 * k), u);
        }
        st_op<NT>(tp<float, 52>(base, i, 48), m);
    }
};

// ---------------------------------------------------------------------------
// links: full 3x3 matrices in registers
// ---------------------------------------------------------------------------
template <class R> struct Mat3 {
    cx<R> m[9];  // row-major
};

template <class R> WC_HD void recon_col2(Mat3<R> &u) {
    // column 2 = conj(col0 x col1)
    cx<R> a0 = u.m[0], a1 = u.m[3], a2 = u.m[6];
    cx<R> b0 = u.m[1], b1 = u.m[4], b2 = u.m[7];
    u.m[2] = conjx(a1 * b2 - a2 * b1);
    u.m[5] = conjx(a2 * b0 - a0 * b2);
    u.m[8] = conjx(a0 * b1 - a1 * b0);
}

template <int P> struct LinkIO;

template <> struct LinkIO<P64> {
    using R = double;
    template <bool NT = true> __device__ static Mat3<R> load(const void *slab, int Vh, int i) {
        Mat3<R> u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            double2 v = ld_op<NT>(tp<double2, 144>(slab, i, 16 * k));
            u.m[k] = {v.x, v.y};
        }
        return u;
    }
};

template <> struct LinkIO<P32> {
    using R = float;
    template <bool NT = true> __device__ static Mat3<R> load(const void *slab, int Vh, int i) {
        float4 a = ld_op<NT>(tp<float4, 48>(slab, i, 0));
        float4 b = ld_op<NT>(tp<float4, 48>(slab, i, 16));
        float4 c = ld_op<NT>(tp<float4, 48>(slab, i, 32));
        Mat3<R> u;
        u.m[0] = {a.x, a.y};
        u.m[3] = {a.z, a.w};
        u.m[6] = {b.x, b.y};
        u.m[1] = {b.z, b.w};
        u.m[4] = {c.x, c.y};
        u.m[7] = {c.z, c.w};
        recon_col2(u);
        return u;
    }
};

template <> struct LinkIO<P16> {
    using R = float;
    template <bool NT = true> __device__ static Mat3<R> load(const void *slab, int Vh, int i) {
        uint4 a = ld_op<NT>(tp<uint4, 24>(slab, i, 0));
        uint2 b = ld_op<NT>(tp<uint2, 24>(slab, i, 16));
        return decode(a, b);
    }
    // the link from its two stored planes
    __device__ static Mat3<R> decode(uint4 a, uint2 b) {
        float2 v0 = h2f(a.x), v1 = h2f(a.y), v2 = h2f(a.z), v3 = h2f(a.w), v4 = h2f(b.x), v5 = h2f(b.y);
        // convert each half once: left to itself the compiler folds the
        // conversion into every product as a mixed-precision FMA, which issues
        // slower than a plain FMA and is used 6 times per entry
        keep(v0); keep(v1); keep(v2); keep(v3); keep(v4); keep(v5);
        Mat3<R> u;
        u.m[0] = {v0.x, v0.y};
        u.m[3] = {v1.x, v1.y};
        u.m[6] = {v2.x, v2.y};
        u.m[1] = {v3.x, v3.y};
        u.m[4] = {v4.x, v4.y};
        u.m[7] = {v5.x, v5.y};
        recon_col2(u);
        return u;
    }
};

// ---------------------------------------------------------------------------
// links from 8 real parameters (reconstruct-8), FP32 storage
//   Stored per link: a2 = U01, a3 = U02, y, t_a = arg(U00)/pi and t_z.
//   With N = |U01|^2 + |U02|^2 = |U10|^2 + |U20|^2 (unit first row and first
//   column), y is whichever of U10, U20 has the smaller modulus and the other,
//   z, is rebuilt from |z|^2 = N - |y|^2 >= N/2, a subtraction that cannot
//   cancel; t_z = arg(z)/pi taken in [0, 2), its sign bit set when y holds U20
//   (a sign bit, unlike an offset, cannot be lost to rounding and costs no
//   precision).  |U00|^2 = 1 - N.
//   Writing a1 = U00, b1 = U10, c1 = U20, orthogonality of the rows to the
//   first row and det U = 1 fix the remaining 2x2 block:
//     U11 = -(b1 a1* a2 + c1* a3*) / N      U12 = (c1* a2* - b1 a1* a3) / N
//     U21 = (b1* a3* - c1 a1* a2) / N       U22 = -(c1 a1* a3 + b1* a2*) / N
//   Two float4 planes: (a2 | a3), (y | t_a, t_z)                  (32 B/site)
//   The rebuilt entries carry a few FP32 rounding steps (every numerator
//   term is O(N), so dividing by N does not amplify them); N must not vanish,
//   and the library checks its minimum before use.
// ---------------------------------------------------------------------------
WC_HD size_t link8_slab_bytes(int Vh) { return (size_t)pad_sites(Vh) * 32; }

__device__ __forceinline__ Mat3<float> recon8(cx<float> a2, cx<float> a3, cx<float> y, float ta, float tz) {
    const float N = norm2(a2) + norm2(a3);
    const bool swap = signbit(tz);
    const float t = fabsf(tz);
    float sa, ca, sz, cz;
    sincospif(ta, &sa, &ca);
    sincospif(t, &sz, &cz);
    const float ma = sqrtf(fmaxf(1.0f - N, 0.0f));
    const float mz = sqrtf(fmaxf(N - norm2(y), 0.0f));
    const cx<float> a1 = {ma * ca, ma * sa}, z = {mz * cz, mz * sz};
    const cx<float> b1 = swap ? z : y, c1 = swap ? y : z;
    const float inv = 1.0f / N;
    const cx<float> ba = cmulc(a1, b1), ca1 = cmulc(a1, c1);  // b1 a1*, c1 a1*
    const cx<float> c1a3 = conjx(c1 * a3), c1a2 = conjx(c1 * a2), b1a3 = conjx(b1 * a3), b1a2 = conjx(b1 * a2);
    Mat3<float> u;
    u.m[0] = a1;
    u.m[1] = a2;
    u.m[2] = a3;
    u.m[3] = b1;
    u.m[6] = c1;
    u.m[4] = -inv * (ba * a2 + c1a3);
    u.m[5] = inv * (c1a2 - ba * a3);
    u.m[7] = inv * (b1a3 - ca1 * a2);
    u.m[8] = -inv * (ca1 * a3 + b1a2);
    return u;
}

struct Link8IO {
    template <bool NT = true> __device__ static Mat3<float> load(const void *slab, int Vh, int i) {
        const float4 a = ld_op<NT>(tp<float4, 32>(slab, i, 0));
        const float4 b = ld_op<NT>(tp<float4, 32>(slab, i, 16));
        return recon8({a.x, a.y}, {a.z, a.w}, {b.x, b.y}, b.z, b.w);
    }
};

// ---------------------------------------------------------------------------
// links stored in full (18 reals), FP32: for links that are not SU(3) to FP32
// accuracy, where neither reconstruction holds.  Row-major entries 0..7 in
// four float4 planes, entry 8 in a float2 plane                 (72 B/site)
// ---------------------------------------------------------------------------
WC_HD size_t link18_slab_bytes(int Vh) { return (size_t)pad_sites(Vh) * 72; }

struct Link18IO {
    template <bool NT = true> __device__ static Mat3<float> load(const void *slab, int Vh, int i) {
        Mat3<float> u;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float4 a = ld_op<NT>(tp<float4, 72>(slab, i, 16 * k));
            u.m[2 * k] = {a.x, a.y};
            u.m[2 * k + 1] = {a.z, a.w};
        }
        const float2 b = ld_op<NT>(tp<float2, 72>(slab, i, 64));
        u.m[8] = {b.x, b.y};
        return u;
    }
};

// the link accessor a stencil instance uses: LR is the link form, 12 (two
// columns, the third rebuilt), 8 (reconstruct-8) or 18 (full); the last two
// exist for the FP32 stencil only
template <int P, int LR> struct LinkLoad {
    template <bool NT> __device__ static Mat3<typename Real<P>::T> load(const void *slab, int Vh, int i) {
        return LinkIO<P>::template load<NT>(slab, Vh, i);
    }
};
template <> struct LinkLoad<P32, 8> {
    template <bool NT> __device__ static Mat3<float> load(const void *slab, int Vh, int i) {
        return Link8IO::template load<NT>(slab, Vh, i);
    }
};
template <> struct LinkLoad<P32, 18> {
    template <bool NT> __device__ static Mat3<float> load(const void *slab, int Vh, int i) {
        return Link18IO::template load<NT>(slab, Vh, i);
    }
};

// ---------------------------------------------------------------------------
// clover blocks: y = M w for a packed Hermitian 6x6 M
// ---------------------------------------------------------------------------
template <class R> struct Herm6 {
    R d[6];
    cx<R> o[15];  // (0,1) (0,2) .. (0,5) (1,2) .. (4,5)
};

template <class R> WC_HD void herm6_apply(const Herm6<R> &M, const cx<R> *w, cx<R> *y) {
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = M.d[i] * w[i];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; i++) {
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            cmac(y[i], M.o[k], w[j]);
            cmacc(y[j], M.o[k], w[i]);
            k++;
        }
    }
}

template <int P> struct CloverIO;

template <> struct CloverIO<P64> {
    using R = double;
    // block b (0: g5 = +1, 1: g5 = -1) of site i
    template <bool NT = true> __device__ static Herm6<R> load(const void *slab, int Vh, int i, int b) {
        Herm6<R> M;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            double2 v = ld_op<NT>(tp<double2, 576>(slab, i, 16 * (18 * b + k)));
            M.d[2 * k] = v.x;
            M.d[2 * k + 1] = v.y;
        }
#pragma unroll
        for (int k = 0; k < 15; k++) {
            double2 v = ld_op<NT>(tp<double2, 576>(slab, i, 16 * (18 * b + 3 + k)));
            M.o[k] = {v.x, v.y};
        }
        return M;
    }
};

template <> struct CloverIO<P32> {
    using R = float;
    template <bool NT = true> __device__ static Herm6<R> load(const void *slab, int Vh, int i, int b) {
        float f[36];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float4 v = ld_op<NT>(tp<float4, 288>(slab, i, 16 * (9 * b + k)));
            f[4 * k] = v.x;
            f[4 * k + 1] = v.y;
            f[4 * k + 2] = v.z;
            f[4 * k + 3] = v.w;
        }
        Herm6<R> M;
#pragma unroll
        for (int k = 0; k < 6; k++) M.d[k] = f[k];
#pragma unroll
        for (int k = 0; k < 15; k++) M.o[k] = {f[6 + 2 * k], f[7 + 2 * k]};
        return M;
    }
};

// FP16 clover: per block b, 4 uint4 planes then 1 uint2 plane (36 halves = 72 B per
// site and block, block b at record offset 72 b), then one FP32 scale plane at
// record offset 144; entry = scale * half.
template <> struct CloverIO<P16> {
    using R = float;
    __device__ static float scale(const void *slab, int i) { return *tp<float, 148>(slab, i, 144); }
    template <bool NT = true> __device__ static Herm6<R> load(const void *slab, int Vh, int i, int b) {
        return load_scaled<NT>(slab, Vh, i, b, scale(slab, i));
    }
    // block b with its entries multiplied by s (s = 1: the stored values)
    template <bool NT = true> __device__ static Herm6<R> load_scaled(const void *slab, int Vh, int i, int b, float s) {
        uint32_t w[18];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint4 v = ld_op<NT>(tp<uint4, 148>(slab, i, 72 * b + 16 * k));
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
        uint2 v = ld_op<NT>(tp<uint2, 148>(slab, i, 72 * b + 64));
        w[16] = v.x;
        w[17] = v.y;
        float f[36];
#pragma unroll
        for (int k = 0; k < 18; k++) {
            float2 h = h2f(w[k]);
            keep(h);  // one conversion per entry, as for the links
            f[2 * k] = s * h.x;
            f[2 * k + 1] = s * h.y;
        }
        Herm6<R> M;
#pragma unroll
        for (int k = 0; k < 6; k++) M.d[k] = f[k];
#pragma unroll
        for (int k = 0; k < 15; k++) M.o[k] = {f[6 + 2 * k], f[7 + 2 * k]};
        return M;
    }
};

// Apply a site's clover pair to a spinor in the Dirac basis.
// The pair holds M1 = (A - B)/2 on the g5 = +1 space (u, -u) and M2 = (A + B)/2 on
// the g5 = -1 space (u, u), where F = [[A, B], [B, A]] in upper/lower spin blocks.
// Then  up = M2 (psi_u + psi_d) + M1 (psi_u - psi_d),
//       dn = M2 (psi_u + psi_d) - M1 (psi_u - psi_d).
template <int P, class R, bool NT = true>
__device__ __forceinline__ void clover_apply(const void *slab, int Vh, int i, const Spinor<R> &in, Spinor<R> &out) {
    cx<R> wm[6], wp[6], ym[6], yp[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        wm[k] = in.c[k] - in.c[k + 6];
        wp[k] = in.c[k] + in.c[k + 6];
    }
    if constexpr (P == P16) {
        // one scale per site for both blocks: apply it once to the result
        const float s = CloverIO<P16>::scale(slab, i);
        {
            Herm6<R> M = CloverIO<P16>::template load_scaled<NT>(slab, Vh, i, 0, 1.0f);
            herm6_apply(M, wm, ym);
        }
        {
            Herm6<R> M = CloverIO<P16>::template load_scaled<NT>(slab, Vh, i, 1, 1.0f);
            herm6_apply(M, wp, yp);
        }
#pragma unroll
        for (int k = 0; k < 6; k++) {
            out.c[k] = s * (yp[k] + ym[k]);
            out.c[k + 6] = s * (yp[k] - ym[k]);
        }
    } else {
        {
            Herm6<R> M = CloverIO<P>::template load<NT>(slab, Vh, i, 0);
            herm6_apply(M, wm, ym);
        }
        {
            Herm6<R> M = CloverIO<P>::template load<NT>(slab, Vh, i, 1);
            herm6_apply(M, wp, yp);
        }
#pragma unroll
        for (int k = 0; k < 6; k++) {
            out.c[k] = yp[k] + ym[k];
            out.c[k + 6] = yp[k] - ym[k];
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 links and site fields addressed by lattice coordinates (used by the
// one-time clover build and by the gradient kernels; the stencil itself uses
// the EO neighbour arithmetic above)
// ---------------------------------------------------------------------------
struct SiteRef {
    int par, i;  // parity and EO index
};

WC_HD SiteRef site_ref(const Geom &g, int x, int y, int z, int t) {
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    x = (x % L0 + L0) % L0;
    y = (y % L1 + L1) % L1;
    z = (z % L2 + L2) % L2;
    t = (t % L3 + L3) % L3;
    const int n = x + L0 * (y + L1 * (z + L2 * t));
    return SiteRef{(x + y + z + t) & 1, n >> 1};
}

// U_mu at a site from the FP64 link copy (tiled slabs [mu][parity])
__device__ __forceinline__ Mat3<double> link64(const double2 *l64, const Geom &g, int mu, SiteRef s) {
    const char *slab = (const char *)l64 + (size_t)(2 * mu + s.par) * link_slab_bytes(P64, g.Vh);
    Mat3<double> u;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        double2 v = *tp<double2, 144>(slab, s.i, 16 * k);
        u.m[k] = {v.x, v.y};
    }
    return u;
}
