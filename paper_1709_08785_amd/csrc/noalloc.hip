// D-hat_ee (Sec. II-B, eq. 8) for callers that cannot allocate device memory.
//
// wc_apply_Dee_oo keeps the odd-parity intermediate F_oo^-1 H_oe in of its two
// MULTs in a lattice-owned buffer that it allocates on first use.  This entry
// point takes that intermediate from a fixed, file-scope device array instead,
// so it calls no allocator at all: code under graph capture, serving loops and
// harnesses that forbid hipMalloc can use it.  The array lives once per GPU
// for the life of the process; its device address is looked up once per
// device and every launch takes that address as an ordinary kernel argument.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

// largest intermediate field this entry point can hold: one parity of a spinor
// field of up to 128 MiB (32^3 x 64 in FP32, 48^3 x 48 in FP16, 32^4 in FP64)
constexpr size_t kScratchBytes = size_t(128) << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// the array's address on the current device (looked up once per device)
int scratch_ptr(void **out) {
    int dev = 0;
    WC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return wc_fail(WC_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return wc_fail(WC_EHIP, std::string("looking up the scratch array: ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return WC_OK;
}

}  // namespace

extern "C" size_t wc_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int wc_apply_Dee_oo_noalloc(wc_lattice *lat, void *out_e, const void *in_e, int prec) {
    if (!lat || !out_e || !in_e) return wc_fail(WC_EINVAL, "null argument");
    if (prec < 0 || prec > 2) return wc_fail(WC_EINVAL, "precision must be WC_FP64, WC_FP32 or WC_FP16");
    if (out_e == in_e) return wc_fail(WC_EINVAL, "wc_apply_Dee_oo_noalloc cannot work in place");
    if (!lat->have_links) return wc_fail(WC_ENOTREADY, "no links loaded");
    if (!lat->have_clover) return wc_fail(WC_ENOTREADY, "no clover term built");
    if (prec == WC_FP16 && lat->su3_err > kSU3MaxErr)
        return wc_fail(WC_EINVAL, "the loaded links are not SU(3) to single precision; the FP16 stencil keeps two columns");
    const size_t need = spinor_bytes(prec, lat->Vh);
    if (need > kScratchBytes)
        return wc_fail(WC_EINVAL, "the intermediate field needs " + std::to_string(need) + " bytes; the fixed scratch of "
                                      "wc_apply_Dee_oo_noalloc holds " + std::to_string(kScratchBytes));
    void *tmp = nullptr;
    if (int rc = scratch_ptr(&tmp)) return rc;
    MultCall c1 = MultCall{};
    c1.prec = prec;
    c1.mode = M_HOPINV;
    c1.red = R_NONE;
    c1.out_par = 1;
    c1.out = tmp;
    c1.in = in_e;
    if (int rc = launch_mult(lat, c1)) return rc;
    MultCall c2 = MultCall{};
    c2.prec = prec;
    c2.mode = M_DHAT;
    c2.red = R_NONE;
    c2.out_par = 0;
    c2.out = out_e;
    c2.in = tmp;
    c2.center = in_e;
    c2.coef = -lat->kappa * lat->kappa;
    return launch_mult(lat, c2);
}
