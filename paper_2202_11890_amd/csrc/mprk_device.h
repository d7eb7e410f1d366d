// mprk_device.h -- device helpers shared by the 2D and 3D stage kernels of
// the MPRK library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "mprk_internal.h"

namespace mprk {
namespace {

__device__ __forceinline__ int wrapx(int c, int nx)
{
    int r = c % nx;
    return r < 0 ? r + nx : r;
}

// Store of a stage result (new stage value, buffer accumulator, retained
// rows).  With `dev` (a per-launch choice of the host) it is a relaxed store
// at device scope, i.e. a plain vector store with the device-coherence bit;
// otherwise an ordinary store.  The stored bits are the same.  Measured per
// step: a single 2D context (1024 x 512 workload) runs 6% (FP64 fluxes) to 8%
// (FP32 fluxes) faster with device-scope stores, while small contexts, the
// batched 2D ensemble and the 3D workload run slower with them, so the host
// chooses per launch record.  Non-temporal stores were slower still.
__device__ __forceinline__ void st_dev(bool dev, double* p, double x)
{
    if (dev) __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = x;
}

// Periodic index for c in [-n, 2n): one conditional add or subtract instead
// of a division.  A tile's halo indices lie in [-2, n + T] for tile width T,
// so this applies whenever n > T (callers test that uniformly).
__device__ __forceinline__ int wrap1(int c, int n)
{
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

// 1/sqrt(x) for positive normal x: hardware estimate refined by two Newton
// steps y <- y + y (1 - x y^2) / 2 (quadratic convergence; a few ulp).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double r = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, r, y);
    r = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, r, y);
}

// 1/x for positive normal x: hardware estimate refined by two Newton steps
// y <- y + y (1 - x y).
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// A kernel argument in the flux type.  The launch record carries FP32 copies,
// rounded to nearest on the host as FT(x) would round them, so FP32 kernels
// take them as uniform operands instead of converting them at every face.
template <class FT>
__device__ __forceinline__ FT arg_ft(double d, float f)
{
    if constexpr (sizeof(FT) == 4) return f;
    else return d;
}

// Reciprocal, square root and reciprocal square root of positive normal
// arguments in the flux type.  FP64: hardware estimates refined by Newton
// steps (a few ulp).  FP32: the hardware instructions (1 ulp).  No scaling
// for subnormals, zero or infinity, which a physical state never produces; a
// non-physical one yields NaN, which the device status check reports.
//
// ws_sqrt and ws_rcp serve only the wave-speed estimate lambda of the LLF
// flux (sound speeds and Roe weights), which scales the dissipation term and
// does not enter the physical flux: in FP64 they take one Newton step from
// the hardware estimate, whose relative error is then the square of the
// estimate's (about 1e-14 and below).  inv_sqrt gives a face state's 1/rho
// for the physical flux and its sqrt(rho), 1/sqrt(rho) for the Roe weights.
template <class FT> struct Fm;
template <> struct Fm<double> {
    static __device__ __forceinline__ double rcp(double x) { return rcp_nr(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return rsqrt_nr(x); }
    static __device__ __forceinline__ double sqrt(double x) { return x * rsqrt_nr(x); }
    static __device__ __forceinline__ double ws_sqrt(double x)
    {
        // s = x y ~ sqrt(x); s + (y/2)(x - s^2)
        const double y = __builtin_amdgcn_rsq(x);
        const double s = x * y;
        return fma(0.5 * y, fma(-s, s, x), s);
    }
    static __device__ __forceinline__ double ws_rcp(double x)
    {
        const double y = __builtin_amdgcn_rcp(x);
        return fma(y, fma(-x, y, 1.0), y);
    }
    // r = 1/x to about an ulp, and y = 1/sqrt(x), s = sqrt(x) to wave-speed
    // accuracy, from one reciprocal square root: y is one Newton step from
    // the estimate (relative error about 1e-14), s = x y, and y^2 is refined
    // by one Newton step of the reciprocal, whose error is then the square
    // of y^2's.
    static __device__ __forceinline__ void inv_sqrt(double x, double& r, double& y, double& s)
    {
        const double y0 = __builtin_amdgcn_rsq(x);
        y = fma(0.5 * y0, fma(-(x * y0), y0, 1.0), y0);
        s = x * y;
        const double r1 = y * y;
        r = fma(r1, fma(-x, r1, 1.0), r1);
    }
};
template <> struct Fm<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float ws_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float ws_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ void inv_sqrt(float x, float& r, float& y, float& s)
    {
        y = __builtin_amdgcn_rsqf(x);
        r = y * y;
        s = x * y;
    }
};

// Viscous coefficient `row` (VK_*) of direction d in the flux type.
template <class FT>
__device__ __forceinline__ FT arg_vk(const DomainArgs& D, int row, int d)
{
    if constexpr (sizeof(FT) == 4) return D.vk_f[row][d];
    else return D.vk[row][d];
}

// The combination of a row: the buffer's or the main one.  Both records are
// read as (uniform) kernel arguments and selected per lane, so that no lane
// loads through a divergent pointer into the argument segment.
__device__ __forceinline__ Combine pick_combine(const Combine& buf, const Combine& main_, bool inb)
{
    const double ab = buf.alpha, am = main_.alpha;
    const double bb = buf.beta, bm = main_.beta;
    const double hb = buf.bh, hm = main_.bh;
    const int mb = buf.mode, mm = main_.mode;
    Combine c;
    c.alpha = inb ? ab : am;
    c.beta = inb ? bb : bm;
    c.bh = inb ? hb : hm;
    c.mode = inb ? mb : mm;
    c.pad = 0;
    return c;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block j to XCD j % 8).
// Give each XCD a contiguous range of the n tiles so that neighbouring tiles,
// which share halo rows and columns, meet in the same L2.
__device__ __forceinline__ int xcd_contiguous(int j, int n)
{
    constexpr int NXCD = 8;
    const int x = j % NXCD, i = j / NXCD;
    const int per = n / NXCD, rem = n % NXCD;
    return (x < rem) ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

}  // namespace
}  // namespace mprk
