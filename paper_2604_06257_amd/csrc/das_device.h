// Device-side geometry and coefficient set-up shared by the plan's window
// kernel and the beamforming kernel, so both take bit-identical decisions
// (sample index, aperture membership).
//
// Precision: the receive distance, the sample coordinate and the carrier phase
// fd * tau (hundreds of cycles) are formed in FP64, because an FP32 phase loses
// ~1e-5 cycles and caps the error near -85 dB.  The fractional phase, the
// interpolation weight and the apodization weight are then taken to FP32 for
// the multiply-accumulate.
//
// Cost layout: what depends on the voxel alone (its coordinates in FP64, and for
// arrays whose elements share one depth plane the depth terms of the distance and
// of the f-number ratio) is formed once per lane; what depends on (voxel,
// transmit) once per transmit (u and the phase are then one FP64 FMA each from
// the receive distance); what depends on (voxel, element) once per element.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "das_device_params.h"

// Per lane (voxel): coordinates (float32, exact in FP64) and the element-plane terms.
struct das_lane {
    float vx, vy, vz;  // voxel coordinates
    double dz2;        // (vz - z0)^2, planar arrays
    float krho;        // 2 f# / (vz - z0), +inf when vz <= z0 (planar arrays)
};

// Receive part: depends on (voxel, element) only.
struct das_rx {
    double r;   // |x_v - p_e|
    float w;    // apodization weight
};

// Transmit part: depends on (voxel, transmit) only.
struct das_txc {
    double a;   // (tau_tx - t0) fs: sample coordinate of the transmit delay
    double b;   // fd tau_tx: carrier cycles of the transmit delay
};

// Per (voxel, element, transmit): what the multiply-accumulate needs.
struct das_coef {
    int i0;        // floor(u)
    int row;       // i0 - first row of the item's window (set by the caller)
    int t;         // transmit of the item (set by the caller; selects the accumulators in per-transmit output)
    float beta;    // u - floor(u)
    float cr, ci;  // w * exp(+j 2 pi fd tau)
};

// rho = lat * krho: 2 f# / dz below the element (dz > 0), +inf above it (w = 0), and 0 when f# = 0 (no
// apodization: the window is then 1 for every pair).
__device__ __forceinline__ float das_krho(double dz, const das_kparams& kp) {
    const float dzf = (float)dz;
    const float k = dzf > 0.0f ? kp.two_fnum * __builtin_amdgcn_rcpf(dzf) : __builtin_inff();
    return kp.use_apod ? k : 0.0f;
}

__device__ __forceinline__ das_lane das_lane_setup(float vx, float vy, float vz, const das_kparams& kp) {
    das_lane L;
    L.vx = vx;
    L.vy = vy;
    L.vz = vz;
    const double dz = (double)vz - kp.z0;
    L.dz2 = dz * dz;
    L.krho = das_krho(dz, kp);
    return L;
}

// Tukey window on the normalised lateral distance rho (0 outside rho < 1; a
// NaN rho, from 0 * inf above the element plane, also gives 0; 1 at rho = 0),
// branch-free.
// The taper cos(pi x) uses the hardware cosine (turns).
__device__ __forceinline__ float das_tukey(float rho, const das_kparams& kp) {
    const float taper = 0.5f + 0.5f * __builtin_amdgcn_cosf(fmaf(rho, kp.inv_2alpha, -kp.edge_2alpha));
    const float w = (rho <= 1.0f - kp.alpha) ? 1.0f : taper;
    return (rho < 1.0f) ? w : 0.0f;
}

// Element coordinates come in FP64 (the plan stores them so).  kPlanar: every element lies in the plane z0
// (the depth terms come from the lane); the result is the same as the general form's for such arrays.
template <bool kPlanar>
__device__ __forceinline__ das_rx das_rx_setup_t(const das_lane& L, double ex, double ey, double ez,
                                                 const das_kparams& kp) {
    const double dx = (double)L.vx - ex;
    const double dy = (double)L.vy - ey;
    const double lat2 = fma(dy, dy, dx * dx);
    double dz2;
    float krho;
    if constexpr (kPlanar) {
        dz2 = L.dz2;
        krho = L.krho;
    } else {
        const double dz = (double)L.vz - ez;
        dz2 = dz * dz;
        krho = das_krho(dz, kp);
    }
    const double r2 = lat2 + dz2;
    das_rx o;
    // |x_v - p_e| to ~1e-13 relative: FP32 reciprocal square root s, r0 = r2 s, then one FP64 Newton step
    // r = r0 + (r2 - r0^2) s / 2 (the floor keeps r2 = 0 finite: r ~ 1e-15 m there)
    const float r2f = fmaxf((float)r2, 1e-30f);
    const float s = __builtin_amdgcn_rsqf(r2f);
    const double r0 = (double)(r2f * s);
    o.r = fma(fma(-r0, r0, r2), (double)(0.5f * s), r0);
    const float rho = __builtin_amdgcn_sqrtf((float)lat2) * krho;
    o.w = das_tukey(rho, kp);  // rho = 0 (f# = 0) gives 1
    return o;
}

__device__ __forceinline__ das_rx das_rx_setup(const das_lane& L, double ex, double ey, double ez,
                                               const das_kparams& kp) {
    return kp.planar ? das_rx_setup_t<true>(L, ex, ey, ez, kp) : das_rx_setup_t<false>(L, ex, ey, ez, kp);
}

__device__ __forceinline__ das_txc das_tx_const(float tx_arrival, const das_kparams& kp) {
    const double t = (double)tx_arrival;
    das_txc o;
    o.a = fma(t, kp.fs, -kp.t0fs);
    o.b = t * kp.fd;
    return o;
}

// u = (tau - t0) fs and fd tau with tau = tau_tx + r / c, each one FP64 FMA.
__device__ __forceinline__ das_coef das_tx_setup(const das_rx& rx, const das_txc& tc, const das_kparams& kp) {
    const double u = fma(rx.r, kp.fs_c, tc.a);
    const double fl = floor(u);
    das_coef o;
    o.i0 = (int)fmin(fmax(fl, -2.0), 1073741824.0);  // rows far outside the record are never in a window
    o.beta = (float)(u - fl);
    double ph = fma(rx.r, kp.fd_c, tc.b);
    ph -= rint(ph);  // carrier phase in turns, in [-0.5, 0.5]
    // v_sin_f32 / v_cos_f32 take turns; max error 1.3e-7 on [-0.5, 0.5]
    const float pf = (float)ph;
    o.cr = rx.w * __builtin_amdgcn_cosf(pf);
    o.ci = rx.w * __builtin_amdgcn_sinf(pf);
    return o;
}

// Whether a (voxel, element, transmit) triple contributes: weight > 0 and the delayed sample inside the
// record (floor(u) in [-1, S - 1], with zero padding on both sides).
__device__ __forceinline__ bool das_active(const das_rx& rx, const das_coef& c, const das_kparams& kp) {
    return rx.w > 0.0f && c.i0 >= -1 && c.i0 <= kp.S - 1;
}
