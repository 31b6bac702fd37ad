// Device-side geometry and coefficient set-up shared by the plan's window
// kernel and the beamforming kernel, so both take bit-identical decisions
// (sample index, aperture membership).
//
// Precision: the receive distance, the delay, the sample coordinate and the
// carrier phase fd * tau (hundreds of cycles) are formed in FP64, because an
// FP32 phase loses ~1e-5 cycles and caps the error near -85 dB.  The
// fractional phase, the interpolation weight and the apodization weight are
// then taken to FP32 for the multiply-accumulate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "das_device_params.h"


// Receive part: depends on (voxel, element) only.
struct das_rx {
    double r;   // |x_v - p_e|
    float w;    // apodization weight
};

// Per (voxel, element, transmit): what the multiply-accumulate needs.
struct das_coef {
    int i0;        // floor(u), valid when active
    int row;       // i0 - first row of the item's window (set by the caller)
    int t;         // transmit of the item (set by the caller; selects the accumulators in per-transmit output)
    float beta;    // u - floor(u)
    float cr, ci;  // w * exp(+j 2 pi fd tau)
    bool active;   // w > 0 and -1 <= i0 <= S - 1
};

// Tukey window on the normalised lateral distance rho (0 outside rho < 1),
// branch-free.  The taper cos(pi x) uses the hardware cosine (turns).
__device__ __forceinline__ float das_tukey(float rho, float alpha, float inv_2alpha) {
    const float edge = 1.0f - alpha;
    const float taper = 0.5f + 0.5f * __builtin_amdgcn_cosf((rho - edge) * inv_2alpha);
    const float w = (rho <= edge) ? 1.0f : taper;
    return (rho < 1.0f) ? w : 0.0f;
}

__device__ __forceinline__ das_rx das_rx_setup(float vx, float vy, float vz, float ex, float ey, float ez,
                                               const das_kparams& kp) {
    const double dx = (double)vx - (double)ex;
    const double dy = (double)vy - (double)ey;
    const double dz = (double)vz - (double)ez;
    das_rx o;
    // |x_v - p_e| to ~1e-15 relative: FP32 square root refined by one FP64
    // Newton step (r + (r2 - r^2) / 2r), cheaper than the FP64 square root.
    const double r2 = dx * dx + dy * dy + dz * dz;
    const float rf = __builtin_amdgcn_sqrtf((float)r2);
    const double r0 = (double)rf;
    o.r = (rf > 0.0f) ? fma(r2 - r0 * r0, (double)(0.5f * __builtin_amdgcn_rcpf(rf)), r0) : 0.0;
    const float dzf = (float)dz;
    const float lat = __builtin_amdgcn_sqrtf((float)(dx * dx + dy * dy));
    const float rho = kp.two_fnum * lat * __builtin_amdgcn_rcpf(dzf);
    const float wa = (dzf > 0.0f) ? das_tukey(rho, kp.alpha, kp.inv_2alpha) : 0.0f;
    o.w = kp.use_apod ? wa : 1.0f;
    return o;
}

__device__ __forceinline__ das_coef das_tx_setup(const das_rx& rx, float tx_arrival, const das_kparams& kp) {
    const double tau = (double)tx_arrival + rx.r * kp.inv_c;
    const double u = (tau - kp.t0) * kp.fs;
    const double fl = floor(u);
    das_coef o;
    o.active = (rx.w > 0.0f) && (fl >= -1.0) && (fl <= (double)(kp.S - 1));
    o.i0 = o.active ? (int)fl : 0;
    o.beta = (float)(u - fl);
    double ph = kp.fd * tau;
    ph -= rint(ph);  // carrier phase in turns, in [-0.5, 0.5]
    // v_sin_f32 / v_cos_f32 take turns; max error 1.3e-7 on [-0.5, 0.5]
    const float pf = (float)ph;
    o.cr = rx.w * __builtin_amdgcn_cosf(pf);
    o.ci = rx.w * __builtin_amdgcn_sinf(pf);
    return o;
}
