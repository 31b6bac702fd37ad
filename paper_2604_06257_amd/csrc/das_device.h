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
    float beta;    // u - floor(u)
    float cr, ci;  // w * exp(+j 2 pi fd tau)
    bool active;   // w > 0 and -1 <= i0 <= S - 1
};

// Tukey window on the normalised lateral distance rho (0 outside rho < 1).
// The taper cos(pi x) uses the hardware cosine, whose argument is in turns.
__device__ __forceinline__ float das_tukey(float rho, float alpha, float inv_2alpha) {
    if (!(rho < 1.0f)) return 0.0f;
    const float edge = 1.0f - alpha;
    if (rho <= edge) return 1.0f;
    return 0.5f + 0.5f * __builtin_amdgcn_cosf((rho - edge) * inv_2alpha);
}

__device__ __forceinline__ das_rx das_rx_setup(float vx, float vy, float vz, float ex, float ey, float ez,
                                               const das_kparams& kp) {
    const double dx = (double)vx - (double)ex;
    const double dy = (double)vy - (double)ey;
    const double dz = (double)vz - (double)ez;
    das_rx o;
    o.r = sqrt(dx * dx + dy * dy + dz * dz);
    if (!kp.use_apod) {
        o.w = 1.0f;
    } else if (!(dz > 0.0)) {
        o.w = 0.0f;
    } else {
        const float lat = sqrtf((float)(dx * dx + dy * dy));
        const float rho = kp.two_fnum * lat * __builtin_amdgcn_rcpf((float)dz);
        o.w = das_tukey(rho, kp.alpha, kp.inv_2alpha);
    }
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
