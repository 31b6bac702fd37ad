// GPU version of the forward echo simulator in _echo.c (input generator).
//
// Same model: for transmit t, element e, frame f
//   iq[t,e,s,f] = sum_k A_k g(ts - tau_k) exp(-j 2 pi fd tau_k) exp(j 2 pi (fc - fd)(ts - tau_k))
// with ts = t0 + s/fs, a Gaussian g truncated at trunc*sigma, and
// tau_k = (n_t . x_k)/c + |x_k - p_e|/c.
//
// One workgroup per (t, e, f) record.  Each thread takes scatterers in turn,
// evaluates its delay in float64 and steps the Gaussian and the carrier
// through the pulse window with the same multiplicative recurrences as the C
// code, adding each sample into an LDS accumulator in 2^-32 fixed point
// (64-bit integer adds are associative, so the result does not depend on the
// order the threads arrive in).  The record is converted to float32 once.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr double kFix = 4294967296.0;  // 2^32

__global__ __launch_bounds__(kThreads) void echo_kernel(float* __restrict__ iq, int T, int E, int S, int F,
                                                        const double* __restrict__ elem,
                                                        const double* __restrict__ normal,
                                                        const double* __restrict__ scat,
                                                        const double* __restrict__ amp, int K, double c, double fs,
                                                        double h, double t0, double inv2s2, double q, double wr,
                                                        double wi, double two_pi_fd, double two_pi_df, double half) {
    extern __shared__ unsigned long long acc[];  // [S][2]
    const int rec = blockIdx.x;                  // (t * E + e) * F + f
    const int f = rec % F;
    const int te = rec / F;
    const int e = te % E, t = te / E;
    for (int i = threadIdx.x; i < 2 * S; i += kThreads) acc[i] = 0ull;
    __syncthreads();
    const double ex = elem[3 * e], ey = elem[3 * e + 1], ez = elem[3 * e + 2];
    const double nx = normal[3 * t], ny = normal[3 * t + 1], nz = normal[3 * t + 2];
    const double* xs = scat + (int64_t)f * K * 3;
    const double* as = amp + (int64_t)f * K;
    for (int k = threadIdx.x; k < K; k += kThreads) {
        const double x = xs[3 * k], y = xs[3 * k + 1], z = xs[3 * k + 2];
        const double dx = x - ex, dy = y - ey, dz = z - ez;
        const double tau = (nx * x + ny * y + nz * z) / c + sqrt(dx * dx + dy * dy + dz * dz) / c;
        long long lo = (long long)ceil((tau - half - t0) * fs);
        long long hi = (long long)floor((tau + half - t0) * fs);
        if (lo < 0) lo = 0;
        if (hi > S - 1) hi = S - 1;
        if (lo > hi) continue;
        const double a = t0 + (double)lo * h - tau;
        double g = as[k] * exp(-a * a * inv2s2);
        double r = exp(-(2.0 * a * h + h * h) * inv2s2);
        const double ph = -two_pi_fd * tau + two_pi_df * a;
        double pr = cos(ph), pi = sin(ph);
        for (long long s = lo; s <= hi; ++s) {
            atomicAdd(&acc[2 * s], (unsigned long long)__double2ll_rn(g * pr * kFix));
            atomicAdd(&acc[2 * s + 1], (unsigned long long)__double2ll_rn(g * pi * kFix));
            g *= r;
            r *= q;
            const double npr = pr * wr - pi * wi;
            pi = pr * wi + pi * wr;
            pr = npr;
        }
    }
    __syncthreads();
    float* dst = iq + 2 * ((int64_t)te * S * F);
    for (int i = threadIdx.x; i < 2 * S; i += kThreads) {
        const int s = i >> 1, comp = i & 1;
        dst[2 * ((int64_t)s * F + f) + comp] = (float)((double)(long long)acc[i] / kFix);
    }
}

}  // namespace

extern "C" {

// iq: device complex64 [T][E][S][F]; elem [E][3], normal [T][3], scat [F][K][3], amp [F][K]: device float64.
// S <= 4096 (the record's accumulator lives in LDS).  Returns 0, -2 for sizes or pointers out of range,
// -5 for a launch failure.
int synth_echo_gpu(float* iq, int T, int E, int S, int F, const double* elem, const double* normal,
                   const double* scat, const double* amp, int K, double c, double fs, double fc, double fd, double t0,
                   double sigma, double trunc_sigmas, void* stream) {
    if (T < 1 || E < 1 || S < 1 || F < 1 || K < 0 || (int64_t)T * E * F > 0x7fffffff || S > 4096) return -2;
    if (!iq || !elem || !normal || (K > 0 && (!scat || !amp))) return -2;
    const double two_pi = 6.283185307179586476925286766559;
    const double h = 1.0 / fs;
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const double q = exp(-h * h / (sigma * sigma));
    const double wr = cos(two_pi * (fc - fd) * h), wi = sin(two_pi * (fc - fd) * h);
    const size_t lds = sizeof(unsigned long long) * 2 * (size_t)S;
    hipLaunchKernelGGL(echo_kernel, dim3((unsigned)((int64_t)T * E * F)), dim3(kThreads), lds,
                       reinterpret_cast<hipStream_t>(stream), iq, T, E, S, F, elem, normal, scat, amp, K, c, fs,
                       h, t0, inv2s2, q, wr, wi, two_pi * fd, two_pi * (fc - fd), trunc_sigmas * sigma);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
