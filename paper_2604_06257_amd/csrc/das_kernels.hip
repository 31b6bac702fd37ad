// gfx950 kernels of the delay-and-sum beamformer.
//
// Work decomposition (one workgroup = one voxel tile of 4 waves x 64 lanes,
// one lane = one voxel slot; grid.y = chunks of FC frames):
//
//   for each element e, transmit t whose tile window is not empty:
//     every lane forms its coefficients (FP64 delay and phase, FP32 result):
//       sample row i0, weight beta, complex C = w exp(+j 2 pi fd tau)
//     the workgroup stages the tile's sample window of channel data into LDS
//       as rows (q[s], q[s+1] - q[s]) for each of the FC frames, frame-major,
//       zero outside the record (interpolation is then one FMA per part)
//     every active lane, for each frame f:
//       (q0, d) = lds[f][i0 - lo]         one ds_read_b128
//       acc[f] += C * (q0 + beta d)       six FP32 FMAs
//   write acc to out[voxel][f]
//
// The channel data is frame-innermost ([T][E][S][F]), so staging reads are
// contiguous across lanes.  Lanes of a wave cover a compact lattice patch
// whose 16-lane rows run along a lateral axis, where the sample index varies
// slowly, so the LDS reads of a row fall in distinct banks.  The sum over
// elements and transmits of each (voxel, frame) is owned by one lane and
// taken in a fixed order: results are deterministic (no atomics).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <climits>

#include "das.h"
#include "das_device.h"
#include "das_internal.h"

namespace das {

// ---------------------------------------------------------------- IQ loads
template <int DT>
struct IQLoad;

template <>
struct IQLoad<DAS_IQ_C64> {
    __device__ static float2 at(const void* base, size_t i) {
        return reinterpret_cast<const float2*>(base)[i];
    }
};

template <>
struct IQLoad<DAS_IQ_C16F> {
    __device__ static float2 at(const void* base, size_t i) {
        const __half2 h = reinterpret_cast<const __half2*>(base)[i];
        return __half22float2(h);
    }
};

template <>
struct IQLoad<DAS_IQ_C16BF> {
    __device__ static float2 at(const void* base, size_t i) {
        const uint32_t u = reinterpret_cast<const uint32_t*>(base)[i];
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    }
};

// Workgroup id -> tile so that each XCD (workgroups are dispatched round-robin
// over the 8 XCDs) works on one contiguous run of tiles: neighbouring tiles
// share channel-data windows, which then stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    const int q = n >> 3, r = n & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// ------------------------------------------------------- window pre-pass
// For every (tile, t, e): first and last sample row used by any active lane.
__global__ __launch_bounds__(kSlots) void window_kernel(PlanDev p, unsigned long long* counts) {
    __shared__ int s_lo[kWaves], s_hi[kWaves], s_cnt[kWaves];
    const das_kparams& kp = p.kp;
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slot = (int64_t)tile * kSlots + threadIdx.x;
    const bool valid = p.slot_vox[slot] >= 0;
    const float vx = p.vx[slot], vy = p.vy[slot], vz = p.vz[slot];
    int n_valid = valid ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) n_valid += __shfl_xor(n_valid, o);
    __shared__ int s_valid[kWaves];
    if (lane == 0) s_valid[wave] = n_valid;
    __syncthreads();
    const int tile_valid = s_valid[0] + s_valid[1] + s_valid[2] + s_valid[3];
    unsigned long long active_sum = 0, processed_sum = 0;
    int max_win = 0;
    for (int e = 0; e < kp.E; ++e) {
        const das_rx rx = das_rx_setup(vx, vy, vz, p.elem[3 * e], p.elem[3 * e + 1], p.elem[3 * e + 2], kp);
        for (int t = 0; t < kp.T; ++t) {
            const das_coef c = das_tx_setup(rx, p.tx[(int64_t)t * kp.n_slots + slot], kp);
            const bool act = valid && c.active;
            int lo = act ? c.i0 : INT_MAX, hi = act ? c.i0 : INT_MIN, cnt = act ? 1 : 0;
            for (int o = 32; o > 0; o >>= 1) {
                lo = min(lo, __shfl_xor(lo, o));
                hi = max(hi, __shfl_xor(hi, o));
                cnt += __shfl_xor(cnt, o);
            }
            if (lane == 0) {
                s_lo[wave] = lo;
                s_hi[wave] = hi;
                s_cnt[wave] = cnt;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int L = s_lo[0], H = s_hi[0], C = s_cnt[0];
                for (int w = 1; w < kWaves; ++w) {
                    L = min(L, s_lo[w]);
                    H = max(H, s_hi[w]);
                    C += s_cnt[w];
                }
                int32_t* win = p.windows + 2 * (((int64_t)tile * kp.T + t) * kp.E + e);
                if (C > 0) {
                    win[0] = L;
                    win[1] = H - L + 1;
                    active_sum += (unsigned long long)C;
                    processed_sum += (unsigned long long)tile_valid;
                    max_win = max(max_win, H - L + 1);
                } else {
                    win[0] = 0;
                    win[1] = 0;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        atomicAdd(&counts[0], active_sum);
        atomicAdd(&counts[1], processed_sum);
        atomicMax(&counts[2], (unsigned long long)max_win);
    }
}

hipError_t launch_windows(const PlanDev& p, unsigned long long* counts_dev, hipStream_t s) {
    if (p.kp.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(window_kernel, dim3(p.kp.n_tiles), dim3(kSlots), 0, s, p, counts_dev);
    return hipGetLastError();
}

// ------------------------------------------------------------- main kernel
// FC frames per workgroup, P = LDS row pitch in 16-byte units (P - 1 rows of
// window per pass; P odd so that frame rows start in different bank groups).
template <int FC, int P, int DT>
__global__ __launch_bounds__(kSlots) void das_kernel(PlanDev p, const void* __restrict__ iq, float2* __restrict__ out) {
    __shared__ float4 lds[FC * P];
    constexpr int kRows = P - 1;
    const das_kparams& kp = p.kp;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int f0 = blockIdx.y * FC;
    const int64_t slot = (int64_t)tile * kSlots + threadIdx.x;
    const int vox = p.slot_vox[slot];
    const float vx = p.vx[slot], vy = p.vy[slot], vz = p.vz[slot];

    float acc_r[FC], acc_i[FC];
#pragma unroll
    for (int f = 0; f < FC; ++f) {
        acc_r[f] = 0.0f;
        acc_i[f] = 0.0f;
    }
    const int32_t* wins = p.windows + 2 * (int64_t)tile * kp.T * kp.E;

    for (int e = 0; e < kp.E; ++e) {
        bool have_rx = false;
        das_rx rx;
        for (int t = 0; t < kp.T; ++t) {
            const int lo0 = wins[2 * (t * kp.E + e)];
            const int nrow = wins[2 * (t * kp.E + e) + 1];
            if (nrow == 0) continue;  // no lane of the tile sees this (t, e)
            if (!have_rx) {
                rx = das_rx_setup(vx, vy, vz, p.elem[3 * e], p.elem[3 * e + 1], p.elem[3 * e + 2], kp);
                have_rx = true;
            }
            const das_coef c = das_tx_setup(rx, p.tx[(int64_t)t * kp.n_slots + slot], kp);
            const bool act = (vox >= 0) && c.active;
            const size_t rec = ((size_t)t * kp.E + e) * (size_t)kp.S;  // record start, in samples
            for (int pass = 0; pass < nrow; pass += kRows) {
                const int lo = lo0 + pass;
                const int n = min(kRows, nrow - pass);
                __syncthreads();  // previous readers of lds are done
                for (int idx = threadIdx.x; idx < n * FC; idx += kSlots) {
                    const int row = idx / FC, f = idx % FC;
                    const int s = lo + row;
                    const int fg = f0 + f;
                    float2 a = make_float2(0.0f, 0.0f), b = make_float2(0.0f, 0.0f);
                    if (fg < kp.F) {
                        if (s >= 0 && s < kp.S) a = IQLoad<DT>::at(iq, (rec + s) * kp.F + fg);
                        if (s + 1 >= 0 && s + 1 < kp.S) b = IQLoad<DT>::at(iq, (rec + s + 1) * kp.F + fg);
                    }
                    lds[f * P + row] = make_float4(a.x, a.y, b.x - a.x, b.y - a.y);
                }
                __syncthreads();
                if (act && c.i0 >= lo && c.i0 < lo + n) {
                    const float4* src = lds + (c.i0 - lo);
#pragma unroll
                    for (int f = 0; f < FC; ++f) {
                        const float4 d = src[f * P];
                        const float tr = fmaf(c.beta, d.z, d.x);
                        const float ti = fmaf(c.beta, d.w, d.y);
                        acc_r[f] = fmaf(c.cr, tr, acc_r[f]);
                        acc_r[f] = fmaf(-c.ci, ti, acc_r[f]);
                        acc_i[f] = fmaf(c.cr, ti, acc_i[f]);
                        acc_i[f] = fmaf(c.ci, tr, acc_i[f]);
                    }
                }
            }
        }
    }
    if (vox >= 0) {
        float2* o = out + (size_t)vox * kp.F;
#pragma unroll
        for (int f = 0; f < FC; ++f)
            if (f0 + f < kp.F) o[f0 + f] = make_float2(acc_r[f], acc_i[f]);
    }
}

template <int FC, int P>
static hipError_t launch_fc(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    const dim3 grid(p.kp.n_tiles, (p.kp.F + FC - 1) / FC);
    float2* o = reinterpret_cast<float2*>(out);
    switch (dtype) {
        case DAS_IQ_C64:
            hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C64>), grid, dim3(kSlots), 0, s, p, iq, o);
            break;
        case DAS_IQ_C16F:
            hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C16F>), grid, dim3(kSlots), 0, s, p, iq, o);
            break;
        default:
            hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C16BF>), grid, dim3(kSlots), 0, s, p, iq, o);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_das(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    if (p.kp.n_tiles == 0) return hipSuccess;
    const int F = p.kp.F;
    // LDS per workgroup: FC * P * 16 bytes (~33 KiB for every variant).
    if (F >= 32) return launch_fc<32, 65>(p, iq, dtype, out, s);
    if (F > 8) return launch_fc<16, 129>(p, iq, dtype, out, s);
    if (F > 4) return launch_fc<8, 257>(p, iq, dtype, out, s);
    if (F > 2) return launch_fc<4, 513>(p, iq, dtype, out, s);
    if (F > 1) return launch_fc<2, 1025>(p, iq, dtype, out, s);
    return launch_fc<1, 2049>(p, iq, dtype, out, s);
}

// ------------------------------------------------- plane-wave arrival table
struct Normals {
    double n[16][3];
};

__global__ void tx_plane_wave_kernel(float* tx, const float* __restrict__ vox, int64_t n_vox, Normals nrm, int32_t t0,
                                     int32_t nt, double inv_c) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    const double x = vox[3 * v], y = vox[3 * v + 1], z = vox[3 * v + 2];
    for (int t = 0; t < nt; ++t) {
        const double a = nrm.n[t][0] * x + nrm.n[t][1] * y + nrm.n[t][2] * z;
        tx[(int64_t)(t0 + t) * n_vox + v] = (float)(a * inv_c);
    }
}

hipError_t launch_tx_plane_wave(float* tx_out, const float* vox_xyz, int64_t n_vox, const double* normals_host,
                                int32_t n_tx, double inv_c, hipStream_t s) {
    if (n_vox == 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n_vox + threads - 1) / threads;
    for (int32_t t0 = 0; t0 < n_tx; t0 += 16) {
        Normals nr;
        const int nt = (n_tx - t0) < 16 ? (n_tx - t0) : 16;
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) nr.n[t][k] = normals_host[3 * (t0 + t) + k];
        hipLaunchKernelGGL(tx_plane_wave_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, tx_out, vox_xyz, n_vox, nr,
                           t0, nt, inv_c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace das
