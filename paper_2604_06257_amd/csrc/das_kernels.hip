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
//       zero outside the record (interpolation is then one FMA per part);
//       with 8 or more frames per workgroup two such windows share one stage
//       (one fill, one barrier) when their rows fit the buffer together
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
#include <type_traits>
#include <cstdio>
#include <cstdlib>

#include "das.h"
#include "das_device.h"
#include "das_internal.h"

namespace das {

// ---------------------------------------------------------------- IQ loads
// Complex samples are read in groups of FPT consecutive frames of one sample
// row: one 16-, 8- or 4-byte load, kept raw in registers until the LDS write.
template <int BYTES>
struct RawT;
template <>
struct RawT<16> {
    using type = uint4;
};
template <>
struct RawT<8> {
    using type = uint2;
};
template <>
struct RawT<4> {
    using type = uint32_t;
};

template <int DT>
struct IQType {
    static constexpr int kBytes = (DT == DAS_IQ_C64) ? 8 : 4;  // bytes per complex sample
    static constexpr int kVec = 16 / kBytes;                    // complex samples per 16 bytes
};

// Frame j of a raw group, as FP32 (re, im).
template <int DT, typename R>
__device__ __forceinline__ float2 decode(const R& raw, int j) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(&raw);
    if constexpr (DT == DAS_IQ_C64) {
        return make_float2(__uint_as_float(w[2 * j]), __uint_as_float(w[2 * j + 1]));
    } else if constexpr (DT == DAS_IQ_C16F) {
        const uint32_t u = w[j];
        return make_float2(__half2float(__ushort_as_half((unsigned short)(u & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(u >> 16))));
    } else {
        const uint32_t u = w[j];
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    }
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
    const das_lane vl = das_lane_setup(p.vx[slot], p.vy[slot], p.vz[slot], kp);
    int n_valid = valid ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) n_valid += __shfl_xor(n_valid, o);
    __shared__ int s_valid[kWaves];
    if (lane == 0) s_valid[wave] = n_valid;
    __syncthreads();
    const int tile_valid = s_valid[0] + s_valid[1] + s_valid[2] + s_valid[3];
    unsigned long long active_sum = 0, processed_sum = 0;
    int max_win = 0;
    for (int e = 0; e < kp.E; ++e) {
        const das_rx rx = das_rx_setup(vl, p.elemd[3 * e], p.elemd[3 * e + 1], p.elemd[3 * e + 2], kp);
        for (int t = 0; t < kp.T; ++t) {
            const das_coef c = das_tx_setup(rx, das_tx_const(p.tx[(int64_t)t * kp.n_slots + slot], kp), kp);
            const bool act = valid && das_active(rx, c, kp);
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
// FC frames per workgroup; P = LDS row pitch in 16-byte units (P - 1 window
// rows per item, P odd so consecutive frame rows start in different banks);
// G element groups of 4 waves share the tile: group g takes items g, g + G,
// ... and the groups' partial sums are added in a fixed order at the end.
//
// Software pipeline (per group; stage k = one item, or two for the variants that pair):
//   write the window of stage k (registers) to LDS buffer k & 1 as rows
//   (q[s], q[s+1] - q[s]); barrier; issue the global loads of a later stage
//   into the freed registers; coefficients of stage k + G (FP64) while FC
//   frames of one LDS read + six FMAs per item accumulate stage k.
// Unpaired variants load stage k + 2G (two register sets, buffer loads over the
// item's record, only where the window has rows).  Paired variants load stage
// k + G into one register set with a branch-free fill: per-lane global loads of
// either record, or of the plan's zero row for rows outside the record or the
// windows; their scalar loads (items, element coordinates) are issued before
// the barrier, whose wait then covers them.
// Fill: thread -> (frame group of FPT frames, run of RPT rows); it loads RPT + 1
// rows of its frames (each sample once) with 16-byte loads when aligned.
// Waves per SIMD that the LDS footprint allows (the compiler may then spend
// registers on instruction-level parallelism instead of occupancy).
// Variants that stage two items per step are capped so that the second item's registers (coefficients,
// transmit time) fit without spilling: 4 waves (128 VGPRs) for 16 frames, 3 (168) for 32; unpaired 8-frame
// variants run at 6 waves (85 VGPRs: their 16 accumulators do not fit 64; at 5 waves c3 ran 2.5 % slower), or 5
// with several element groups (at 6 they spilled; the c2 grid at 8 frames 0.0363 -> 0.0356 ms), 4-frame ones at 7
// (73 VGPRs: at 8 they spilled, and the c2 grid at 4 frames ran 0.0347 against 0.0292 ms).
template <int FC, int P, int G>
constexpr int das_waves_per_simd() {
    constexpr int bytes = G * 2 * FC * P * 16;
    constexpr int wgs = (160 * 1024) / bytes;
    constexpr int cap = !stage_pairs(FC) ? (FC >= 8 ? (G >= 2 ? 5 : 6) : (FC >= 4 ? 7 : 8)) : (FC >= 32 ? 3 : 4);
    return (wgs * G) < 1 ? 1 : ((wgs * G) > cap ? cap : wgs * G);
}

// NTX > 1: per-transmit output.  Each lane keeps NTX sets of FC accumulators and adds an item into the set of
// its transmit (wave-uniform, so the choice is a scalar branch); out is [T][V][F] (tx_stride = V * F).  Only
// for variants with at most 2 frames per workgroup (registers), and T <= NTX.
template <int FC, int P, int G, int NTX>
constexpr int das_waves_ntx() {
    constexpr int w = das_waves_per_simd<FC, P, G>();
    return (NTX > 1 && FC > 1 && w > 6) ? 6 : w;  // per-transmit accumulators of 2 frames: 80 VGPRs
}

template <int FC, int P, int DT, int G, int NTX = 1>
__global__ __launch_bounds__(kSlots* G) __attribute__((amdgpu_waves_per_eu(das_waves_ntx<FC, P, G, NTX>(),
                                                                            das_waves_ntx<FC, P, G, NTX>())))
void das_kernel(PlanDev p, const void* __restrict__ iq, float2* __restrict__ out, int vec, int64_t tx_stride) {
    static_assert(NTX == 1 || (FC <= 2 && !stage_pairs(FC)), "per-transmit output: FC <= 2");
    constexpr int kRows = P - 1;
    constexpr int kBuf = FC * P;  // float4 per buffer
    constexpr int kEB = IQType<DT>::kBytes;
    constexpr int FPT = FC < IQType<DT>::kVec ? FC : IQType<DT>::kVec;  // frames per fill thread
    constexpr int NFG = FC / FPT;                                      // frame groups per row
    constexpr int RPT = (kRows * NFG + kSlots - 1) / kSlots;           // rows per fill thread
    using Raw = typename RawT<FPT * kEB>::type;
    // the fill threads' runs of RPT rows cover every window row of every frame group
    static_assert(((kRows + RPT - 1) / RPT) * NFG <= kSlots, "fill threads do not cover the stage");
    extern __shared__ float4 lds[];  // [G][2][FC][P]
    const das_kparams& kp = p.kp;
    // workgroup -> (tile, frame chunk): all chunks of the heaviest tiles are dispatched first
    const int nchunk = (p.kp.F + FC - 1) / FC;
    const int unit = p.wg_unit[blockIdx.x];
    const int tile = unit / nchunk;
    const int f0 = (unit % nchunk) * FC;
    // group index is wave-uniform (a group is 4 whole waves); say so to the compiler
    const int grp = (G == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kSlots));
    const int gt = threadIdx.x % kSlots;  // slot within the tile
    const int64_t slot = (int64_t)tile * kSlots + gt;
    const int vox = p.slot_vox[slot];
    const das_lane L = das_lane_setup(p.vx[slot], p.vy[slot], p.vz[slot], kp);
    float4* buf0 = lds + grp * 2 * kBuf;
    float4* buf1 = buf0 + kBuf;
    const int fgrp = gt % NFG, row0 = (gt / NFG) * RPT;
    const int fbase = f0 + fgrp * FPT;

    float acc_r[NTX * FC], acc_i[NTX * FC];
#pragma unroll
    for (int f = 0; f < NTX * FC; ++f) {
        acc_r[f] = 0.0f;
        acc_i[f] = 0.0f;
    }
    const int first = p.item_off[tile];
    const int nitems = p.item_off[tile + 1] - first;  // stages of this tile
    // two items per stage (the second may be empty) for variants that pair, else one
    constexpr int kIS = stage_pairs(FC) ? 2 : 1;
    const int4* items = p.items + kIS * (int64_t)first;
    const int nsteps = (nitems + G - 1) / G;

    // Channel data: record (t, e) holds S rows of F samples.  Rows outside [0, S) are the record's zero padding:
    // a lane reads the plan's zero row for them (and for anything it does not need), so every load is in bounds
    // and the fill has no branch on the thread.
    const int64_t rec_bytes = (int64_t)kp.S * kp.F * kEB;
    const int lane_off = fbase * kEB;  // this thread's frames within a row
    const int row_bytes = kp.F * kEB;
    const bool fill_frames = fbase < kp.F;
    // Loads are addressed as the IQ pointer plus a 64-bit byte offset per lane (the pointer keeps them global
    // loads; an address rebuilt from an integer would make them flat loads, which also count against the LDS
    // wait counter).  The zero row is reached through its offset from the IQ pointer.
    const char* const gbase = reinterpret_cast<const char*>(iq);
    const int64_t zoff = reinterpret_cast<const char*>(p.zrow) - gbase;
    // Byte offset of record (t, e), formed on the scalar unit (items are wave-uniform) and kept opaque, so that a
    // lane's choice between the two records of a stage is a select of two offsets, not a per-lane multiply.
    auto record = [&](const int4& it) {
        const int64_t a = ((int64_t)it.x * kp.E + it.y) * rec_bytes;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)a);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)a >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    // Sample frames [fbase, fbase + FPT) of one row at byte offset o (used when ok, else the zero row): one load
    // when the groups are aligned (kVec: the kernel argument vec, a separate pipeline so that the compiler cannot
    // merge the two forms into 8-byte loads), else one per sample, frames past F reading the zero row (they feed
    // no output).  Conditions are combined with & so that they stay selects, not branches.
    auto load_group = [&](int64_t o, bool ok, Raw& dst, auto vec_tag) {
        if constexpr (decltype(vec_tag)::value) {
            dst = *reinterpret_cast<const Raw*>(gbase + (ok ? o : zoff));
        } else {
            uint32_t* w = reinterpret_cast<uint32_t*>(&dst);
#pragma unroll
            for (int q = 0; q < FPT; ++q) {
                const bool okq = ok & (fbase + q < kp.F);
                if (kEB == 8) {
                    const uint2 v = *reinterpret_cast<const uint2*>(gbase + (okq ? o + q * 8 : zoff));
                    w[2 * q] = v.x;
                    w[2 * q + 1] = v.y;
                } else {
                    w[q] = *reinterpret_cast<const uint32_t*>(gbase + (okq ? o + q * 4 : zoff));
                }
            }
        }
    };
    // Variants without stage pairs (one record per stage, 6 or more waves per SIMD) read through a buffer
    // resource over the item's record, whose range check returns zero for offsets outside it (rows before 0 or
    // past S - 1: the zero padding); only the fill threads with rows in the window load.  (The branch-free fill
    // of the paired variants measured slower here: its per-lane addresses take registers that these variants'
    // occupancy leaves to the multiply-accumulate's LDS reads.)
    const bool full_frames = vec && (fbase + FPT <= kp.F);
    auto load_raw = [&](const __amdgpu_buffer_rsrc_t& rs, int off, Raw& dst) {
        if (full_frames) {
            if constexpr (sizeof(Raw) == 16) {
                dst = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
            } else if constexpr (sizeof(Raw) == 8) {
                dst = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
            } else {
                dst = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
            }
        } else {
            // unaligned rows or the last partial frame group: one sample at a time
            uint32_t* w = reinterpret_cast<uint32_t*>(&dst);
#pragma unroll
            for (int q = 0; q < FPT; ++q) {
                if (kEB == 8) {
                    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off + q * 8, 0, 0);
                    w[2 * q] = (uint32_t)v[0];
                    w[2 * q + 1] = (uint32_t)v[1];
                } else {
                    w[q] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, off + q * 4, 0, 0);
                }
            }
        }
    };
    const int lane_row_off = row0 * row_bytes + lane_off;
    auto load_single = [&](int k, Raw (&raw)[RPT + 1], float& txa, int4& ia, auto one_tx) {
        ia = items[k];
        if constexpr (decltype(one_tx)::value == 0) txa = p.tx[(int64_t)ia.x * kp.n_slots + slot];
        if (row0 < ia.w && fill_frames) {
            const char* rec = gbase + ((int64_t)ia.x * kp.E + ia.y) * rec_bytes;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(rec), (short)0, (int)rec_bytes, 0x00020000);
            const int base = ia.z * row_bytes + lane_row_off;  // wave-uniform product plus a per-lane constant
#pragma unroll
            for (int j = 0; j <= RPT; ++j) load_raw(rs, base + j * row_bytes, raw[j]);
        }
    };
    // Stage rows 0 .. a.w - 1 are item a's window; item b's window starts at row bb(a) = a.w rounded up to a
    // multiple of RPT, so the RPT rows of a fill thread (and the sample after them) come from one record.
    auto bbase = [&](const int4& ia) { return (ia.w + RPT - 1) / RPT * RPT; };
    // The items of stage k (scalar loads).  The pipeline issues them, and the element coordinates below, just
    // before a barrier: that barrier's wait for the LDS writes then covers them, and no scalar load is in flight
    // during the multiply-accumulate (scalar loads return out of order, so one outstanding would turn every
    // wait for an LDS read into a wait for all of them).
    auto fetch_items = [&](int k, int4& ia, int4& ib, int64_t& reca, int64_t& recb) {
        ia = items[kIS * k];
        // without stage pairing the second item is a constant empty one and its code folds away
        ib = stage_pairs(FC) ? items[kIS * k + 1] : make_int4(0, 0, 0, 0);
        reca = record(ia);
        recb = record(ib);
    };
    struct ecrd {
        double x, y, z;
    };
    auto elem_of = [&](const int4& it) {
        const double* e = p.elemd + 3 * it.y;
        return ecrd{e[0], e[1], e[2]};
    };
    // Transmit times and this fill thread's window rows of a stage's items (vector loads, in flight for two
    // steps).  Sample row of stage row r: ia.z + r (first window) or ib.z + r - bb (second window).
    auto issue_loads = [&](const int4& ia, const int4& ib, int64_t reca, int64_t recb, Raw (&raw)[RPT + 1],
                           float& txa, float& txb, auto one_tx, auto vec_tag) {
        if constexpr (decltype(one_tx)::value == 0) {  // with one transmit its time is a per-lane constant
            txa = p.tx[(int64_t)ia.x * kp.n_slots + slot];
            txb = ib.w > 0 ? p.tx[(int64_t)ib.x * kp.n_slots + slot] : 0.0f;
        }
        const int bb = bbase(ia);
        const bool in_b = (ib.w > 0) & (row0 >= bb);
        const bool act = fill_frames & (row0 < (in_b ? bb + ib.w : ia.w));
        const int r0 = (in_b ? ib.z - bb : ia.z) + row0;  // sample row of this thread's first stage row
        const int off0 = r0 * row_bytes + lane_off;  // records are < 2 GiB: 32-bit offsets
        const int64_t rec = in_b ? recb : reca;
#pragma unroll
        for (int j = 0; j <= RPT; ++j)
            load_group(rec + (uint32_t)(off0 + j * row_bytes), act & ((unsigned)(r0 + j) < (unsigned)kp.S), raw[j],
                       vec_tag);
    };
    // LDS frame slot of frame f: frames of one fill thread go to slots NFG
    // apart, so the 16 lanes of a write hit 16 different bank groups.
    // own: whether this thread writes its rows (paired variants: every thread that owns rows, zeros for rows
    // outside the windows, which no lane reads; unpaired: the threads with rows in the window)
    auto store_item = [&](const Raw (&raw)[RPT + 1], float4* buf, bool own) {
        if (own) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                // when RPT does not divide the window rows, the last fill thread's run passes row kRows - 1:
                // rows kRows and up belong to the pad or the next frame slot, which no lane reads but another
                // thread may be writing, so they are not stored
                if (kRows % RPT != 0 && row0 + j >= kRows) break;
#pragma unroll
                for (int q = 0; q < FPT; ++q) {
                    const float2 a = decode<DT>(raw[j], q), b = decode<DT>(raw[j + 1], q);
                    buf[(fgrp + q * NFG) * P + row0 + j] = make_float4(a.x, a.y, b.x - a.x, b.y - a.y);
                }
            }
        }
    };
    // Coefficients of an item for this lane; lanes whose sample row is outside the item's window get zero
    // weights and row 0 (so the MAC runs without branches and adds exact zeros).  A row inside the window is
    // inside the record (windows span the rows of active lanes only); lanes outside the aperture carry w = 0;
    // empty slots compute a valid voxel's sums that are never stored.  base = the item's first stage row.
    // The receive part is kept while consecutive items share the element, the transmit part while they share
    // the transmit (all items, when T = 1).
    //
    // With one transmit every item starts a new element (or continues a split window), so the coefficients
    // are formed without branches from the item alone: the compiler then interleaves the next stage's FP64
    // set-up chain with the current stage's multiply-accumulate, which hides both the chain's latency and the
    // LDS reads'.  With several transmits the receive part is cached across the transmits of an element.
    int last_e = -1, last_t = -1;
    das_rx rx;
    das_txc tc;
    const das_txc tc0 = das_tx_const(p.tx[slot], kp);  // transmit 0
    // one_tx: a std::integral_constant<int, 0 | 1 | 2>: 0 = several transmits (cached receive part), 1 = one
    // transmit and a planar array, 2 = one transmit and elements at several depths.
    // ee: the item's element coordinates when the caller fetched them early (paired variants); the unpaired
    // variants read them here (a scalar load per item, or per element with several transmits).
    auto coef_item = [&](const int4& it, const ecrd& ee, float txv, bool live, int base, auto one_tx) {
        das_coef c;
        if constexpr (decltype(one_tx)::value != 0) {
            const ecrd e = stage_pairs(FC) ? ee : elem_of(it);
            c = das_tx_setup(das_rx_setup_t<decltype(one_tx)::value == 1>(L, e.x, e.y, e.z, kp), tc0, kp);
        } else {
            // marked unlikely (it is taken once per element, every T-th item), so that the compiler keeps
            // the branch rather than forming the receive part for every item
            if (__builtin_expect(it.y != last_e, 0)) {
                const ecrd e = stage_pairs(FC) ? ee : elem_of(it);
                rx = das_rx_setup(L, e.x, e.y, e.z, kp);
                last_e = it.y;
            }
            if (it.x != last_t) {
                tc = das_tx_const(txv, kp);
                last_t = it.x;
            }
            c = das_tx_setup(rx, tc, kp);
        }
        const unsigned d = (unsigned)c.i0 - (unsigned)it.z;
        const bool use = live && d < (unsigned)it.w;
        c.row = use ? (int)d + base : 0;
        c.t = it.x;
        // beta stays: with zero weights the lane adds exact zeros whatever it interpolates
        c.cr = use ? c.cr : 0.0f;
        c.ci = use ? c.ci : 0.0f;
        return c;
    };
    auto mac_into = [&](const das_coef& c, const float4* buf, int a0) {
        const float4* src = buf + c.row;
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            const float4 d = src[((f % FPT) * NFG + f / FPT) * P];
            const float tr = fmaf(c.beta, d.z, d.x);
            const float ti = fmaf(c.beta, d.w, d.y);
            acc_r[a0 + f] = fmaf(c.cr, tr, acc_r[a0 + f]);
            acc_r[a0 + f] = fmaf(-c.ci, ti, acc_r[a0 + f]);
            acc_i[a0 + f] = fmaf(c.cr, ti, acc_i[a0 + f]);
            acc_i[a0 + f] = fmaf(c.ci, tr, acc_i[a0 + f]);
        }
    };
    auto mac_item = [&](const das_coef& c, const float4* buf) {
        if constexpr (NTX == 1) {
            mac_into(c, buf, 0);
        } else {
            const int t = __builtin_amdgcn_readfirstlane(c.t);
#pragma unroll
            for (int j = 0; j < NTX; ++j)
                if (t == j) mac_into(c, buf, j * FC);
        }
    };

    // Step s of this group handles stage k_s = s * G + grp.  Registers of pipeline
    // slot s % 2 hold the window, transmit times and items of k_s (loaded at step
    // s - 2); coefficients of k_s were formed during step s - 1.
    // Both window buffers start zeroed, so a step without a stage (its
    // coefficients are zero) multiplies zeros, never stale or unset LDS.
    for (int i = gt; i < 2 * kBuf; i += kSlots) buf0[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    __syncthreads();
    auto pipeline_pairs = [&](auto one_tx, auto vec_tag) {
        constexpr bool kOne = decltype(one_tx)::value != 0;
        if (nitems == 0) return;  // nothing to add: the sums stay zero
        // Stage k's window is loaded during step k - G into one register set and written to LDS at the start
        // of step k; items are fetched two stages ahead (scalar), element coordinates one stage ahead.  Every
        // step loads and stores a window, so that the loads in flight are the same on every path (the compiler
        // can then wait for exactly the ones it needs); stages past the tile's last repeat the last one's items
        // and carry zero weights.
        const int klast = nitems - 1;
        Raw raw[RPT + 1];
        float tn0 = 0.0f, tn1 = 0.0f;  // transmit times of stage k + G
        int4 n0i, n1i, m0i, m1i;       // items of stages k + G and k + 2G
        int64_t rn0, rn1, rm0, rm1;    // their record offsets
        int4 c0i, c1i;                                         // items of stage grp (prologue)
        int64_t rc0, rc1;
        float tc0_ = 0.0f, tc1_ = 0.0f;
        fetch_items(min(grp, klast), c0i, c1i, rc0, rc1);
        issue_loads(c0i, c1i, rc0, rc1, raw, tc0_, tc1_, one_tx, vec_tag);
        fetch_items(min(grp + G, klast), n0i, n1i, rn0, rn1);
        das_coef none;
        none.i0 = 0;
        none.row = 0;
        none.t = 0;
        none.beta = none.cr = none.ci = 0.0f;
        // The second item's coefficients: with one transmit, always formed (zero weights when the stage has no
        // second item), keeping the step one basic block; otherwise only when the stage has one (a wave-uniform
        // branch: an empty item must not evict the cached receive geometry).
        auto second = [&](const int4& i1, const ecrd& e1, float tx1, bool has, int base) {
            if constexpr (kOne) return coef_item(i1, e1, tx1, has, base, one_tx);
            else return has ? coef_item(i1, e1, tx1, true, base, one_tx) : none;
        };
        das_coef c0 = coef_item(c0i, elem_of(c0i), tc0_, grp < nitems, 0, one_tx);
        bool two = grp < nitems && c1i.w > 0;
        das_coef c1 = second(c1i, elem_of(c1i), tc1_, two, bbase(c0i));
        // One step (stage k): write stage k's window to its buffer; fetch the items of stage k + 2G and the
        // element coordinates of stage k + G; barrier; load stage k + G's window and transmit times; form its
        // coefficients while multiply-accumulating stage k.
        auto step_p = [&](int k, float4* buf) {
            store_item(raw, buf, row0 < kRows);
            const ecrd e0 = elem_of(n0i), e1 = elem_of(n1i);
            fetch_items(min(k + 2 * G, klast), m0i, m1i, rm0, rm1);
            __syncthreads();
            issue_loads(n0i, n1i, rn0, rn1, raw, tn0, tn1, one_tx, vec_tag);
            const bool live = k + G < nitems;
            const das_coef d0 = coef_item(n0i, e0, tn0, live, 0, one_tx);  // stage k + G
            const bool ntwo = live && n1i.w > 0;
            const das_coef d1 = second(n1i, e1, tn1, ntwo, bbase(n0i));
            mac_item(c0, buf);
            if (two) mac_item(c1, buf);
            c0 = d0;
            c1 = d1;
            two = ntwo;
            n0i = m0i;
            n1i = m1i;
            rn0 = rm0;
            rn1 = rm1;
        };
        for (int step = 0; step < nsteps; step += 2) {
            step_p(step * G + grp, buf0);
            if (step + 1 < nsteps) step_p((step + 1) * G + grp, buf1);
        }
    };
    // Unpaired variants: one item per stage, its loads and store only where the window has rows.
    auto pipeline_single = [&](auto one_tx) {
        Raw ra[RPT + 1], rb[RPT + 1];
        float txa = 0.0f, txb = 0.0f;
        const int4 z4 = make_int4(0, 0, 0, 0);
        int4 ia = z4, ib = z4;
        if (grp < nitems) load_single(grp, ra, txa, ia, one_tx);
        if (grp + G < nitems) load_single(grp + G, rb, txb, ib, one_tx);
        const ecrd none_e{0.0, 0.0, 0.0};
        das_coef c0 = coef_item(ia, none_e, txa, grp < nitems, 0, one_tx);
        auto step_s = [&](int k, Raw (&rx_)[RPT + 1], float& tx_, int4& i_, float ty, const int4 j, float4* buf) {
            if (k < nitems) store_item(rx_, buf, row0 < i_.w && fill_frames);
            __syncthreads();
            if (k + 2 * G < nitems) load_single(k + 2 * G, rx_, tx_, i_, one_tx);
            const das_coef n0 = coef_item(j, none_e, ty, k + G < nitems, 0, one_tx);  // stage k + G
            mac_item(c0, buf);
            c0 = n0;
        };
        for (int step = 0; step < nsteps; step += 2) {
            step_s(step * G + grp, ra, txa, ia, txb, ib, buf0);
            if (step + 1 < nsteps) step_s((step + 1) * G + grp, rb, txb, ib, txa, ia, buf1);
        }
    };
    auto run = [&](auto one_tx) {
        if constexpr (stage_pairs(FC)) {
            if (vec) pipeline_pairs(one_tx, std::true_type{});
            else pipeline_pairs(one_tx, std::false_type{});
        } else {
            pipeline_single(one_tx);
        }
    };
    if (kp.T > 1) run(std::integral_constant<int, 0>{});
    else if (kp.planar) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 2>{});
    if (G > 1) {
        // Fixed-order reduction of the groups' partial sums through LDS:
        // ((g0 + g1) + g2) + ...
        float2* red = reinterpret_cast<float2*>(lds);  // [NTX * FC][kSlots]
        for (int g = 1; g < G; ++g) {
            __syncthreads();
            if (grp == g) {
#pragma unroll
                for (int f = 0; f < NTX * FC; ++f) red[f * kSlots + gt] = make_float2(acc_r[f], acc_i[f]);
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int f = 0; f < NTX * FC; ++f) {
                    const float2 v = red[f * kSlots + gt];
                    acc_r[f] += v.x;
                    acc_i[f] += v.y;
                }
            }
        }
    }
    if (grp == 0 && vox >= 0) {
#pragma unroll
        for (int j = 0; j < NTX; ++j) {
            if (NTX > 1 && j >= kp.T) break;
            float2* o = out + j * tx_stride + (size_t)vox * kp.F;
#pragma unroll
            for (int f = 0; f < FC; ++f)
                if (f0 + f < kp.F) o[f0 + f] = make_float2(acc_r[j * FC + f], acc_i[j * FC + f]);
        }
    }
}

// ------------------------------------------------ direct kernel (1-2 frames)
// With one or two frames per workgroup a staged window row serves only the few voxels that read it, once, and the
// stage's fill and barrier cost more than they save.  This kernel reads each lane's two samples (rows i0 and
// i0 + 1 of its frames) straight from the record through the buffer resource, whose range check returns zero
// outside the record (the zero padding), and interpolates them: no LDS staging and no barrier between items.
// Element groups split a tile's items and fold their partial sums in a fixed order at the end, as in
// das_kernel.  The next item's coefficients and loads are issued before the current item's multiply-accumulate.
template <int FC, int DT, int G, int NTX = 1>
__global__ __launch_bounds__(kSlots* G) void das_direct_kernel(PlanDev p, const void* __restrict__ iq,
                                                               float2* __restrict__ out, int vec, int64_t tx_stride) {
    static_assert(FC == 1 || FC == 2, "direct kernel: 1 or 2 frames per workgroup");
    constexpr int kEB = IQType<DT>::kBytes;
    using Raw = typename RawT<FC * kEB>::type;  // FC consecutive frames of one sample row
    const das_kparams& kp = p.kp;
    const int nchunk = (kp.F + FC - 1) / FC;
    const int unit = p.wg_unit[blockIdx.x];
    const int tile = unit / nchunk;
    const int f0 = (unit % nchunk) * FC;
    const int grp = (G == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kSlots));
    const int gt = threadIdx.x % kSlots;
    const int64_t slot = (int64_t)tile * kSlots + gt;
    const int vox = p.slot_vox[slot];
    const das_lane L = das_lane_setup(p.vx[slot], p.vy[slot], p.vz[slot], kp);
    float acc_r[NTX * FC], acc_i[NTX * FC];
#pragma unroll
    for (int f = 0; f < NTX * FC; ++f) {
        acc_r[f] = 0.0f;
        acc_i[f] = 0.0f;
    }
    const int first = p.item_off[tile];
    const int nitems = p.item_off[tile + 1] - first;
    const int4* items = p.items + first;
    const int64_t rec_bytes = (int64_t)kp.S * kp.F * kEB;
    const int row_bytes = kp.F * kEB;
    const int frame_off = f0 * kEB;
    // whole-group loads when every row's group of FC frames is aligned (and complete); else sample by sample
    const bool grouped = vec && (f0 + FC <= kp.F);
    int last_e = -1, last_t = -1;
    das_rx rx;
    das_txc tc;
    const das_txc tc0 = das_tx_const(p.tx[slot], kp);
    auto coef = [&](const int4& it, auto one_tx) {
        das_coef c;
        if constexpr (decltype(one_tx)::value != 0) {
            const double* e = p.elemd + 3 * it.y;
            c = das_tx_setup(das_rx_setup_t<decltype(one_tx)::value == 1>(L, e[0], e[1], e[2], kp), tc0, kp);
        } else {
            if (__builtin_expect(it.y != last_e, 0)) {
                const double* e = p.elemd + 3 * it.y;
                rx = das_rx_setup(L, e[0], e[1], e[2], kp);
                last_e = it.y;
            }
            if (it.x != last_t) {
                tc = das_tx_const(p.tx[(int64_t)it.x * kp.n_slots + slot], kp);
                last_t = it.x;
            }
            c = das_tx_setup(rx, tc, kp);
        }
        // lanes whose row is outside the item's window add exact zeros (rows in a window are in the record)
        const unsigned d = (unsigned)c.i0 - (unsigned)it.z;
        const bool use = d < (unsigned)it.w;
        c.row = use ? c.i0 : -2;  // row -2 reads as zero
        c.t = it.x;
        c.cr = use ? c.cr : 0.0f;
        c.ci = use ? c.ci : 0.0f;
        return c;
    };
    // samples (rows i0 and i0 + 1, this chunk's frames) of an item for this lane
    auto load = [&](const int4& it, const das_coef& c, Raw& q0, Raw& q1) {
        const char* rec = reinterpret_cast<const char*>(iq) + ((int64_t)it.x * kp.E + it.y) * rec_bytes;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(rec), (short)0, (int)rec_bytes, 0x00020000);
        // 32-bit offsets: a negative row wraps to an offset past the record, which reads as zero
        const int off = c.row * row_bytes + frame_off;
        if (grouped) {
            if constexpr (sizeof(Raw) == 16) {
                q0 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
                q1 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b128(rs, off + row_bytes, 0, 0));
            } else if constexpr (sizeof(Raw) == 8) {
                q0 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                q1 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b64(rs, off + row_bytes, 0, 0));
            } else {
                q0 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
                q1 = __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b32(rs, off + row_bytes, 0, 0));
            }
        } else {
            uint32_t* w0 = reinterpret_cast<uint32_t*>(&q0);
            uint32_t* w1 = reinterpret_cast<uint32_t*>(&q1);
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                if (kEB == 8) {
                    const auto a = __builtin_amdgcn_raw_buffer_load_b64(rs, off + f * 8, 0, 0);
                    const auto b = __builtin_amdgcn_raw_buffer_load_b64(rs, off + row_bytes + f * 8, 0, 0);
                    w0[2 * f] = (uint32_t)a[0];
                    w0[2 * f + 1] = (uint32_t)a[1];
                    w1[2 * f] = (uint32_t)b[0];
                    w1[2 * f + 1] = (uint32_t)b[1];
                } else {
                    w0[f] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, off + f * 4, 0, 0);
                    w1[f] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, off + row_bytes + f * 4, 0, 0);
                }
            }
        }
    };
    auto mac_into = [&](const das_coef& c, const Raw& q0, const Raw& q1, int a0) {
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            const float2 a = decode<DT>(q0, f), b = decode<DT>(q1, f);
            const float tr = fmaf(c.beta, b.x - a.x, a.x);
            const float ti = fmaf(c.beta, b.y - a.y, a.y);
            acc_r[a0 + f] = fmaf(c.cr, tr, acc_r[a0 + f]);
            acc_r[a0 + f] = fmaf(-c.ci, ti, acc_r[a0 + f]);
            acc_i[a0 + f] = fmaf(c.cr, ti, acc_i[a0 + f]);
            acc_i[a0 + f] = fmaf(c.ci, tr, acc_i[a0 + f]);
        }
    };
    auto mac = [&](const das_coef& c, const Raw& q0, const Raw& q1) {
        if constexpr (NTX == 1) {
            mac_into(c, q0, q1, 0);
        } else {
            const int t = __builtin_amdgcn_readfirstlane(c.t);
#pragma unroll
            for (int j = 0; j < NTX; ++j)
                if (t == j) mac_into(c, q0, q1, j * FC);
        }
    };
    // Compounded output: items alternate between two register sets (a, b): the samples of one item are loaded
    // while the other's set-up and multiply-accumulate run, and are first used an item later, with no copy between
    // the sets (a copy at the loop's end would wait for the loads just issued).  Every half-step loads (past the
    // last item, the last one again, never accumulated), so that the loads in flight are the same on every path
    // and each multiply-accumulate waits only for its own.  (c2 grid: F = 1 0.0183 -> 0.0173 ms, F = 2 0.0213 ->
    // 0.0208 ms.)  Per-transmit output keeps the one-set loop: with its NTX accumulator sets the two-set form
    // measured 1-2 % slower (c5 geometry, 3 transmits).
    auto run = [&](auto one_tx) {
        if (grp >= nitems) return;
        if constexpr (NTX == 1) {
            const int klast = nitems - 1;
            int4 ita = items[grp], itb;
            das_coef ca = coef(ita, one_tx), cb;
            Raw qa0, qa1, qb0, qb1;
            load(ita, ca, qa0, qa1);
            for (int k = grp; k < nitems; k += 2 * G) {
                itb = items[min(k + G, klast)];
                cb = coef(itb, one_tx);
                load(itb, cb, qb0, qb1);
                // keep the loads above the other set's multiply-accumulate (the scheduler would otherwise sink
                // them below it and give both sets the same registers, which serialises load and use)
                __builtin_amdgcn_sched_barrier(0);
                mac(ca, qa0, qa1);
                if (k + G >= nitems) break;
                ita = items[min(k + 2 * G, klast)];
                ca = coef(ita, one_tx);
                load(ita, ca, qa0, qa1);
                __builtin_amdgcn_sched_barrier(0);
                mac(cb, qb0, qb1);
            }
        } else {
            int4 it = items[grp];
            das_coef c = coef(it, one_tx);
            Raw q0, q1;
            load(it, c, q0, q1);
            for (int k = grp; k < nitems; k += G) {
                das_coef cn = c;
                Raw n0 = q0, n1 = q1;
                if (k + G < nitems) {
                    const int4 itn = items[k + G];
                    cn = coef(itn, one_tx);
                    load(itn, cn, n0, n1);
                }
                mac(c, q0, q1);
                c = cn;
                q0 = n0;
                q1 = n1;
            }
        }
    };
    if (kp.T > 1) run(std::integral_constant<int, 0>{});
    else if (kp.planar) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 2>{});
    if constexpr (G > 1) {
        // fixed-order reduction of the groups' partial sums through LDS: ((g0 + g1) + g2) + ...
        extern __shared__ float4 lds[];
        float2* red = reinterpret_cast<float2*>(lds);  // [NTX * FC][kSlots]
        for (int g = 1; g < G; ++g) {
            __syncthreads();
            if (grp == g) {
#pragma unroll
                for (int f = 0; f < NTX * FC; ++f) red[f * kSlots + gt] = make_float2(acc_r[f], acc_i[f]);
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int f = 0; f < NTX * FC; ++f) {
                    const float2 v = red[f * kSlots + gt];
                    acc_r[f] += v.x;
                    acc_i[f] += v.y;
                }
            }
        }
    }
    if (grp == 0 && vox >= 0) {
#pragma unroll
        for (int j = 0; j < NTX; ++j) {
            if (NTX > 1 && j >= kp.T) break;
            float2* o = out + j * tx_stride + (size_t)vox * kp.F;
#pragma unroll
            for (int f = 0; f < FC; ++f)
                if (f0 + f < kp.F) o[f0 + f] = make_float2(acc_r[j * FC + f], acc_i[j * FC + f]);
        }
    }
}

// P = 0 denotes the direct kernel (no staging; LDS only for the group reduction).
template <int FC, int P, int G, int NTX = 1>
static size_t lds_bytes() {
    const size_t win = (size_t)G * 2 * FC * P * sizeof(float4);
    const size_t red = (size_t)(G > 1 ? 1 : 0) * NTX * FC * kSlots * sizeof(float2);
    return win > red ? win : red;
}

// Vector (16/8/4-byte) loads need every frame group of every row aligned.
template <int FC, int DT>
static int vec_loads_ok(const PlanDev& p, const void* iq) {
    constexpr int kEB = IQType<DT>::kBytes;
    constexpr int FPT = FC < IQType<DT>::kVec ? FC : IQType<DT>::kVec;
    return (p.kp.F % FPT == 0) && (reinterpret_cast<uintptr_t>(iq) % (FPT * kEB) == 0);
}

template <int FC, int P, int G, int NTX = 1>
static hipError_t launch_v(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    const dim3 grid((unsigned)(p.kp.n_tiles * ((p.kp.F + FC - 1) / FC)));
    const dim3 block(kSlots * G);
    const size_t sh = lds_bytes<FC, P, G, NTX>();
    float2* o = reinterpret_cast<float2*>(out);
    const int64_t txs = (int64_t)p.n_vox * p.kp.F;
    if constexpr (P == 0) {
        switch (dtype) {
            case DAS_IQ_C64:
                hipLaunchKernelGGL((das_direct_kernel<FC, DAS_IQ_C64, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C64>(p, iq), txs);
                break;
            case DAS_IQ_C16F:
                hipLaunchKernelGGL((das_direct_kernel<FC, DAS_IQ_C16F, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C16F>(p, iq), txs);
                break;
            default:
                hipLaunchKernelGGL((das_direct_kernel<FC, DAS_IQ_C16BF, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C16BF>(p, iq), txs);
                break;
        }
        return hipGetLastError();
    } else {
        switch (dtype) {
            case DAS_IQ_C64:
                hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C64, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C64>(p, iq), txs);
                break;
            case DAS_IQ_C16F:
                hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C16F, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C16F>(p, iq), txs);
                break;
            default:
                hipLaunchKernelGGL((das_kernel<FC, P, DAS_IQ_C16BF, G, NTX>), grid, block, sh, s, p, iq, o,
                                   vec_loads_ok<FC, DAS_IQ_C16BF>(p, iq), txs);
                break;
        }
        return hipGetLastError();
    }
}

template <int FC, int P, int G, int NTX = 1>
static hipError_t set_lds_limit_ntx() {
    const int sh = (int)lds_bytes<FC, P, G, NTX>();
    hipError_t e;
    if constexpr (P == 0) {
        if ((e = hipFuncSetAttribute((const void*)das_direct_kernel<FC, DAS_IQ_C64, G, NTX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sh)) != hipSuccess)
            return e;
        if ((e = hipFuncSetAttribute((const void*)das_direct_kernel<FC, DAS_IQ_C16F, G, NTX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sh)) != hipSuccess)
            return e;
        return hipFuncSetAttribute((const void*)das_direct_kernel<FC, DAS_IQ_C16BF, G, NTX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, sh);
    } else {
        if ((e = hipFuncSetAttribute((const void*)das_kernel<FC, P, DAS_IQ_C64, G, NTX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sh)) != hipSuccess)
            return e;
        if ((e = hipFuncSetAttribute((const void*)das_kernel<FC, P, DAS_IQ_C16F, G, NTX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sh)) != hipSuccess)
            return e;
        return hipFuncSetAttribute((const void*)das_kernel<FC, P, DAS_IQ_C16BF, G, NTX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, sh);
    }
}

// Per-transmit output exists for the variants with at most 2 frames per workgroup.
constexpr int kPerTx = 4;
template <int FC, int P, int G>
static constexpr bool has_per_tx() {
    return FC <= 2;
}

template <int FC, int P, int G>
static hipError_t set_lds_limit() {
    hipError_t e = set_lds_limit_ntx<FC, P, G, 1>();
    if (e != hipSuccess) return e;
    if constexpr (has_per_tx<FC, P, G>()) return set_lds_limit_ntx<FC, P, G, kPerTx>();
    return hipSuccess;
}

template <int FC, int P, int G>
static hipError_t launch_per_tx_v(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    if constexpr (has_per_tx<FC, P, G>()) return launch_v<FC, P, G, kPerTx>(p, iq, dtype, out, s);
    return hipErrorInvalidValue;
}

// Variants: FC = frames per workgroup (power of two), P = row pitch, G = groups.
// FC * (P - 1) <= 2048 keeps the prefetch at <= 8 float4 per thread and the
// frame stride inside the 16-bit LDS immediate offset.  P = 0: the direct
// kernel (1 or 2 frames per workgroup, samples read without staging).
#define DAS_VARIANTS(X)                                                                              \
    X(32, 41, 3) X(32, 49, 3) X(32, 33, 2) X(32, 65, 2) X(16, 33, 2) X(16, 65, 2) X(16, 129, 2) X(8, 33, 1) X(8, 65, 1)       \
    X(8, 129, 1) X(8, 257, 1) X(4, 33, 1) X(4, 65, 1) X(4, 129, 1) X(4, 257, 1) X(4, 513, 1) X(2, 129, 1)      \
    X(2, 257, 1) X(2, 513, 1) X(2, 1025, 1) X(1, 65, 1) X(1, 129, 1) X(1, 257, 1) X(1, 513, 1) X(1, 1025, 1) X(1, 2049, 1) \
    X(1, 65, 4) X(1, 129, 4) X(1, 257, 4) X(2, 129, 4) X(2, 257, 4) X(4, 65, 4) X(4, 129, 4) X(8, 65, 2) X(8, 65, 4) X(8, 33, 2) X(8, 129, 2) X(16, 65, 4) X(4, 65, 2) \
    X(1, 65, 2) X(1, 129, 2) X(1, 257, 2) X(2, 129, 2) X(2, 257, 2) X(4, 129, 2) X(8, 129, 4)                  \
    X(1, 0, 1) X(1, 0, 2) X(1, 0, 4) X(2, 0, 1) X(2, 0, 2) X(2, 0, 4)

// Variant choice (measured on MI355X with the c1 / c2 / c3 workloads and sweeps of grid size (64-1024 tiles),
// frame count (1-24) and element count (64-256) around the c2 geometry):
//  - one or two frames per workgroup take the direct kernel when tiles carry fewer than 1200 items;
//  - frames are cut into chunks of FC; more chunks mean more workgroups, which
//    the heaviest-first dispatch order balances, at the cost of forming the
//    coefficients once per chunk;
//  - the LDS pitch is the smallest that holds the largest tile window in one
//    piece (a split window costs a whole extra multiply-accumulate pass), and at least 65 rows for
//    8- and 16-frame chunks (33-row variants measured 5-17% slower there);
//  - few tiles (fewer than two per CU at FC = 32) favour 16-frame chunks; 5-8 frames take 8-frame chunks
//    (c3, 8 frames on 3456 tiles: 5.13 ms against 6.84 ms in 4-frame chunks);
//  - with fewer workgroups than CUs (256), the frame chunk is halved until there are enough;
//  - a launch should then hold about 6144 waves (FC <= 4) or 2560 waves (FC >= 8), or 8192 when tiles carry
//    1024 or more (transmit, element) items on average (3D, many elements: a c3 slab of 576 tiles ran 2.09 ms
//    with 9216 waves and 2.67 ms with 4608): element groups (4 waves each) are added until it does, up to 4
//    groups (16 waves per workgroup).
static bool variant_exists(int fc, int pitch, int g) {
#define DAS_HAS(FC_, P_, G_) \
    if (FC_ == fc && P_ == pitch && G_ == g) return true;
    DAS_VARIANTS(DAS_HAS)
#undef DAS_HAS
    return false;
}

// smallest pitch >= min_pitch with a (fc, pitch, g) variant, or -1 (pitch 0 is the direct kernel)
static int pitch_at_least(int fc, int min_pitch, int g) {
    int best = -1;
#define DAS_PIT(FC_, P_, G_) \
    if (FC_ == fc && G_ == g && P_ >= min_pitch && (best < 0 || P_ < best)) best = P_;
    DAS_VARIANTS(DAS_PIT)
#undef DAS_PIT
    return best;
}

Variant choose_variant(int frames, int max_window, int64_t n_tiles, double items_per_tile) {
    int fc;
    if (frames >= 32) fc = (n_tiles < 512) ? 16 : 32;
    else if (frames > 8) fc = 16;
    else if (frames > 4) fc = 8;
    else fc = frames > 2 ? 4 : frames > 1 ? 2 : 1;
    if (const char* env = std::getenv("DAS_VARIANT")) {  // tuning override: "fc,pitch,groups"
        int f = 0, pp = 0, g = 0;
        if (std::sscanf(env, "%d,%d,%d", &f, &pp, &g) == 3 && f <= (frames >= 32 ? 32 : fc * 2) &&
            variant_exists(f, pp, g))
            return Variant{f, pp, g};
    }
    if (fc == 32 && max_window <= 40) return Variant{32, 41, 3};
    if (fc == 32 && max_window <= 48) return Variant{32, 49, 3};
    auto chunks = [&](int f) { return (int64_t)((frames + f - 1) / f); };
    if (fc <= 16)
        while (fc > 1 && n_tiles * chunks(fc) < 256) fc /= 2;
    const int base_g = fc >= 16 ? 2 : 1;
    const int min_pitch = fc >= 8 ? 65 : 0;
    Variant best{0, 0, 0};
    // the direct kernel for 1-2 frames unless tiles carry many items (3D apertures of many elements and
    // transmits): there every item's 16 bytes per lane of gathers outweigh the staged window's few hundred
    // (c2 grid, 1 frame: 0.0233 -> 0.0186 ms; c5 geometry, 11 angles: 5.47 -> 7.23 ms)
    const bool direct = fc <= 2 && items_per_tile < 1200.0 && variant_exists(fc, 0, base_g);
    if (direct) best = {fc, 0, base_g};
#define DAS_PICK(FC_, P_, G_)                                                                       \
    if (!direct && FC_ == fc && G_ == base_g && P_ >= min_pitch && P_ > 0) {                        \
        if (best.fc == 0 || (best.pitch - 1 < max_window && P_ > best.pitch)) best = {FC_, P_, G_}; \
    }
    DAS_VARIANTS(DAS_PICK)
#undef DAS_PICK
    if (best.fc == 0 || best.fc > 16) return best;
    const int64_t target = items_per_tile >= 1024.0 ? 8192 : (best.fc <= 4 ? 6144 : 2560);
    for (int g = base_g; g <= 4; g *= 2) {
        const int p = pitch_at_least(best.fc, best.pitch, g);
        if (p >= 0 && (n_tiles * chunks(best.fc) * 4 * g >= target || g == 4)) return Variant{best.fc, p, g};
    }
    return best;
}

int list_variants(int32_t* out, int capacity) {
    int n = 0;
#define DAS_LIST(FC_, P_, G_)                 \
    {                                         \
        if (out != nullptr && n < capacity) { \
            out[3 * n] = FC_;                 \
            out[3 * n + 1] = P_;              \
            out[3 * n + 2] = G_;              \
        }                                     \
        ++n;                                  \
    }
    DAS_VARIANTS(DAS_LIST)
#undef DAS_LIST
    return n;
}

hipError_t prepare_variant(const PlanDev& p) {
#define DAS_LIMIT(FC_, P_, G_) \
    if (p.fc == FC_ && p.pitch == P_ && p.groups == G_) return set_lds_limit<FC_, P_, G_>();
    DAS_VARIANTS(DAS_LIMIT)
#undef DAS_LIMIT
    return hipErrorInvalidValue;
}

hipError_t launch_das(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    if (p.kp.n_tiles == 0) return hipSuccess;
#define DAS_LAUNCH(FC_, P_, G_) \
    if (p.fc == FC_ && p.pitch == P_ && p.groups == G_) return launch_v<FC_, P_, G_>(p, iq, dtype, out, s);
    DAS_VARIANTS(DAS_LAUNCH)
#undef DAS_LAUNCH
    return hipErrorInvalidValue;
}

bool per_tx_supported(const PlanDev& p) { return p.fc <= 2 && p.kp.T <= kPerTx; }

hipError_t launch_das_per_tx(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s) {
    if (p.kp.n_tiles == 0) return hipSuccess;
#define DAS_LAUNCH_TX(FC_, P_, G_) \
    if (p.fc == FC_ && p.pitch == P_ && p.groups == G_) return launch_per_tx_v<FC_, P_, G_>(p, iq, dtype, out, s);
    DAS_VARIANTS(DAS_LAUNCH_TX)
#undef DAS_LAUNCH_TX
    return hipErrorInvalidValue;
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
