/*
 * das.h -- C ABI of the MI355X (gfx950) delay-and-sum ultrasound beamformer.
 *
 * The operation (mach paper, Sec. 2.1 "Delay-and-sum beamforming", Sec. 4.3
 * "Algorithmic optimizations", Sec. 4.1 benchmark parameters, Table 4 array
 * shapes): for every voxel v and frame f,
 *
 *   y[v,f] = sum_t sum_e  w(v,e) * L_f(t,e,u) * exp(+j 2 pi fd tau)
 *   tau    = tau_tx[t,v] + |x_v - p_e| / c        (precomputed transmit arrival
 *                                                  + receive delay computed on
 *                                                  the fly, Sec. 4.3)
 *   u      = (tau - t0) * fs                       (fractional sample index)
 *   L_f    = (1-beta) q(i0) + beta q(i0+1),  i0 = floor(u), beta = u - i0,
 *            q(s) = iq[t,e,s,f] inside the record, 0 outside (linear
 *            interpolation, Sec. 4.1; zero padding is this library's reading)
 *   w(v,e) = Tukey_alpha(rho),  rho = 2 f# |(x_v - p_e)_xy| / (z_v - z_e)
 *            (f-number receive apodization, Sec. 4.1; window shape is this
 *            library's reading: w = 0 for rho >= 1 or z_v <= z_e, w = 1 when
 *            f# = 0)
 *
 * Compounding is the plain sum over transmits (Sec. 2.1).  Points processed
 * per call, in the paper's accounting (Eq. 1): V * E * T * F.
 *
 * Conventions
 *   - Every pointer named "device" is GPU memory (hipMalloc / torch CUDA
 *     tensors); "host" pointers are CPU memory.  Arrays are C-contiguous.
 *   - Coordinates are metres, times seconds, frequencies hertz.
 *   - Complex arrays are interleaved (re, im).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream only enqueue work on it; the caller
 *     synchronises.
 *   - Return value: DAS_OK (0) or a negative das_status.  No exception ever
 *     crosses this boundary; das_last_error() returns a thread-local message
 *     for the last failure on the calling thread.
 *   - Argument checks run before any GPU call, so invalid arguments are
 *     reported without touching the device.
 */
#ifndef DAS_H
#define DAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum das_status {
    DAS_OK = 0,
    DAS_EINVAL = -1, /* null pointer, non-finite or out-of-range parameter */
    DAS_ESHAPE = -2, /* a size is negative, zero where it must not be, or too large */
    DAS_EDTYPE = -3, /* unknown IQ dtype */
    DAS_EALIGN = -4, /* a device pointer is not aligned as required */
    DAS_EHIP = -5,   /* a HIP runtime call failed (message has the HIP error) */
    DAS_ENOMEM = -6  /* device or host allocation failed */
};

/* IQ storage types.  All are interleaved complex; arithmetic is FP32 (delays
 * and phases are formed in FP64) whatever the storage type. */
enum das_iq_dtype {
    DAS_IQ_C64 = 0,  /* complex64: 2 x float32, 8 bytes per sample      */
    DAS_IQ_C16F = 1, /* 2 x IEEE binary16, 4 bytes per sample            */
    DAS_IQ_C16BF = 2 /* 2 x bfloat16, 4 bytes per sample                 */
};

/* Acquisition and reconstruction parameters (paper Sec. 3.3: transducer
 * geometry, transmitted wavefronts, centre / demodulation frequency,
 * sampling rate, speed of sound; Sec. 4.1: f-number). */
typedef struct das_params {
    int32_t n_tx;        /* T >= 1: transmits (compounded plane waves)       */
    int32_t n_elem;      /* E >= 1: receive elements (channels)              */
    int32_t n_samples;   /* S >= 1: samples per record; (S + 4200) * F * 8
                            bytes must stay below 2 GiB                      */
    int32_t n_frames;    /* F >= 1: frames (ensemble)                        */
    int64_t n_vox;       /* V >= 0: output points                            */
    double sound_speed;  /* c > 0 [m/s]                                      */
    double fs;           /* IQ sampling rate > 0 [Hz]                        */
    double f_demod;      /* demodulation frequency fd >= 0 [Hz]              */
    double t0;           /* time of sample 0 [s]; sample s is at t0 + s / fs */
    double f_number;     /* f# >= 0; 0 disables apodization                  */
    double tukey_alpha;  /* taper fraction in [0, 1]; 0 = boxcar, 1 = Hann   */
} das_params;

/* Opaque, immutable beamforming plan: geometry, the transmit table and the
 * voxel tiling resident in device memory owned by the plan. */
typedef struct das_plan das_plan;

/* Create a plan (paper Sec. 3.3 steps 1-3: geometry, grid, precomputed
 * transmit arrival times).
 *   out         host: receives the plan handle (set to NULL on failure).
 *   p           host: parameters, copied.
 *   elem_xyz    device float32 [E, 3]: receive-element positions.
 *   vox_xyz     device float32 [V, 3]: output points (any order; a regular
 *               lattice is detected and tiled, otherwise points are grouped
 *               by a space-filling curve).
 *   tx_arrival  device float32 [T, V]: transmit wavefront arrival time at
 *               each point [s] (e.g. from das_tx_plane_wave, or any external
 *               simulator).
 *   stream      hipStream_t used for the uploads and set-up kernels; the call
 *               synchronises it before returning.
 * The plan copies what it needs: the caller may free all inputs afterwards.
 * Allocates device memory proportional to V * (T + 4) + E plus the tiling. */
int das_plan_create(das_plan **out, const das_params *p, const float *elem_xyz,
                    const float *vox_xyz, const float *tx_arrival, void *stream);

/* Beamform one batch (paper Sec. 2.1 / Eq. 1; the timed kernel of Sec. 4.2).
 *   plan   a plan from das_plan_create.
 *   iq     device [T, E, S, F] complex samples of type `dtype`, frame
 *          innermost (Sec. 4.4 frame-contiguous layout); 8-byte aligned for
 *          C64, 4-byte aligned for 16-bit types.
 *   dtype  a das_iq_dtype.
 *   out    device complex64 [V, F] (frame innermost), 8-byte aligned,
 *          fully overwritten; must not alias iq.
 *   stream hipStream_t to enqueue on.
 * Allocates nothing; asynchronous.  A plan may be executed concurrently on
 * several streams (it is read-only). */
int das_execute(const das_plan *plan, const void *iq, int dtype, void *out, void *stream);

/* Beamform without compounding: each transmit's volume separately (the
 * per-plane output layout of the paper's Table 4, i.e. the T = 1 calls of
 * das_execute in one launch).  The receive geometry of a (voxel, element) pair
 * is computed once for all transmits.
 *   iq, dtype, stream  as for das_execute.
 *   out    device complex64 [T, V, F], 8-byte aligned, fully overwritten.
 * Supported when T <= 4 and F <= 2 (the plan's kernel then keeps one set of
 * accumulators per transmit); DAS_ESHAPE otherwise.  Allocates nothing;
 * asynchronous.  The sum over T equals das_execute's output up to the order
 * of the float32 additions. */
int das_execute_per_tx(const das_plan *plan, const void *iq, int dtype, void *out, void *stream);

/* Release a plan and its device memory.  NULL is accepted (no-op).  The
 * caller must ensure no execution using the plan is still in flight. */
int das_plan_destroy(das_plan *plan);

/* Plane-wave transmit arrival table (paper Sec. 3.3 step 3 and Sec. 4.3:
 * arrival time of each transmitted wavefront at each voxel, precomputed once).
 * The wave with unit normal n crosses the array origin at t = 0 and reaches x
 * at (n . x) / c, with n = (sin th cos ph, sin ph, cos th cos ph).
 *   tx_out     device float32 [T, V], written.
 *   vox_xyz    device float32 [V, 3].
 *   angles     host double [T, 2]: (theta, phi) radians per transmit.
 *   n_tx, n_vox, sound_speed: T >= 1, V >= 0, c > 0.
 *   stream     hipStream_t.  Asynchronous; allocates nothing. */
int das_tx_plane_wave(float *tx_out, const float *vox_xyz, int64_t n_vox, const double *angles,
                      int32_t n_tx, double sound_speed, void *stream);

/* Plan statistics (for throughput accounting). */
typedef struct das_plan_info {
    int64_t n_vox;             /* V                                            */
    int64_t n_slots;           /* voxel slots: tiles x 256 lanes               */
    int64_t n_tiles;           /* workgroup tiles                              */
    int64_t total_triples;     /* V * E * T (Eq. 1 points per frame)           */
    int64_t active_triples;    /* (voxel, element, transmit) with w > 0 and the
                                  delayed sample inside the record             */
    int64_t processed_triples; /* (slot, element, transmit) the kernel visits:
                                  valid slots of tiles whose window for (t, e)
                                  is not empty (tile-granular aperture)        */
    int32_t tile_dims[3];      /* lattice points per tile along x, y, z (0 when
                                  the points are not a lattice)                */
    int32_t max_window;        /* largest per-tile sample window (rows)        */
    int32_t kernel_fc;         /* kernel variant: frames per workgroup,        */
    int32_t kernel_pitch;      /*   LDS row pitch (window rows + 1; 0 = the
                                      direct kernel: 1-2 frames per workgroup,
                                      samples read without LDS staging),       */
    int32_t kernel_groups;     /*   element groups of 4 waves per tile         */
} das_plan_info;

/* Fill `info` (host) for `plan`.  Host-only, synchronous. */
int das_plan_query(const das_plan *plan, das_plan_info *info);

/* The voxel tiling das_plan_create uses, computed on host arrays (no GPU
 * call).  Points that form a (possibly partial) regular lattice are cut into
 * tiles of 256 lattice points (2D: 32 lateral x 8 deep, 3D: 8 x 8 x 4), and
 * each tile into four 64-lane waves; other point sets are ordered along a
 * Morton curve and cut into runs of 256.
 *   vox_xyz     host float32 [V, 3], finite.
 *   slot_to_vox host int32 [capacity] or NULL: for each slot (tile-major,
 *               then wave, then lane) the voxel index, or -1 for an empty slot.
 *   capacity    length of slot_to_vox (ignored when it is NULL).
 *   n_slots     host, required: receives n_tiles * 256.
 *   tile_dims   host int32 [3] or NULL: receives the tile shape (0s when not
 *               a lattice).
 * Call with slot_to_vox = NULL to learn n_slots; DAS_ESHAPE if capacity is
 * smaller than n_slots. */
int das_tile_order(const float *vox_xyz, int64_t n_vox, int32_t *slot_to_vox, int64_t capacity,
                   int64_t *n_slots, int32_t *tile_dims);

/* Static text for a status code. */
const char *das_status_string(int status);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *das_last_error(void);

/* ABI version: (major << 16) | minor (this header: 1.4; 1.4 added das_power_doppler_noalloc to das_post.h). */
int das_version(void);

/* The compiled beamforming kernel variants, as (frames per workgroup, LDS row
 * pitch, element groups) triples, pitch 0 being the direct kernel (1 or 2
 * frames per workgroup, no LDS staging); das_plan_info reports which one a
 * plan uses.
 *   fc_pitch_groups  host int32 [3 * capacity] or NULL: receives the first
 *                    min(count, capacity) triples.
 *   capacity         >= 0 (0 with NULL asks for the count only).
 * Returns the number of variants (> 0), or a negative status (DAS_EINVAL).
 * Host-only; no GPU call.
 *
 * das_plan_create picks the variant from the frame count, the largest tile
 * window and the tile count.  For tuning and tests, the environment variable
 * DAS_VARIANT="fc,pitch,groups", read at plan creation, forces a listed
 * variant when fc is at most twice the frames per workgroup the plan would
 * choose (any fc up to 32 when F >= 32); otherwise it is ignored.  Every
 * variant computes the same sums (element groups fold their partial sums in
 * a different order, so results may differ in the last bits). */
int das_kernel_variants(int32_t *fc_pitch_groups, int32_t capacity);

/* The variant das_plan_create picks, from the quantities it picks it by:
 *   n_frames        F >= 1;
 *   max_window      the largest per-tile sample window in rows (>= 0), as
 *                   das_plan_info.max_window reports it;
 *   n_tiles         workgroup tiles (>= 1);
 *   items_per_tile  processed (slot, element, transmit) triples / voxels, i.e.
 *                   the slot-weighted mean count of non-empty windows per tile
 *                   (>= 0; das_plan_info.processed_triples / n_vox);
 *   fc_pitch_groups host int32 [3]: receives (frames per workgroup, LDS pitch,
 *                   element groups).
 * The DAS_VARIANT override (above) applies here as at plan creation.
 * Returns DAS_OK, DAS_EINVAL (NULL output, out-of-range argument) or
 * DAS_ESHAPE (no compiled variant).  Host-only; no GPU call. */
int das_choose_kernel_variant(int32_t n_frames, int32_t max_window, int64_t n_tiles, double items_per_tile,
                              int32_t *fc_pitch_groups);

#ifdef __cplusplus
}
#endif

#endif /* DAS_H */
