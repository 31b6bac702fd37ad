/*
 * das_post.h -- C ABI of the post-processing kernels (gfx950).
 *
 * The paper lists the steps that follow a beamforming call: log compression
 * for B-mode images and clutter filtering for Doppler imaging (Sec. 3.3), and
 * states its validation in their terms: Power Doppler pixel errors in dB of
 * power relative to the reference image's peak, B-mode pixel errors in dB of
 * amplitude (Sec. 5).  The clutter filter is the SVD filter of the Doppler work
 * the paper cites there: remove the largest singular components of the
 * Casorati matrix (voxels x frames).
 *
 * Input y is the beamformer's output: complex64 [V][F], frame innermost (the
 * layout das_execute writes).  All pointers are device memory; calls enqueue on
 * `stream` (hipStream_t as void*) and allocate nothing (the caller passes the
 * work buffer).  Results are deterministic.  Return 0 (DAS_OK) or a negative
 * das_status from das.h; the message is das_post_last_error().
 */
#ifndef DAS_POST_H
#define DAS_POST_H

#include <stdint.h>

#include "das.h"

#ifdef __cplusplus
extern "C" {
#endif

/* B-mode: out_db[v][f] = max(20 log10(|y[v][f]| / peak_f), -dynamic_range_db)
 * with peak_f = max_v |y[v][f]| (each frame normalised to its own peak; a zero
 * pixel or an all-zero frame gives -dynamic_range_db).  float32 [V][F] output.
 * work holds das_bmode_work(V, F) floats; on return its last F floats are the
 * per-frame peaks.  DAS_ESHAPE unless V >= 1 and 1 <= F <= 1024; DAS_EINVAL for a
 * non-positive or non-finite dynamic range. */
int das_bmode(const void *y, int64_t V, int F, float dynamic_range_db, float *out_db, float *work,
              int64_t work_floats, void *stream);
int64_t das_bmode_work(int64_t V, int F);

/* Power Doppler with an SVD clutter filter:
 *   pd[v] = sum_f |(C - U_k S_k V_k^H)[v][f]|^2 = |c_v|^2 - sum_{j<k} |c_v . v_j|^2
 * where C = y [V][F], v_j are its right singular vectors in order of decreasing
 * singular value and k = n_clutter (0 <= k <= F; k = 0 gives the frame energy,
 * k = F zero).  For 0 < k < F the k eigenvectors of C^H C with the largest
 * eigenvalues come from a float64 solver (Householder tridiagonalisation, Sturm
 * multisection, twisted-factorisation eigenvectors; a spectrum with repeated
 * eigenvalues among the k largest takes a Jacobi solver instead).  float32 [V]
 * output, float64 arithmetic.  work holds das_power_doppler_work(V, F)
 * doubles, 16-byte aligned (its contents on return are internal).  DAS_ESHAPE unless V >= 1
 * and 1 <= F <= 32; DAS_EINVAL unless 0 <= n_clutter <= F. */
int das_power_doppler(const void *y, int64_t V, int F, int n_clutter, float *pd, double *work, int64_t work_doubles,
                      void *stream);
int64_t das_power_doppler_work(int64_t V, int F);

/* Power Doppler as das_power_doppler, for callers that cannot allocate device
 * memory or pass a work buffer (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): its work lives in a fixed 8.03 MiB
 * device array of the library, one per GPU, kept until the process ends.  The
 * call allocates nothing and takes the same arguments minus the work buffer.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (concurrent streams or threads) race and must be serialised by the caller.
 * The result is bitwise that of das_power_doppler (the array holds the same
 * voxel chunking for every frame count).  The voxel count is not limited
 * (chunks grow with V).  DAS_ESHAPE unless V >= 1 and 1 <= F <= 32; DAS_EINVAL unless
 * 0 <= n_clutter <= F; DAS_EHIP if the array's address cannot be obtained. */
int das_power_doppler_noalloc(const void *y, int64_t V, int F, int n_clutter, float *pd, void *stream);

/* Thread-local message of the last failing call of this header ("" if none). */
const char *das_post_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DAS_POST_H */
