/*
 * kfmi.h -- C ABI of the MI355X (gfx950) Kalman-filter track fitting and
 * combinatorial track building library.
 *
 * Method: Cerati et al., "Parallelized Kalman-Filter-Based Reconstruction of
 * Particle Tracks on Many-Core Processors and GPUs".  Track state is the
 * 6-vector (x, y, z, px, py, pz) with a 6x6 covariance and hits are 3-D points
 * with a 3x3 covariance, all in global coordinates (Sec. 2.1); tracking is
 * seeding, building and fitting (Sec. 2); building looks hits up in
 * directionally projective bins per layer and keeps either the best hit or
 * the best N candidates per seed, ranked by number of hits then chi2
 * (Sec. 3, 3.1, 4.3).  The paper prints no formulas: propagation is the
 * helix of a charged particle in a uniform field B = (0, 0, bz) to the first
 * crossing of a cylinder, the covariance is transported with the
 * surface-constrained Jacobian, and updates are the standard Kalman gain
 * update with measurement matrix H = [I3 0].
 *
 * Conventions for every call:
 *   - Arrays are DEVICE pointers, float32, structure of arrays with a leading
 *     dimension `ld` >= n (element stride between components):
 *       state  [6][ld]   (x, y, z, px, py, pz)            cm, GeV/c
 *       cov    [21][ld]  packed lower triangle, k = i(i+1)/2 + j (j <= i),
 *                         indices in the state order
 *       charge int8 [n]  (+1 / -1)
 *       hits   pos [3][ldh], cov [6][ldh] packed (xx, yx, yy, zx, zy, zz)
 *   - The caller owns every buffer.  The library never allocates device
 *     memory except inside kf_ctx_create (none today) and where a call says
 *     so; scratch space is passed in by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *     validate their arguments on the host and then run asynchronously on
 *     that stream.
 *   - Return value: KF_OK or a negative KF_ERR_*; kf_last_error() gives a
 *     message for the calling thread.
 *   - Per-track outcomes go to int32 status words (KF_ST_* bits).  A track
 *     stops at its first fatal bit and its outputs keep the last valid state.
 */
#ifndef KFMI_H
#define KFMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KF_OK 0
#define KF_ERR_INVALID_ARG (-1) /* null pointer, n < 0, ld < n, bad option value */
#define KF_ERR_GEOMETRY (-2)    /* radii not positive / not increasing, too many layers, no geometry set */
#define KF_ERR_DEVICE (-3)      /* a HIP call failed (message kept) */
#define KF_ERR_UNSUPPORTED (-4) /* device is not gfx950 */
#define KF_ERR_WORKSPACE (-5)   /* workspace missing or too small */

#define KF_ST_NO_CROSSING 1 /* the helix does not reach the radius within half a turn */
#define KF_ST_OUT_OF_Z 2    /* crossing beyond the layer's |z| half length */
#define KF_ST_NONFINITE 4   /* non-finite state or covariance */
#define KF_ST_NOT_PD 8      /* residual covariance H C H^T + V not positive definite */
#define KF_ST_STOPPED 16    /* energy loss left no kinetic energy */

#define KF_MAX_LAYERS 32

typedef struct kf_ctx kf_ctx;

/* Barrel geometry: n_layers concentric cylinders of radius r[l] (strictly
 * increasing, > 0) and half length z_half[l]; x_over_x0[l] is the thickness
 * in radiation lengths at normal incidence (0 = no material); uniform field
 * bz tesla; mean energy loss eloss_per_x0 GeV per radiation length; mass of
 * the tracked particle in GeV (used for beta in multiple scattering). */
typedef struct {
  int32_t n_layers;
  float r[KF_MAX_LAYERS];
  float z_half[KF_MAX_LAYERS];
  float x_over_x0[KF_MAX_LAYERS];
  float bz;
  float eloss_per_x0;
  float mass;
} kf_geometry;

/* Create a context bound to HIP device `device`.  Fails with
 * KF_ERR_UNSUPPORTED unless the device is gfx950.  *out is set to NULL on
 * failure.  The context holds host-side state only. */
int32_t kf_ctx_create(kf_ctx** out, int32_t device);
void kf_ctx_destroy(kf_ctx* ctx);
/* Message of the last failed call on this thread (never NULL). */
const char* kf_last_error(void);

/* Copy the geometry into the context (validated; see kf_geometry). */
int32_t kf_set_geometry(kf_ctx* ctx, const kf_geometry* g);

/* Propagation of each track to a cylinder (Sec. 2.1/3: the core KF step that
 * moves a track to the next layer).  In place on state/cov: track i is moved
 * to the first crossing, within less than half a turn of its helix, of the
 * cylinder of radius r_target[i] (or r_scalar if r_target is NULL), and its
 * covariance is transported with the surface-constrained Jacobian.  If
 * material_layer >= 0 that layer's thin-scatterer material (multiple
 * scattering and mean energy loss) is first applied at the track's current
 * position.  z_half > 0 flags crossings with |z| > z_half as OUT_OF_Z
 * (0 = no check).  status[n] receives this call's status bits; tracks with a
 * nonzero status are left unchanged. */
int32_t kf_propagate_to_r(kf_ctx* ctx, int64_t n, int64_t ld, float* state, float* cov, const int8_t* charge,
                          const float* r_target, float r_scalar, float z_half, int32_t material_layer,
                          int32_t* status, void* stream);

/* Kalman update of track i with hit i (Sec. 2.1: 3x3 measurement in global
 * coordinates): r = m - H x, R = H C H^T + V, chi2 = r^T R^-1 r,
 * K = C H^T R^-1, x += K r, C -= K H C.  chi2[n] receives chi2.  With
 * KF_UPDATE_CHI2_ONLY the state is left unchanged (hit scoring).  Tracks with
 * R not positive definite get KF_ST_NOT_PD and are left unchanged. */
#define KF_UPDATE_CHI2_ONLY 1u
int32_t kf_update(kf_ctx* ctx, int64_t n, int64_t ld, float* state, float* cov, const float* hit_pos,
                  const float* hit_cov, int64_t ldh, float* chi2, int32_t* status, uint32_t flags, void* stream);

/* Track fit (Sec. 2, Sec. 4.2: the KF repeated over each track's assigned
 * hits, one track per GPU lane).  For each track, starting from the prior
 * (state_in, cov_in) and for every layer l up to the last layer with a hit:
 * propagate to r[l], update with hit_idx[l][i] if >= 0, then add layer l's
 * material unless l is the last hit layer.  No z acceptance check is made
 * (the hits are assigned).  Outputs: the state and covariance after the last
 * update, chi2 sum, number of hits used, status.  state_out/cov_out may alias
 * state_in/cov_in.  hit_idx is [n_layers][ld_idx] int32 (-1 = no hit),
 * indices into the hit arrays.
 * With KF_FIT_EMIT_RESIDUALS, residual_out [KF_RES_FEATURES+2][ld_res] receives
 * for every track and every layer l >= 1 that has a hit, a record of the
 * prediction before the update (features, then the true-hit offsets dphi, dz);
 * records are written at row index l-1 + (n_layers-1) * i, unused rows get
 * NaN.  (Learned search window training data.) */
#define KF_FIT_EMIT_RESIDUALS 1u
#define KF_RES_FEATURES 8
typedef struct {
  int64_t n, ld;
  const float* state_in;
  const float* cov_in;
  const int8_t* charge;
  const int32_t* hit_idx;
  int64_t ld_idx;
  const float* hit_pos;
  const float* hit_cov;
  int64_t ldh;
  float* state_out;
  float* cov_out;
  float* chi2_out;
  int32_t* nhits_out;
  int32_t* status_out;
  uint32_t flags;
  float* residual_out;
  int64_t ld_res;
  void* stream;
} kf_fit_args;
int32_t kf_fit(kf_ctx* ctx, const kf_fit_args* args);

#ifdef __cplusplus
}
#endif
#endif
