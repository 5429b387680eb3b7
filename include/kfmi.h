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
/* KF_FIT_FP64: keep the track in double-precision registers between layers
 * (HBM stays float32).  Default: float32 registers; updates always compute in
 * double precision. */
#define KF_FIT_FP64 2u
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

/* Smoother (Sec. 2: a Kalman filter followed by a smoother is the final fit of
 * a found track; it gives every layer the estimate from all of the track's
 * hits).  The forward pass is kf_fit's; a Rauch-Tung-Striebel backward pass
 * then runs from the last hit layer inward, with the pseudo-inverse of each
 * prediction's covariance on its cylinder (a prediction has no radial
 * variance).  Same inputs and layouts as kf_fit.  Outputs:
 *   state_out [n_layers][6][ld], cov_out [n_layers][21][ld] (packed): for every
 *     layer up to the track's last hit layer, the smoothed state at that layer
 *     (after its crossing and update, before its material); NaN after it.
 *     A track whose fit fails (status != 0) is not smoothed: the rows of the
 *     layers its filter completed hold the filtered states, later rows NaN.
 *   chi2_out, nhits_out (nullable): as kf_fit;  status_out: kf_fit's bits
 *     (ST_NOT_PD also when a prediction's surface block is not positive
 *     definite in the backward pass; rows above that layer are then smoothed,
 *     the others filtered).
 * The output arrays must not alias the inputs.  flags: KF_FIT_FP64 keeps the
 * filter in double-precision registers; the gain is always formed in double
 * precision.  Errors: KF_ERR_INVALID_ARG (sizes, null arrays, unknown flags),
 * KF_ERR_GEOMETRY (no geometry set). */
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
  void* stream;
} kf_smooth_args;
int32_t kf_smooth(kf_ctx* ctx, const kf_smooth_args* args);


/* ------------------------------------------------------------------------
 * Hit binning (Sec. 3: hits of each layer are placed into directionally
 * projective bins that give a fast look-up of the hits compatible with a
 * track's estimate; Sec. 4.3: on the GPU this reorganisation runs on the
 * device).  For every (event e, layer l) the hits [layer_offsets[e*L+l],
 * layer_offsets[e*L+l+1]) are binned by
 *   i_phi = floor((atan2(y, x) + pi) n_phi / (2 pi)),
 *   i_eta = floor((asinh(z / r_l) + eta_l) n_eta / (2 eta_l)),
 *   eta_l = asinh(z_half_l / r_l),          both clamped to their range,
 * evaluated in double precision on the float32 coordinates; bin id =
 * i_eta * n_phi + i_phi, 1 <= n_phi * n_eta <= 32768.  The sort is stable:
 * inside a bin hits keep their original order.  The grid only decides how
 * finely kf_build's windows select records; a finer grid than the paper's
 * 64 x 16 scans fewer records with identical candidates.
 * Inputs (device): layer_offsets [n_events * n_layers + 1] int64 (ascending,
 * last entry <= ldh), hit_pos [3][ldh], hit_cov [6][ldh].
 * Outputs (device):
 *   bin_offsets [n_events * n_layers][n_phi * n_eta + 1] int32 -- absolute
 *               slot indices, bin b of (e, l) holds slots [o[b], o[b+1]);
 *   perm [ldh] int32 -- original hit index of each slot;
 *   binned [ldh][KF_BINNED_FLOATS] float32 -- the hit record of each slot:
 *               x, y, z, local index (int32 bits, index within its (e, l)),
 *               then the packed covariance (6), then 2 zero pads (48 bytes);
 *   layer_vmax [n_events * n_layers][2] float32 -- largest x-y eigenvalue
 *               and largest zz variance of the layer's hit covariances.
 * Workspace: kf_bin_hits_workspace_size(ldh, n_events) bytes of device
 * memory owned by the caller (per-hit bin ids, and the order in which the
 * (event, layer) pairs are binned: largest first, which does not change the
 * result). */
#define KF_BINNED_FLOATS 12
typedef struct {
  int64_t n_events;
  const int64_t* layer_offsets;
  const float* hit_pos;
  const float* hit_cov;
  int64_t ldh;
  int32_t n_phi, n_eta;
  int32_t* bin_offsets;
  int32_t* perm;
  float* binned;
  float* layer_vmax;
  void* workspace;
  size_t workspace_bytes;
  void* stream;
} kf_bin_args;
size_t kf_bin_hits_workspace_size(int64_t ldh, int64_t n_events);
int32_t kf_bin_hits(kf_ctx* ctx, const kf_bin_args* args);

/* ------------------------------------------------------------------------
 * Combinatorial track building (Sec. 3 "best hit" and combinatorial KF,
 * Sec. 3.1 clone engine, Sec. 4.3 ranking by number of hits then chi2).
 * Every seed starts as one candidate with nhits = 3 and chi2 = 0 at the
 * layer of its third hit.  For each layer l = first_layer .. n_layers-1 every
 * live candidate gets the material of layer l-1, is propagated to layer l
 * (|z| <= z_half), and emits one child per hit of the same event and layer
 * with chi2 increment < chi2_cut (found through the bins overlapping the
 * box |r sin(dphi)| <= sqrt(cut R_tt), |dz| <= sqrt(cut R_zz), which bounds
 * the chi2 ellipsoid) plus one hole child without a hit; a candidate that
 * cannot be propagated (status bits) is carried unchanged as its only child.
 * All children of a seed are ranked by (more hits, smaller chi2, parent
 * rank, hit index, hole last) and the best max_cands survive; only the
 * survivors are updated (clone engine).  max_cands = 1 is the best-hit
 * search.
 * Seeds (device): seed_offsets [n_events+1] int64 (seeds of event e are
 * [o[e], o[e+1])), seed_state [6][ld_seed], seed_cov [21][ld_seed],
 * seed_charge [n_seeds] int8, seed_hits [3][ld_seed] int32 (global hit
 * indices of layers 0..2, copied to the output hit lists).
 * Hits: layer_offsets as for kf_bin_hits and its outputs bin_offsets,
 * binned, layer_vmax with the same n_phi, n_eta.
 * Outputs (device), N = max_cands, S = n_seeds:
 *   n_cands [S] int32; cand_hits [n_layers][S][N] int32 (global hit index,
 *   -1 = no hit; slots k >= n_cands[s] are -1); cand_chi2 [S][N] float32;
 *   cand_nhits [S][N] int32; cand_status [S][N] int32; best_state [6][ld_seed]
 *   and best_cov [21][ld_seed] of the rank-0 candidate (nullable);
 *   counters [KF_BUILD_COUNTERS] uint64 (nullable, accumulated): hits
 *   box-tested, chi2 evaluations, compatible hits, candidate-layer steps,
 *   survivor updates with a hit, learned-window fallbacks to the plain window.
 * Modes: KF_BUILD_TILED (default) runs every layer of a tile of seeds inside
 * one launch, a seed's candidates in consecutive lanes of a wave;
 * KF_BUILD_PERSISTENT launches one grid sized to the device whose waves pull
 * tiles from a device work queue (needs workspace); KF_BUILD_SERIAL gives one
 * lane to each seed, which takes its candidates one after the other (Sec. 4.3's
 * proposed one thread per seed), with the candidates in workspace buffers
 * (plain window, KF_PREC_F32 only; about 240 * max_cands bytes per seed of
 * workspace).  The results do not depend on the mode.
 * Windows: a candidate's compatible hits are those with chi2 < chi2_cut.  The
 * plain window (KF_WINDOW_PLAIN) only limits the bins scanned: it bounds the
 * chi2 < chi2_cut region, so it changes no result.  KF_WINDOW_LEARNED (a
 * project addition) evaluates the search-window network (see below, weights in
 * args->mlp_packed) on the candidate's prediction, giving scales (s_t, s_z);
 * compatible hits must then also lie within learned_nsigma * s_t along the
 * layer's tangential direction and learned_nsigma * s_z in z of the predicted
 * position; if no hit of the layer passes both, the candidate falls back to
 * the plain definition for that layer (counted). */
#define KF_BUILD_COUNTERS 6
#define KF_BUILD_TILED 0
#define KF_BUILD_PERSISTENT 1
#define KF_BUILD_SERIAL 2
#define KF_WINDOW_PLAIN 0
#define KF_WINDOW_LEARNED 1
#define KF_PREC_F32 0
#define KF_PREC_F64 1
typedef struct {
  int32_t max_cands;   /* 1..8 */
  float chi2_cut;      /* > 0 */
  int32_t n_phi, n_eta;
  float window_margin; /* relative margin on the window half widths, >= 0 */
  int32_t mode;        /* KF_BUILD_TILED, KF_BUILD_PERSISTENT or KF_BUILD_SERIAL */
  int32_t window_mode; /* KF_WINDOW_PLAIN or KF_WINDOW_LEARNED */
  int32_t waves_per_block; /* 0 = library choice */
  int32_t blocks_per_cu;   /* persistent mode occupancy, 0 = library choice */
  int32_t precision;       /* KF_PREC_F32 or KF_PREC_F64: candidate registers (HBM is float32 either way) */
  float learned_nsigma;    /* KF_WINDOW_LEARNED: half widths in units of the network's scales, > 0 */
  int32_t seed_order;      /* 1: process each event's seeds grouped by direction (needs workspace); 0: as given.
                              Results do not depend on it. */
} kf_build_cfg;
typedef struct {
  int64_t n_events, n_seeds, ld_seed;
  int32_t first_layer;
  const int64_t* seed_offsets;
  const float* seed_state;
  const float* seed_cov;
  const int8_t* seed_charge;
  const int32_t* seed_hits;
  const int64_t* layer_offsets;
  const int32_t* bin_offsets;
  const float* binned;
  const float* layer_vmax;
  int32_t* n_cands;
  int32_t* cand_hits;
  float* cand_chi2;
  int32_t* cand_nhits;
  int32_t* cand_status;
  float* best_state;
  float* best_cov;
  uint64_t* counters;
  void* workspace;
  size_t workspace_bytes;
  void* stream;
  const void* mlp_packed; /* KF_WINDOW_LEARNED: KF_MLP_PACKED_BYTES from kf_mlp_pack, else ignored */
} kf_build_args;
/* Device workspace of kf_build for this configuration and problem size (0 if
 * none is needed): the persistent work queue and, with seed_order, the
 * direction cells of every event and the seed order.  Contents on entry are
 * irrelevant; kf_build overwrites what it uses. */
size_t kf_build_workspace_size(const kf_build_cfg* cfg, int64_t n_events, int64_t n_seeds);
int32_t kf_build(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* args);
/* ------------------------------------------------------------------------
 * Binning and building from host memory with the transfers overlapped
 * (Sec. 4.2: streams let transfers overlap computation; Sec. 4.3: transfers
 * took about half of the GPU build time).  The events are cut into n_chunks
 * runs of consecutive events with about equal seed counts; each chunk's hits
 * and seeds are copied to the device, binned (kf_bin_hits with cfg's grid) and
 * built (kf_build with cfg), and its outputs are copied into the host output
 * arrays at the chunk's seeds.  Input copies and output copies run on two
 * library streams and the kernels on two more (consecutive chunks alternate,
 * so one chunk's launch tail overlaps the next chunk's kernels), all linked by
 * events, with n_slots device slots for a chunk's inputs and outputs: the
 * copies of one chunk overlap the kernels of others.  The results equal one
 * kf_build over all events (hit indices are global).
 * Inputs (HOST; page-locked memory lets the copies overlap), the layouts of
 * kf_bin_hits and kf_build with leading dimensions n_hits and n_seeds:
 *   layer_offsets [n_events * n_layers + 1] (from 0 to n_hits, every (event,
 *   layer) below 2^24 - 1 hits), hit_pos [3][n_hits], hit_cov [6][n_hits],
 *   seed_offsets [n_events + 1] (from 0 to n_seeds), seed_state
 *   [6][n_seeds], seed_cov [21][n_seeds], seed_charge [n_seeds], seed_hits
 *   [3][n_seeds] (global hit indices).
 * Outputs (HOST), as kf_build's with S = n_seeds: n_cands [S], cand_hits
 *   [n_layers][S][N], cand_chi2, cand_nhits, cand_status [S][N], best_state
 *   [6][S] and best_cov [21][S] (nullable together).  counters (DEVICE,
 *   nullable) accumulate as in kf_build; mlp_packed (DEVICE) as in kf_build.
 * Workspace (DEVICE): kf_build_host_workspace_size() bytes (0 if the offsets
 *   are invalid): n_slots chunk slots sized by the largest chunk, plus the
 *   binning and building scratch of each kernel stream.
 * Ordering: the call's work starts after the work already queued on
 * `stream`, and `stream` waits for all of it: the host outputs are complete
 * once `stream` has been synchronised; inputs, outputs and workspace must stay
 * valid until then.  The host offsets are read during the call. */
typedef struct {
  int64_t n_events, n_seeds, n_hits;
  int32_t first_layer;
  int32_t n_chunks; /* 1 .. n_events */
  int32_t n_slots;  /* 1 .. 4 device chunk slots (3 or 4 overlap copies with two chunks' kernels) */
  const int64_t* layer_offsets;
  const float* hit_pos;
  const float* hit_cov;
  const int64_t* seed_offsets;
  const float* seed_state;
  const float* seed_cov;
  const int8_t* seed_charge;
  const int32_t* seed_hits;
  int32_t* n_cands;
  int32_t* cand_hits;
  float* cand_chi2;
  int32_t* cand_nhits;
  int32_t* cand_status;
  float* best_state;
  float* best_cov;
  uint64_t* counters;
  const void* mlp_packed;
  void* workspace;
  size_t workspace_bytes;
  void* stream;
} kf_build_host_args;
size_t kf_build_host_workspace_size(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_host_args* args);
int32_t kf_build_host(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_host_args* args);

/* kf_build_noalloc: kf_build for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same configuration, arguments, kernels and results as
 * kf_build, but args->workspace and args->workspace_bytes are ignored: the
 * work queue, direction cells and seed order live in a static device array of
 * KF_BUILD_NOALLOC_SCRATCH_BYTES (16 MiB) that each device the library runs on
 * holds until the process ends.  The call allocates nothing.  It returns
 * KF_ERR_WORKSPACE when kf_build_workspace_size(cfg, n_events, n_seeds)
 * exceeds that maximum (with seed_order: about 8 KB per event plus 4 bytes per
 * seed, e.g. 64 events and 3.9 M seeds).  Every call on a device shares that
 * device's array and clears what must start at zero itself; calls that overlap
 * on one device (other streams, other host threads, other contexts) race and
 * must be serialised by the caller. */
#define KF_BUILD_NOALLOC_SCRATCH_BYTES (16u << 20)
int32_t kf_build_noalloc(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* args);


/* ------------------------------------------------------------------------
 * Learned search window (project addition beyond the paper): a network
 * 8 -> 64 -> 64 -> 2 with ReLU hidden layers maps the features of a
 * prediction (see KF_FIT_EMIT_RESIDUALS) to o = (log s_t, log s_z), the
 * scales of the tangential and z offsets of the track's own hit.  Training
 * minimises the mean Gaussian negative log-likelihood
 *     l = sum_k [ r_k^2 exp(-2 o_k) / 2 + o_k ]
 * over records; the optimiser is Adam.  Matrix products run on the bf16
 * matrix cores with float32 accumulation.
 * Parameters (device, float32): KF_MLP_PARAMS values in the order W1 [64][8],
 * b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2] (row-major).
 * kf_mlp_pack converts them to the kernels' layout, a device buffer of
 * KF_MLP_PACKED_BYTES bytes (bf16 matrix-core operand tiles + float32 biases).
 * Records: x [KF_RES_FEATURES][ldx], targets t [2][ldt], outputs y [2][ldy]
 * (float32 device arrays; rows with any non-finite entry are skipped by
 * kf_mlp_grad and give NaN in kf_mlp_forward). */
#define KF_MLP_PARAMS 4866
#define KF_MLP_PACKED_BYTES 23048
int32_t kf_mlp_pack(kf_ctx* ctx, const float* params, void* packed, void* stream);
int32_t kf_mlp_forward(kf_ctx* ctx, int64_t n, const float* x, int64_t ldx, const void* packed, float* y, int64_t ldy,
                       void* stream);
/* Mean loss and its gradient over the n records: grad [KF_MLP_PARAMS]
 * (same order as the parameters), loss [1], count [1] (records used, as a
 * float).  Workspace: kf_mlp_grad_workspace_size() bytes.  Deterministic. */
size_t kf_mlp_grad_workspace_size(void);
int32_t kf_mlp_grad(kf_ctx* ctx, int64_t n, const float* x, int64_t ldx, const float* t, int64_t ldt,
                    const void* packed, float* grad, float* loss, float* count, void* workspace,
                    size_t workspace_bytes, void* stream);
/* One Adam step (bias-corrected, step >= 1) on params from grad, with first
 * and second moments m, v [KF_MLP_PARAMS]; then repacks into packed. */
int32_t kf_mlp_adam(kf_ctx* ctx, float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* packed, void* stream);

/* ------------------------------------------------------------------------
 * Runtime: graph capture and launch autotuning.
 *
 * The paper attributes part of its GPU time to kernel launches and to a
 * single event not filling the device (Sec. 4.2, 4.3).  A graph replays a
 * captured sequence of calls with one launch; the autotuner picks the build
 * launch shape for a problem size.
 *
 * kf_graph_begin starts capturing on `stream` (a created stream, not the
 * default one); every kf_* call issued on that stream by this thread until
 * kf_graph_end is recorded instead of run (arguments, pointers and the
 * geometry are frozen at capture time; none of the captured calls allocates
 * or clears memory with a memset).  A begun capture must always be ended,
 * also after a failed call.  kf_graph_launch replays the graph on any stream.
 * kf_graph_destroy releases it. */
typedef struct kf_graph kf_graph;
int32_t kf_graph_begin(kf_ctx* ctx, void* stream);
int32_t kf_graph_end(kf_ctx* ctx, void* stream, kf_graph** out);
int32_t kf_graph_launch(kf_graph* graph, void* stream);
void kf_graph_destroy(kf_graph* graph);

/* kf_build_autotune: synchronous.  Times kf_build (cfg as given, args as
 * given, counters ignored) over the launch shapes {tiled, persistent,
 * serial} x waves_per_block {1, 2, 4} x blocks_per_cu {1, 2, 3, 4, 8, 12, 14}
 * (persistent only, serial only, if args carries a large enough workspace;
 * serial only for the plain window in single precision), `reps` timed runs
 * each after one warm-up, and
 * writes the fastest mode / waves_per_block / blocks_per_cu into *cfg and its
 * average time into *best_ms (nullable).  The outputs in args are
 * overwritten like by any build.  Results are cached in the context per
 * (device architecture, digest of the kernel sources the library was built
 * from, max_cands, precision, window_mode, power-of-two bucket of n_seeds,
 * bins), so entries loaded from another device or library build never match;
 * a cached entry is returned without timing.  kf_autotune_save / _load
 * write and read the cache as one JSON object per line. */
int32_t kf_build_autotune(kf_ctx* ctx, kf_build_cfg* cfg, const kf_build_args* args, int32_t reps, float* best_ms);
/* kf_fit_autotune: synchronous.  Times kf_fit (args as given, outputs
 * overwritten, reps calls per shape) at 64, 128 and 256 threads per block and
 * keeps the fastest for this problem class (device architecture, kernel source
 * digest, flags, power-of-two bucket of n); later kf_fit calls of that class
 * launch with it.  A cached entry is returned without timing.  Outputs: the
 * block size and its average time per call (nullable). */
int32_t kf_fit_autotune(kf_ctx* ctx, const kf_fit_args* args, int32_t reps, int32_t* best_block, float* best_ms);
int32_t kf_autotune_save(kf_ctx* ctx, const char* path);
int32_t kf_autotune_load(kf_ctx* ctx, const char* path);

#ifdef __cplusplus
}
#endif
#endif
