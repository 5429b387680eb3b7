/*
 * kf_oracle.h -- FP64 CPU oracle for Kalman-filter track fitting and
 * combinatorial track building (test infrastructure only).
 *
 * Only the test suite, the smoke check and the CPU-baseline timing may load
 * this library.  It shares no code, header or table with the GPU library.
 *
 * Layouts (array-of-structures, row-major, double precision):
 *   state  [n][6]  (x, y, z, px, py, pz)          cm, GeV/c
 *   cov    [n][36] full symmetric 6x6
 *   hits   pos [H][3], cov [H][9] full symmetric 3x3
 *   field  B = (0, 0, bz) tesla; charge +-1
 */
#ifndef KF_ORACLE_H
#define KF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LAYERS 32

/* per-track status bits */
#define OR_NO_CROSSING 1
#define OR_OUT_OF_Z 2
#define OR_NONFINITE 4
#define OR_NOT_PD 8
#define OR_STOPPED 16

typedef struct {
  int32_t n_layers;
  double r[OR_MAX_LAYERS];
  double z_half[OR_MAX_LAYERS];
  double x_over_x0[OR_MAX_LAYERS];
  double bz;
  double eloss_per_x0;
  double mass;
} or_geometry;

/* Propagate one track to the cylinder of radius R (first crossing within less
 * than half a turn of the helix).  s (6) and C (36) are replaced by the state
 * and transported covariance at the crossing on success; J (36, nullable)
 * receives the surface-constrained Jacobian; path (nullable) the transverse
 * path length.  z_half <= 0 disables the z check.  Returns status bits. */
int32_t or_propagate_one(const or_geometry* g, double* s, double* C, int32_t q, double R, double z_half,
                         double* J, double* path);

/* Material of layer `layer` applied to a track sitting on it (thin scatterer):
 * mean energy loss and multiple-scattering variance.  Returns status bits. */
int32_t or_material_one(const or_geometry* g, int32_t layer, double* s, double* C);

/* Kalman update of one track with one 3-D hit.  chi2 receives r^T R^-1 r.
 * If chi2_only, s and C are left unchanged.  Returns status bits. */
int32_t or_update_one(double* s, double* C, const double* hit_pos, const double* hit_cov, double* chi2,
                      int32_t chi2_only);

/* Batched forms over n tracks (AoS).  r_target (nullable) overrides r_scalar per
 * track; material_layer < 0 applies no material.  status[n] written. */
int32_t or_propagate(const or_geometry* g, int64_t n, double* state, double* cov, const int8_t* q,
                     const double* r_target, double r_scalar, double z_half, int32_t material_layer,
                     int32_t* status);
int32_t or_update(int64_t n, double* state, double* cov, const double* hit_pos, const double* hit_cov,
                  double* chi2, int32_t* status, int32_t chi2_only);

/* Track fit: Kalman filter over each track's assigned hits, inside out.
 * hit_idx [n][L] (-1 = no hit on that layer).  The output state and covariance
 * are those after the last update.  Returns 0 or a negative error. */
int32_t or_fit(const or_geometry* g, int64_t n, const double* state_in, const double* cov_in, const int8_t* q,
               const int32_t* hit_idx, const double* hit_pos, const double* hit_cov, double* state_out,
               double* cov_out, double* chi2_out, int32_t* nhits_out, int32_t* status_out);

/* Smoother (Rauch-Tung-Striebel backward pass after the fit).  The forward
 * pass is or_fit's; state_out [n][L][6] and cov_out [n][L][36] receive, for
 * every layer 0 .. last hit layer, the smoothed state at that layer (after its
 * crossing and update, before its material).  Rows after the last hit layer
 * are NaN.  A track whose fit fails (status_out != 0, or_fit's bits) is not
 * smoothed: the rows of the layers its filter completed hold the filtered
 * states, later rows NaN.  Returns 0 or a negative error. */
int32_t or_smooth(const or_geometry* g, int64_t n, const double* state_in, const double* cov_in, const int8_t* q,
                  const int32_t* hit_idx, const double* hit_pos, const double* hit_cov, double* state_out,
                  double* cov_out, int32_t* status_out);
/* Moore-Penrose pseudo-inverse Cp (36) of a 6x6 covariance C whose null space
 * is the radial direction (x, y, 0, 0, 0, 0) of a position on a cylinder.
 * Returns 0 unless C is positive definite on the orthogonal complement. */
int32_t or_surface_pinv(const double* C, double x, double y, double* Cp);
/* One backward step: A = Cf F^T Cp_inv, xs = xf + A (xs_next - xp),
 * Cs = Cf + A (Cs_next - Cp) A^T (all 6-vectors and row-major 6x6). */
void or_rts_step(const double* xf, const double* Cf, const double* F, const double* xp, const double* Cp,
                 const double* Cp_inv, const double* xs_next, const double* Cs_next, double* xs, double* Cs);

/* Hit binning per (event, layer): phi bin i_phi in [0, n_phi), eta bin in
 * [0, n_eta) over the layer's acceptance, bin id = i_eta * n_phi + i_phi.
 * layer_offsets[E*L+1]; bin_offsets[(E*L)*(nb+1)] absolute indices into the
 * sorted order; perm[H] = original index of sorted slot; bin_of[H] (nullable)
 * = bin of each original hit.  Order inside a bin = original index. */
int32_t or_bin_hits(const or_geometry* g, int64_t n_events, const int64_t* layer_offsets, const double* hit_pos,
                    int32_t n_phi, int32_t n_eta, int32_t* bin_offsets, int64_t* perm, int32_t* bin_of);

/* Combinatorial track building (clone-engine semantics: all compatible
 * (candidate, hit) pairs of a seed are ranked, the best max_cands survive).
 *
 * seeds: state [S][6], cov [S][36], q [S], seed_event [S], seed_hits [S][3]
 * (global hit indices recorded on layers 0..2), first_layer.
 * mode 0 = brute force over every hit of the layer, 1 = binned window scan.
 * Outputs: n_cands[S], cand_hits [S][N][L] (global index, -1 hole),
 * cand_chi2 [S][N], cand_nhits [S][N], cand_status [S][N], best_state [S][6],
 * best_cov [S][36], margin_cut[S] (smallest relative distance of any decision
 * quantity from its threshold), margin_rank[S] (smallest relative chi2 gap
 * between rank-adjacent equal-nhits children near the cut-off),
 * hits_examined[S] (chi2 evaluations), margin_window[S] (learned window:
 * smallest relative distance of a compatible hit from the learned box edge),
 * fallbacks[S] (candidate-layers with compatible hits, none of them inside
 * the learned window).  All output pointers but n_cands and cand_hits are nullable. */
typedef struct {
  int32_t max_cands;
  int32_t mode;
  double chi2_cut;
  int32_t n_phi, n_eta;
  double window_margin; /* relative safety margin on the window half-widths */
  /* learned search window (project addition, NULL = plain): network
   * parameters (OR_MLP_PARAMS values, see or_mlp_forward) and the half widths
   * in units of its scales.  A candidate's compatible hits must then also lie
   * within nsigma s_t along the tangential direction and nsigma s_z in z of
   * its prediction; when no hit does, the plain definition applies. */
  const double* mlp_params;
  double learned_nsigma;
  /* optional, for callers that build one set of events in several calls
   * (NULL = computed inside from the hits): the binned mode's bin offsets and
   * permutation as or_bin_hits gives them for this cfg's grid, and per
   * (event, layer) the largest x-y eigenvalue and largest zz entry of the hit
   * covariances, as or_layer_vmax gives them */
  const int32_t* bin_offsets;
  const int64_t* perm;
  const double* layer_vmax;
} or_build_cfg;

/* Per (event, layer): the largest eigenvalue of the x-y block and the largest
 * zz entry of its hits' covariances (full 3x3, row-major), into vmax[2 E L]. */
void or_layer_vmax(const or_geometry* g, int64_t n_events, const int64_t* layer_offsets, const double* hit_cov,
                   double* vmax);

int32_t or_build(const or_geometry* g, const or_build_cfg* cfg, int64_t n_events, const int64_t* layer_offsets,
                 const double* hit_pos, const double* hit_cov, int64_t n_seeds, const int64_t* seed_event,
                 const double* seed_state, const double* seed_cov, const int8_t* seed_q, const int64_t* seed_hits,
                 int32_t first_layer, int32_t* n_cands, int32_t* cand_hits, double* cand_chi2, int32_t* cand_nhits,
                 int32_t* cand_status, double* best_state, double* best_cov, double* margin_cut,
                 double* margin_rank, int64_t* hits_examined, double* margin_window, int64_t* fallbacks);

/* Search-window network 8 -> 64 -> 64 -> 2 with ReLU hidden layers, as the
 * device evaluates it: weights, inputs and hidden activations rounded to
 * bfloat16 (or_bf16), biases to float32, sums in double precision.
 * params: W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]. */
#define OR_MLP_PARAMS 4866
double or_bf16(double x);
void or_mlp_forward(const double* params, const double x[8], double o[2]);
/* Features of a prediction (state, 6x6 covariance) crossing from radius
 * r_from to r_to (z half length zh): q/pT, cot(theta), z/zh, sin of the angle
 * between the transverse momentum and the radial direction, r_from/100,
 * r_to/100, log of the tangential and z standard deviations. */
void or_window_features(const double s[6], const double C[36], int q, double r_from, double r_to, double zh,
                        double f[8]);

#ifdef __cplusplus
}
#endif
#endif
