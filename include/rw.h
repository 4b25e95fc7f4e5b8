/*
 * rw.h -- C ABI of the MI355X ray-wave hybrid PSF library (librw.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the
 * differentiable ray-wave forward model of arXiv 2605.15418 ("A general
 * differentiable ray-wave framework for hybrid refractive-diffractive system
 * modeling and optimization") and its hand-written adjoint:
 *
 *   conventional ray trace to the DOE (Results, "Ray-Wave Simulator
 *   Formalism", first paragraph) -> tangent frame and square DOE patch of the
 *   complex transmission A exp(i phi) (second paragraph) -> zero-padded
 *   angular spectrum with the evanescent cut (second paragraph; zero padding
 *   in the patch-size study) -> Monte Carlo secondary wavevectors with the
 *   weights of Eq. 1 drawn from p ~ |U~| or uniform (sampling-density study,
 *   Fig. 3; reparameterised sampling, Fig. 1c) -> conventional trace to the
 *   sensor -> coherent wavelet sum of Eq. 2 -> |U|^2 -> loss of Eq. 5.
 *
 * Conventions for every entry point:
 *  - Lengths are millimetres, wavelengths millimetres.
 *  - Array arguments are DEVICE pointers unless their name ends in _host.
 *    The caller owns every device buffer, including the workspace.  The plan
 *    owns only small constant tables allocated in rw_plan_create.
 *  - Calls are asynchronous on the given HIP stream (hipStream_t passed as
 *    void*; NULL = default stream).  No call synchronises the device except
 *    rw_get_stats.  No C++ exception crosses the ABI.
 *  - Every function returns an rw_status; on error rw_last_error() gives a
 *    thread-local message.  Invalid shapes are rejected at plan creation.
 *  - A plan may be used by one thread at a time.
 *
 * Layouts (row-major):
 *  DOE maps         [H][W]         pixel (iy, ix) centred at (x0 + ix pitch, y0 + iy pitch)
 *  PSF / target     [L][F][Q][Q]   pair p = l * F + f; row = y index, column = x index,
 *                                  pixel (r, c) at psf_center + ((c - Q/2), (r - Q/2)) * psf_pitch
 *  ray order        pair-major, then ray r = iy * rays_side + ix of the launch grid
 *  sample indices   [n_pairs][rays_side^2][n_ssr] int32: bin j = (jx + M/2) * M + (jy + M/2)
 *                   of the shifted M x M spectrum (the inverse-CDF order), -1 where the ray
 *                   emits nothing
 */
#ifndef RW_H
#define RW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RW_OK = 0,
  RW_ERR_INVALID_ARG = 1,   /* null pointer, out-of-range enum, bad value      */
  RW_ERR_SHAPE = 2,         /* sizes the kernels do not support               */
  RW_ERR_STATE = 3,         /* backward before forward, workspace too small   */
  RW_ERR_NONFINITE = 4,     /* NaN / Inf input (rw_config.check_finite)       */
  RW_ERR_OOM = 5,           /* a plan table could not be allocated            */
  RW_ERR_HIP = 6,           /* a HIP runtime call failed                      */
  RW_ERR_UNSUPPORTED = 7    /* a valid request outside what the kernels cover */
} rw_status;

enum { RW_SURF_ASPHERE = 0, RW_SURF_PLANE = 1, RW_SURF_GAUSS = 2 };

/* One refractive surface of the sequential system (even asphere or plane):
 * sag z(r) = c r^2 / (1 + sqrt(1 - (1 + conic) c^2 r^2)) + A4 r^4 + A6 r^6 + A8 r^8 + A10 r^10
 * relative to z_vertex.  n_A, n_B: two-term Cauchy law n = n_A + n_B / lambda_um^2 of the
 * medium AFTER the surface (the medium before the first surface is air, n = 1).
 * semi_aperture <= 0 means no clip.  Exactly one surface carries the DOE (carries_doe = 1):
 * at that surface rays are intersected but not refracted; the DOE emission refracts them. */
typedef struct {
  int kind;
  int carries_doe;
  double z_vertex;
  double curvature;
  double conic;
  double asph[4];           /* A4, A6, A8, A10 */
  double semi_aperture;
  double n_A, n_B;
  /* gauss_width > 0 (kind RW_SURF_GAUSS): the Gaussian-like substrate of the conformal
   * DOE demonstration (Fig. 6b) adds gauss_height (exp(-r^2 / gauss_width^2) - 1) to the
   * sag (zero at the vertex; vertex radius gauss_width^2 / (2 |gauss_height|)). */
  double gauss_height, gauss_width;
} rw_surface;

/* DOE map on the xy projection of its surface (the paper's conformal DOE is defined
 * "as projected to a flat xy-plane"); the map extent is the system stop. */
enum { RW_FIELD_AMP_PHASE = 0, RW_FIELD_TWO_PHASE = 1 };
typedef struct {
  int H, W;
  double pitch;
  double x0, y0;            /* centre of pixel (0, 0) */
  /* 1: a reflective DOE (the conformal demonstration): the secondaries leave with
   * the normal component of their direction flipped, back into the medium before
   * the DOE surface, which must be the last surface; the sensor lies in front of it. */
  int reflective;
  /* RW_FIELD_AMP_PHASE: t = A exp(i phi) from the (doe_phase, doe_amp) maps;
   * RW_FIELD_TWO_PHASE: t = exp(i phi1) + exp(i phi2) (the beam-splitting design),
   * doe_phase holding phi1 and doe_amp phi2, and d_phase / d_amp their gradients. */
  int field;
} rw_doe_desc;

enum { RW_PARAM_CURV = 0, RW_PARAM_CONIC = 1, RW_PARAM_A4 = 2, RW_PARAM_A6 = 3,
       RW_PARAM_A8 = 4, RW_PARAM_A10 = 5, RW_PARAM_GAP = 6 };

/* Lens parameter i sets field `field` of surface `surface` to scale * lens_params[i].
 * GAP: the axial distance from the surface to the next surface (to the sensor after
 * the last one); every later surface and the sensor move with it. */
typedef struct {
  int surface;
  int field;
  double scale;
} rw_param_ref;

enum { RW_SAMPLE_MAG = 0, RW_SAMPLE_UNI = 1, RW_SAMPLE_FULL = 2 };
enum { RW_PREC_FP64 = 0, RW_PREC_MIXED = 1, RW_PREC_FP32 = 2 };
/* Gradient of the Monte Carlo draws (reparameterised sampling, Fig. 1c):
 * G1: the a.e. derivative with the drawn bins held fixed;
 * G1_DETACH: the same with the sampling density p held constant as well (only the
 *     drawn bins' spectrum values carry the gradient); its mean over the draws is
 *     the FULL-mode gradient of any loss linear in the sensor field;
 * G2: Gumbel-softmax straight-through -- per draw the hard one-hot sample keeps its
 *     value while the gradient flows through softmax((log p + z) / tau), z the
 *     replica's Gumbel perturbations regenerated conditioned on the drawn bin; both
 *     the weight and the wavevector are relaxed.  Differs from G1 only for p ~ |U~|
 *     (MAG); needs the sensor directly after the DOE. */
enum { RW_GRAD_G1 = 0, RW_GRAD_G2 = 1, RW_GRAD_G1_DETACH = 2 };

typedef struct {
  int n_lambda;
  const double* lambda_host;        /* [n_lambda] mm                                    */
  int n_field;
  const double* field_tan_host;     /* [n_field][2] (tan theta_x, tan theta_y)          */
  const double* launch_center_host; /* [n_field][2] centre of the launch grid           */
  double launch_z;                  /* launch plane, before the first surface           */
  double launch_half;               /* half side of the square launch grid              */
  int rays_side;                    /* rays per pair = rays_side^2                      */
  double sensor_z;                  /* sensor plane                                     */
  int psf_q;                        /* Q: PSF side in pixels (even)                     */
  double psf_pitch;
  const double* psf_center_host;    /* [n_lambda][n_field][2]                           */
  int patch_p;                      /* P: patch side in DOE samples                     */
  int pad_factor;                   /* M = pad_factor * P                               */
  int n_ssr;                        /* N: secondary rays per incident ray (MAG, UNI)    */
  int sampling;                     /* RW_SAMPLE_*                                      */
  int precision;                    /* RW_PREC_*                                        */
  int batched;                      /* 1: each stage is one launch over all pairs;
                                       0: one launch per pair (plain comparator form)  */
  int spread_width;                 /* NUFFT kernel width w, 0 = precision default      */
  uint64_t seed;                    /* Philox key of the secondary-ray draws            */
  int grad;                         /* RW_GRAD_*                                        */
  double tau;                       /* G2 softmax temperature (> 0)                     */
  /* Patch classes (curvature bound, Eq. 4): besides patch_p, up to three smaller
   * patch sides; each ray takes the largest side D = P pitch with
   * arcsin(D / 2 R_loc) <= curv_eps, R_loc the smallest principal radius of the DOE
   * surface at the hit (the smallest side when none qualifies).  n_patch_class = 0:
   * every ray uses patch_p.  Every class satisfies the M rules of patch_p. */
  int n_patch_class;
  int patch_class_p[3];
  double curv_eps;
  /* 1: rw_forward checks lens_params, the DOE maps and the target for NaN / Inf
   * first (one reduction kernel and a synchronisation of the stream) and returns
   * RW_ERR_NONFINITE without running the pass; 0: no check. */
  int check_finite;
  /* Device bytes for the secondary-ray records of one launch group of pairs (the
   * records as produced, after the super-bin pass and sorted, plus the tiled
   * interpolation's slots and results); 0 = 96 GiB.  Pairs whose records exceed
   * it run in several groups. */
  uint64_t record_budget_bytes;
  /* Adaptive patch sizing (the paper's future work; reading in the design notes):
   * K > 0 local periods.  Each ray also takes the smallest patch class side P with
   * (P pitch)^2 |grad phi|^2 >= (2 pi K)^2 -- the patch spans K periods of the map's
   * local grating -- and the largest where the map is flatter; of this side and the
   * curvature side of Eq. 4 the smaller wins.  |grad phi| at the map pixel nearest
   * the hit (clamped one pixel from the edge): per axis the mean of the two
   * one-pixel differences of doe_phase, each wrapped to [-pi, pi], over the pitch.
   * Needs n_patch_class >= 1 and the amplitude-phase field.  0: off. */
  double bandwidth_periods;
  /* Adaptive ray sampling (the paper's future work; reading in the design notes):
   * 1 = a ray of patch class side P_k draws N_k = max(1, floor(n_ssr P_k^2 / P_0^2))
   * secondaries instead of n_ssr (the Monte Carlo budget per spectrum bin kept across
   * classes; Eq. 1 divides by N_k).  Sample indices keep n_ssr slots per ray, -1
   * beyond N_k.  Needs patch classes and MAG or UNI sampling.  0: n_ssr for every ray. */
  int class_draws;
  /* 1: run-to-run reproducible forward.  The Eq. 2 records are spread as 64-bit
   * fixed-point integers (each tap scaled by 2^s, s fixed by the largest record
   * value and the record count of the launch group, and rounded; sums by integer
   * atomics, exact in any order), so the PSF and the loss of two forwards on the
   * same inputs agree bit for bit.  A tap is rounded to within about n 2^-61 of
   * the largest record value, n the group's record slots.  The forward bytes of
   * rw_plan_workspace_bytes grow by 16 nf^2 per pair of a launch group (nf the
   * spreading grid's side) and a list of slices.  rw_backward,
   * rw_forward_backward and rw_autotune return RW_ERR_UNSUPPORTED for such a plan:
   * their map- and lens-gradient sums are float atomics.  0: the tiled spreading. */
  int deterministic;
} rw_config;

typedef struct rw_plan rw_plan;

/* Counters of the last forward.  Rays that end early (Q14 of the design notes:
 * terminated, kept in the ray order with zero amplitude) are counted by cause. */
typedef struct {
  uint64_t rays_total;          /* incident rays launched                                */
  uint64_t rays_alive;          /* incident rays that reached the DOE inside the stop    */
  uint64_t secondaries;         /* secondary rays that reached the sensor with a weight  */
  uint64_t killed_no_hit;       /* no ray-surface intersection (Newton failed)           */
  uint64_t killed_aperture;     /* outside a surface's semi-aperture                     */
  uint64_t killed_tir;          /* total internal reflection                             */
  uint64_t killed_outside_doe;  /* hit the DOE surface outside the map (the stop)        */
  uint64_t secondaries_lost;    /* drawn secondaries that failed between DOE and sensor  */
  uint64_t evanescent_bins;     /* evanescent bins of the alive rays' spectra ...        */
  uint64_t spectrum_bins;       /* ... out of this many (M^2 per alive ray)              */
  uint64_t rays_by_class[4];    /* alive rays per patch class (largest side first)       */
} rw_stats;

/* Creates a plan: validates shapes, builds constant tables (wavelength-dependent
 * indices, NUFFT deconvolution weights, FFT twiddles) in device memory.
 * All pointers in cfg are host pointers read during this call only.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_SHAPE, RW_ERR_UNSUPPORTED, RW_ERR_OOM, RW_ERR_HIP. */
rw_status rw_plan_create(const rw_surface* surfaces_host, int n_surf, const rw_doe_desc* doe_host,
                         const rw_param_ref* params_host, int n_params, const rw_config* cfg_host,
                         rw_plan** out_plan);

/* Creates the plan of a system with two DOEs in sequence (Formalism, first
 * paragraph: the ray-wave construction extends to several DOEs, since secondary
 * rays are propagated by conventional ray tracing).  Exactly two surfaces carry a
 * DOE: doe1_host describes the first map, doe2_host the second (same H and W, same
 * field mode, neither reflective).  A secondary of the first DOE is traced through
 * the surfaces between the two (which refract) to the second DOE's surface, where
 * it is an incident ray: a plane-wave wavelet whose complex amplitude is its Eq. 1
 * weight and whose phase is its optical path; the second map is its stop.  The
 * second DOE applies the same patch (patch_p, pad_factor: one class), spectrum and
 * sampling (cfg.sampling) and draws n_ssr2 secondaries per incident ray (MAG, UNI),
 * which go on to the sensor: N1 n_ssr2 records per launched ray.
 *  cfg.n_ssr = N1 = n1^2 draws per launched ray at the first DOE (under FULL every
 *  bin: n1 = M).  Secondary i (the draw, or under FULL the bin J) of launched ray
 *  (iy, ix) is ray (iy n1 + i / n1, ix n1 + i % n1) of the second DOE's ray grid of
 *  side rays_side n1 (pair-major like the launch grid); the second DOE's draws take
 *  that ray's index and Philox stream 1 (counter (i >> 2, ray, pair, 1)).
 *  Maps: doe_phase, doe_amp of rw_forward (and the gradients of rw_backward) are
 *  [2][H][W] (first DOE, then second).
 *  Sample indices (replay_idx, idx_out): the first DOE's [n_pairs][rays_side^2][N1]
 *  followed by the second DOE's [n_pairs][(rays_side n1)^2][n_ssr2]; none under FULL.
 *  rw_backward gives both maps' gradients (G1 or G1_DETACH with frozen draws) in
 *  d_phase, d_amp [2][H][W]: the relayed rays' positions and directions follow from
 *  the drawn bins, so the maps act through the wavelets' amplitudes.  Lens gradients
 *  (d_lens with lens parameters), the G2 mode, rw_forward_backward and rw_autotune
 *  return RW_ERR_UNSUPPORTED.
 *  rw_get_stats counts the rays of both DOEs; rw_export_doe_hits gives the second
 *  DOE's incident rays.
 * Errors: as rw_plan_create; RW_ERR_INVALID_ARG (not two DOE surfaces, different
 *         field modes), RW_ERR_SHAPE (different map sizes, n_ssr not a square, grid
 *         side above 32768), RW_ERR_UNSUPPORTED (reflective DOE, patch classes,
 *         M above 128 -- 64 in FP64). */
rw_status rw_plan_create_cascade(const rw_surface* surfaces_host, int n_surf,
                                 const rw_doe_desc* doe1_host, const rw_doe_desc* doe2_host,
                                 int n_ssr2, const rw_param_ref* params_host, int n_params,
                                 const rw_config* cfg_host, rw_plan** out_plan);

/* Device workspace sizes (256-byte aligned buffers):
 *  *fwd_bytes        the workspace of a forward pass that is not followed by a backward;
 *  *bwd_extra_bytes  (may be NULL) what a forward must have on top of fwd_bytes to leave
 *                    the state of rw_backward (the drawn bins, the records' slots) and
 *                    what the backward itself uses.
 * rw_forward with fwd_bytes <= workspace_bytes < fwd_bytes + bwd_extra_bytes runs
 * forward-only: rw_backward then returns RW_ERR_STATE.  The same workspace must be
 * passed to the backward. */
rw_status rw_plan_workspace_bytes(const rw_plan* plan, size_t* fwd_bytes, size_t* bwd_extra_bytes);

/* Forward pass.
 *  lens_params [n_params] float  normalised lens parameters (may be NULL if n_params = 0)
 *  doe_phase, doe_amp [H][W] float
 *  target [L][F][Q][Q] float or NULL: if given, the loss of Eq. 5 (sum over pairs of
 *         ||alpha* I - T||^2 with alpha* = <I,T>/<I,I>) is written to loss_out[0]
 *         and kept for rw_backward; the target must stay valid until then.
 *  psf_out [L][F][Q][Q] float (written)
 *  replay_idx: NULL, or sample indices (layout above) used instead of the Philox draws
 *  idx_out: NULL, or receives the sample indices that were used
 * Errors: RW_ERR_INVALID_ARG (null required pointer), RW_ERR_STATE (workspace smaller than
 *         fwd_bytes), RW_ERR_HIP. */
rw_status rw_forward(rw_plan* plan, const float* lens_params, const float* doe_phase,
                     const float* doe_amp, const float* target, float* psf_out, float* loss_out,
                     void* workspace, size_t workspace_bytes, const int32_t* replay_idx,
                     int32_t* idx_out, void* stream);

/* Forward pass that allocates nothing, for callers that cannot call hipMalloc (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments and results as a forward-only rw_forward, but the workspace is a
 * device array of the library, 256 MiB per GPU (RW_STATIC_SCRATCH_BYTES), held by each
 * GPU the library runs on until the process ends; the caller still passes every input
 * and output.  The call records no events and no graph (profiling and rw_set_graph do
 * not apply to it), and rw_backward cannot follow it (RW_ERR_STATE).  Every call on one
 * GPU uses the same array and leaves its contents to the next call (each forward
 * clears what it needs); calls that overlap on one GPU, from any plan or stream, race.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_UNSUPPORTED (fwd_bytes of the plan above 256 MiB),
 *         RW_ERR_HIP. */
#define RW_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
rw_status rw_forward_static(rw_plan* plan, const float* lens_params, const float* doe_phase,
                            const float* doe_amp, const float* target, float* psf_out,
                            float* loss_out, const int32_t* replay_idx, int32_t* idx_out,
                            void* stream);

/* Backward pass (adjoint G1: the a.e. derivative with the sample indices of the
 * preceding forward held fixed).
 *  dL_dpsf [L][F][Q][Q] float, or NULL to differentiate the Eq. 5 loss of the forward
 *  d_phase, d_amp [H][W] float (overwritten), d_lens [n_params] float (overwritten, may be
 *  NULL if n_params = 0).
 * Must follow rw_forward on the same plan and workspace.
 * Errors: RW_ERR_STATE (no forward, or NULL dL_dpsf without a forward target),
 *         RW_ERR_UNSUPPORTED (lens gradients need a planar DOE followed directly by the sensor),
 *         RW_ERR_HIP. */
rw_status rw_backward(rw_plan* plan, const float* dL_dpsf, float* d_phase, float* d_amp,
                      float* d_lens, void* workspace, size_t workspace_bytes, void* stream);

/* One training step on the loss of Eq. 5 (a target is required): the forward and
 * the backward of rw_forward + rw_backward with dL/dpsf from the loss, fused per
 * launch group of pairs -- each pair's loss and cogradient depend on its own PSF
 * only, so a group's backward runs right after its forward while the group's
 * binned records are still resident, and every group takes the tiled type-2
 * interpolation (with rw_backward only a plan whose records fit one group does).
 * Arguments as in rw_forward / rw_backward (psf_out, loss_out, d_phase, d_amp
 * written; d_lens written when the plan has lens parameters and it is not NULL);
 * the workspace must hold fwd + bwd bytes.  Afterwards rw_backward may still be
 * called on the same workspace (it recomputes the records it needs).  Recorded as
 * one HIP graph under rw_set_graph.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_STATE (workspace), RW_ERR_UNSUPPORTED (lens
 *         gradients through more than 4 surfaces after the DOE), RW_ERR_HIP. */
rw_status rw_forward_backward(rw_plan* plan, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, const float* target, float* psf_out,
                              float* loss_out, float* d_phase, float* d_amp, float* d_lens,
                              void* workspace, size_t workspace_bytes, void* stream);

/* Counters of the last forward (synchronises the stream of that forward). */
rw_status rw_get_stats(rw_plan* plan, rw_stats* out_host);

/* Stage timing.  While enabled, every launch of a stage is bracketed by HIP
 * events recorded on the stream of the call, and rw_get_profile sums their
 * elapsed times (it synchronises those events).  Stages: */
enum { RW_STAGE_TRACE = 0, RW_STAGE_DOE_FWD = 1, RW_STAGE_BIN = 2, RW_STAGE_SPREAD = 3,
       RW_STAGE_GRID_FWD = 4, RW_STAGE_GRID_BWD = 5, RW_STAGE_DOE_BWD = 6,
       RW_STAGE_TRACE_BWD = 7, RW_STAGE_INTERP = 8, RW_N_STAGES = 9 };
typedef struct {
  double ms[RW_N_STAGES];          /* summed kernel time per stage            */
  uint64_t launches[RW_N_STAGES];  /* number of timed launches per stage      */
} rw_profile;
/* enable = 1 starts (and clears) the accumulation, 0 stops it. */
rw_status rw_set_profiling(rw_plan* plan, int enable);
rw_status rw_get_profile(rw_plan* plan, rw_profile* out_host);

/* Launch-shape autotuning of the ray-wave kernels.  Times the forward and the
 * backward DOE kernels on the inputs of the preceding rw_forward (same plan and
 * workspace; the first pairs, about 2^19 rays) for persistent workgroups in
 * {256, 512, 1024, 2048} x spatial ray
 * blocks of {4, 8, 16}^2 rays, keeps the fastest shape of each direction in the
 * plan, and writes it to shape_out[4] (forward workgroups, forward block side,
 * backward workgroups, backward block side) if not NULL.  Synchronises the stream.
 * The trial launches overwrite forward state: call rw_forward again before
 * rw_backward.  Recorded graphs are dropped.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_STATE (no forward on this workspace), RW_ERR_HIP. */
rw_status rw_autotune(rw_plan* plan, void* workspace, size_t workspace_bytes, int* shape_out,
                      void* stream);

/* Applies a launch shape (as rw_autotune writes it: forward workgroups, forward
 * ray-block side, backward workgroups, backward ray-block side), e.g. one cached
 * from an earlier rw_autotune on the same GPU architecture and plan geometry.
 * Recorded graphs are dropped.  Errors: RW_ERR_INVALID_ARG (workgroups outside
 * [1, the plan's maximum], block side not 4, 8 or 16). */
rw_status rw_set_launch_shape(rw_plan* plan, const int* shape_host);

/* Captured launch sequences.  enable = 1: rw_forward and rw_backward record their
 * whole launch sequence into a HIP graph the first time they are called with a given
 * set of pointer arguments (on a capture stream the plan owns) and from then on replay
 * that graph on the caller's stream; a call with other pointers records anew.  Stage
 * profiling covers eager calls only.  enable = 0 drops the recorded graphs.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_HIP (from the call that records). */
rw_status rw_set_graph(rw_plan* plan, int enable);

/* One Adam update (Kingma & Ba, 2015) of n float parameters in place, stream-ordered,
 * for the end-to-end design loop that descends the Eq. 5 loss (Demonstrations,
 * Fig. 5).  With g = grads[i]:
 *   m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   p -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * then p is clamped to [lo, hi] unless lo > hi.  params, grads, m, v: device
 * arrays of n floats owned by the caller (m, v zero before the first step); t >= 1
 * is the step number.  Allocates nothing.
 * Errors: RW_ERR_INVALID_ARG (null array with n > 0, t < 1, beta outside [0, 1),
 *         eps <= 0), RW_ERR_HIP. */
rw_status rw_adam_step(float* params, const float* grads, float* m, float* v, size_t n,
                       float lr, float beta1, float beta2, float eps, int t, float lo,
                       float hi, void* stream);

/* The DOE kernels' patch transform on its own (Formalism: the angular spectrum of
 * a P x P patch zero-padded to M x M), for timing it against other ways of
 * computing the same DFT: in [n][P][P] complex float (interleaved re, im, rows of
 * P), out [n][M][M] complex float, X[ky][kx] = sum_{y,x < P} in[y][x]
 * exp(-2 pi i (ky y + kx x) / M) in natural frequency order.  One 512-thread
 * workgroup per patch with the lane-group LDS FFT of the DOE kernels for M <= 64.
 * Device arrays owned by the caller; stream-ordered; allocates nothing.
 * Errors: RW_ERR_INVALID_ARG, RW_ERR_SHAPE (M not in {16, 32, 64}, P outside
 *         [1, M]), RW_ERR_HIP. */
rw_status rw_patch_dft(int M, int P, long long n, const void* in, void* out, void* stream);

/* Diagnostic export of the incident ray state at the DOE of the last forward:
 * out [n_rays_total][8] double = (px, py, pz, dx, dy, dz, opl, alive). */
rw_status rw_export_doe_hits(const rw_plan* plan, const void* workspace, double* out,
                             void* stream);

rw_status rw_plan_destroy(rw_plan* plan);
const char* rw_status_string(rw_status s);
const char* rw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RW_H */
