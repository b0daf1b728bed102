/*
 * gftorf.h -- C ABI of the MI355X (gfx950) differentiable C-ToF Gaussian rasterizer.
 *
 * The library renders, for a batch of time frames of a dynamic scene of 3D
 * Gaussians, the RGB image (paper §3, Eq. 2), the raw continuous-wave
 * time-of-flight quad images (§3, Eq. 4) and the mean depth (§3.1, Eq. 5),
 * and back-propagates upstream image gradients to every Gaussian parameter
 * (supplement C, Eqs. S1-S3, plus the background term those equations omit).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array pointers are DEVICE pointers unless a comment says "host".
 *   The caller owns every buffer; the library never allocates device memory
 *   inside these calls and never synchronises the stream (except
 *   gftorf_read_status), so fwd / bwd / loss / adam can be captured in a
 *   HIP graph.
 * - `stream` is a hipStream_t passed as void* (NULL = the legacy stream).
 * - Return value: GFTORF_OK (0) or a negative error code.  On error nothing
 *   has been enqueued, except for GFTORF_EHIP where a launch failed midway.
 *   gftorf_last_error() returns a thread-local message for the last failure.
 * - Parameter arrays are float32 structure-of-arrays: [3][n] means three
 *   contiguous rows of n floats.
 * - Images are float32 [F][C][H][W], row-major.
 * - Camera convention: world -> camera p = R x + t (R row-major), OpenCV
 *   axes (x right, y down, z forward); pixel (i, j) is sampled at
 *   (i + 0.5, j + 0.5); u = fx X / Z + cx.  The light source is co-located
 *   with the camera (paper §1 assumptions).
 */
#ifndef GFTORF_H
#define GFTORF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GFTORF_OK 0
#define GFTORF_EINVAL (-1)     /* bad argument (NULL, size, unsupported option)        */
#define GFTORF_ENOWS (-2)      /* workspace smaller than gftorf_workspace_size()       */
#define GFTORF_EHIP (-3)       /* a HIP runtime call failed                             */
#define GFTORF_EOVERFLOW (-4)  /* read_status: pairs exceeded max_pairs in last fwd     */

#define GFTORF_MAX_FREQ 4      /* modulation frequencies per call                       */
#define GFTORF_MAX_PHASE 4     /* phase offsets per frequency                           */
#define GFTORF_MAX_QUAD 16     /* GFTORF_MAX_FREQ * GFTORF_MAX_PHASE                    */

/* Gaussian parameters (paper §3: centre, covariance from scale + rotation,
 * opacity, colour, reflectivity).  The time dependence replaces the paper's
 * deformation MLP (§4) by an analytic trajectory:
 *   x(t) = mean + vel t + acc t^2 / 2,
 *   q(t) = quat + (t / 2) (0, omega) (x) quat   (first-order constant rate),
 * and the rotation is M(q) / |q|^2, so quaternions need not be unit length. */
typedef struct gftorf_gaussians {
    int64_t n;
    const float* mean;          /* [3][n] m                                        */
    const float* vel;           /* [3][n] m/s, or NULL (static)                    */
    const float* acc;           /* [3][n] m/s^2, or NULL                           */
    const float* scale;         /* [3][n] linear standard deviations, m            */
    const float* quat;          /* [4][n] (w, x, y, z)                             */
    const float* omega;         /* [3][n] rad/s, or NULL                           */
    const float* opacity_logit; /* [n]   o = sigmoid(logit)                        */
    const float* rgb;           /* [3][n] colour c_k (Eq. 2)                       */
    const float* albedo;        /* [n]   reflectivity r_k (Eq. 3/4)                */
    /* View-dependent colour and reflectivity (paper §3): real spherical
     * harmonics of degree sh_degree (0..3, K = (sh_degree + 1)^2
     * coefficients) at the unit direction from the optical centre to the
     * Gaussian centre, basis order (l, m) = (0,0), (1,-1), (1,0), (1,1), ...,
     * Condon-Shortley phase.  c = max(0, 1/2 + sum_i Y_i k_i) per channel,
     * r = max(0, 1/2 + sum_i Y_i k_i).  A non-NULL array replaces rgb or
     * albedo (which may then be NULL); their gradient outputs are then zero. */
    int32_t sh_degree;          /* 0..3; read only when an sh array is set       */
    int32_t reserved;           /* must be 0                                       */
    const float* sh_rgb;        /* [K][3][n] colour coefficients, or NULL          */
    const float* sh_albedo;     /* [K][n] reflectivity coefficients, or NULL       */
    /* Per-frame centre offsets [n_frames][3][n] (paper §4: the deformation
     * network moves every Gaussian from its canonical centre by delta x_k(t);
     * gftorf_mlp_fwd produces them at the frames' times), or NULL.  Frame f
     * adds delta[f] to the trajectory position, as the last binary64 step of
     * the centre before projection. */
    const float* delta;
} gftorf_gaussians;

/* Gradient outputs, same layout as gftorf_gaussians.  Each non-NULL array is
 * OVERWRITTEN (not accumulated).  A NULL entry is skipped. */
typedef struct gftorf_gaussians_grad {
    float* mean;
    float* vel;
    float* acc;
    float* scale;
    float* quat;
    float* omega;
    float* opacity_logit;
    float* rgb;
    float* albedo;
    float* sh_rgb;              /* [K][3][n], used with gftorf_gaussians.sh_rgb    */
    float* sh_albedo;           /* [K][n], used with gftorf_gaussians.sh_albedo    */
    float* delta;               /* [n_frames][3][n]: dL/d(frame f's centre); valid
                                   with or without input offsets; 0 for culled items */
} gftorf_gaussians_grad;

/* One rendered frame; an ARRAY of these lives in DEVICE memory, so a graph
 * replay can change times, poses and backgrounds between launches.
 *
 * Asynchronous raw quartets (paper §4, Eq. 7): a camera captures the raw
 * quads of one quartet at different times.  A frame with t_hi > t_lo places
 * every Gaussian centre on the straight line between its trajectory
 * positions at the two integer timesteps t_lo and t_hi:
 *   x = ((t_hi - time) x(t_lo) + (time - t_lo) x(t_hi)) / (t_hi - t_lo),
 * which for t_hi - t_lo = 1 is Eq. 7 literally.  The rotation is evaluated
 * at `time` (the unnormalised quaternion is affine in time, so the same
 * interpolation leaves it unchanged).  With t_hi <= t_lo the trajectory is
 * evaluated at `time` directly.
 * quad_mask selects the quad channels (bit freq * n_phase + phase) the frame
 * renders: the forward writes only those channels of `quad`, the backward
 * reads only those channels of d_quad (the others count as zero) and gives
 * zero background gradient to the others.  0 means every channel. */
typedef struct gftorf_frame {
    float R[9];                       /* world -> camera rotation, row-major      */
    float t[3];                       /* world -> camera translation              */
    float fx, fy, cx, cy;             /* pinhole intrinsics, pixels               */
    float time;                       /* s, evaluates the Gaussian trajectories   */
    float bg_rgb[3];                  /* c_bg (Eq. 2)                             */
    float bg_quad[GFTORF_MAX_QUAD];   /* q_bg [n_freq][n_phase] (Eq. 4)           */
    float t_lo, t_hi;                 /* s, Eq. 7 interpolation anchors           */
    uint32_t quad_mask;               /* rendered quad channels, 0 = all          */
    uint32_t reserved;                /* must be 0                                */
} gftorf_frame;

/* Per-call constants (host memory).  The paper states neither the rasterizer
 * constants nor the tile shape; the defaults in the Python binding are
 * alpha_min = 1/255, alpha_max = 0.99, T_min = 1e-4, extent_sigma = 3,
 * dilation = 0.3 px^2, near_z = 0.2 m, source_intensity s = 1, bg_T_power 1. */
typedef struct gftorf_config {
    int32_t width, height;            /* image size, pixels (all frames)          */
    int32_t n_freq;                   /* 1..GFTORF_MAX_FREQ                        */
    int32_t n_phase;                  /* 1..GFTORF_MAX_PHASE                       */
    double freq_hz[GFTORF_MAX_FREQ];  /* modulation frequencies f (Eq. 3)          */
    float phase[GFTORF_MAX_PHASE];    /* quad offsets phi_j (paper §2)             */
    int32_t tile_w, tile_h;           /* 8x8, 16x16 or 32x8                        */
    float alpha_min;                  /* skip a Gaussian with alpha < alpha_min    */
    float alpha_max;                  /* alpha = min(alpha_max, o G)               */
    float T_min;                      /* stop before T (1 - alpha) < T_min         */
    float extent_sigma;               /* support radius in std-devs; <= 0: all tiles */
    float dilation;                   /* added to the 2D covariance diagonal, px^2 */
    float near_z;                     /* cull p_z <= near_z, m                     */
    float source_intensity;           /* s in s r_k / d_k^2 (Eq. 3/4)              */
    int32_t bg_T_power;               /* 1: q_bg T_final (literal Eq. 4); 2: T^2   */
    int64_t max_pairs;                /* capacity of the (tile, Gaussian) lists    */
} gftorf_config;

/* Forward outputs.  rgb [F][3][H][W], quad [F][n_freq*n_phase][H][W] (quad
 * channel index = freq * n_phase + phase), depth [F][H][W]: each may be NULL
 * (not written).  T_final [F][H][W] and n_contrib [F][H][W] are required:
 * the backward pass reads them.
 * Time-of-flight epilogue, per frequency f, from the rendered quads Q_j
 * (background included): S^ = sum_j cos(phi_j) Q_j, C^ = sum_j sin(phi_j) Q_j
 * -- for the offsets 0, pi/2, pi, 3pi/2 exactly Q0 - Qpi and Qpi/2 - Q3pi/2
 * of paper Eq. 1.  phasor [F][n_freq][2][H][W] = (C^, S^), the phasor of
 * Eq. 3; d_tof [F][n_freq][H][W] = c / (4 pi f) (atan2(S^, C^) mod 2 pi)
 * (Eq. 1 with the quadrant resolved); amplitude [F][n_freq][H][W] =
 * |(C^, S^)| / 2 (paper §2).  These three may be NULL; they are outputs only
 * (the backward pass does not differentiate them). */
typedef struct gftorf_outputs {
    float* rgb;
    float* quad;
    float* depth;
    float* T_final;
    int32_t* n_contrib;
    float* phasor;
    float* d_tof;
    float* amplitude;
} gftorf_outputs;

typedef struct gftorf_status {
    int64_t n_pairs;     /* (tile, Gaussian) pairs of the last forward (may exceed max_pairs) */
    int64_t max_pairs;   /* capacity the workspace was carved for                             */
    int32_t overflow;    /* 1 if n_pairs > max_pairs: the last forward is INVALID              */
    int32_t nonfinite;   /* Gaussians culled because an input was NaN / Inf                   */
    int64_t n_evaluated; /* (pixel, list entry) opacity evaluations of the last forward       */
    int64_t n_composited;/* (pixel, list entry) pairs composited by the last forward          */
    /* sticky over every forward on ws since its first 64 bytes were last
     * cleared (by the caller, or gftorf_clear_status): e.g. across replays
     * of a captured optimisation step, whose parameters move between forwards */
    int32_t overflow_seen;   /* 1 if any of those forwards overflowed                      */
    int32_t sort_fault;      /* 1 if the last forward's depth sort gave up waiting on an
                                earlier sort tile (its outputs are then invalid)           */
    int64_t n_pairs_seen;    /* largest pair count among them                              */
} gftorf_status;

/* Bytes of workspace needed for n Gaussians, n_frames frames and cfg
 * (including cfg->max_pairs).  Returns 0 if the arguments are invalid. */
size_t gftorf_workspace_size(int64_t n, int32_t n_frames, const gftorf_config* cfg);

/* Forward rendering of n_frames frames in one batched launch per stage
 * (paper §3 Eqs. 2, 4, 5; every frame carries its own time, so raw quads
 * of a dynamic scene can be rendered at the instants they were captured).
 * Stages: per (frame, Gaussian) projection and tile rectangle -> stable
 * frame-major depth sort of the items -> per-tile Gaussian lists built in
 * depth order (chunk counts, column scan, ordered placement) -> front-to-back
 * compositing, one workgroup per (frame, tile).
 * The workspace `ws` keeps the sorted lists and per-Gaussian records that
 * gftorf_render_bwd needs: pass the same ws, untouched, to the backward.
 * If the pair count exceeds cfg->max_pairs the outputs are invalid and
 * gftorf_read_status reports overflow. */
int gftorf_render_fwd(const gftorf_gaussians* g, const gftorf_frame* frames, int32_t n_frames,
                      const gftorf_config* cfg, const gftorf_outputs* out,
                      void* ws, size_t ws_bytes, void* stream);

/* Backward of gftorf_render_fwd (supplement C: Eq. S2 for RGB and depth,
 * Eq. S3 for the quads, plus the background terms -c_bg T_final/(1-alpha_k)
 * and -p q_bg T_final^p/(1-alpha_k)).  Upstream gradients d_rgb, d_quad,
 * d_depth have the output layouts; NULL means zero.  `saved` must be the
 * outputs of the forward that filled `ws`.  d_bg, if not NULL, receives
 * dL/d(bg_rgb, bg_quad) as [n_frames][3 + n_freq*n_phase] (overwritten).
 * Gradients are exact for the forward's discrete decisions (tile lists,
 * order, skips, stops, clamp) held fixed; FP32 atomics make the result
 * deterministic only up to summation order. */
int gftorf_render_bwd(const gftorf_gaussians* g, const gftorf_frame* frames, int32_t n_frames,
                      const gftorf_config* cfg, const gftorf_outputs* saved,
                      const float* d_rgb, const float* d_quad, const float* d_depth,
                      const gftorf_gaussians_grad* grad, float* d_bg,
                      void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream`, then copies the status of the last forward that
 * used `ws` into *out (host).  Returns GFTORF_EOVERFLOW if it overflowed,
 * GFTORF_EHIP if its depth sort gave up a wait (sort_fault; small batches
 * sort each pass in one launch whose workgroups wait, boundedly, for the
 * digit counts of the frame's earlier sort tiles).
 * n_evaluated / n_composited are summed here from the forward's per-tile
 * counts (zero if no forward has filled this workspace since its first 64
 * bytes were cleared). */
int gftorf_read_status(const void* ws, gftorf_status* out, void* stream);

/* Clears the status header of ws (its first 64 bytes: the last forward's
 * fields and the sticky overflow_seen / n_pairs_seen) with a kernel on
 * `stream`, so it may be captured in a graph.  Errors: GFTORF_EINVAL (NULL
 * or misaligned ws), GFTORF_EHIP. */
int gftorf_clear_status(void* ws, void* stream);

/* Introspection of the forward's binning, for tests and tools: copies
 * (device to device, asynchronously on `stream`) from the workspace of the
 * last forward with the same (n, n_frames, cfg):
 *   pair_key / pair_item: the first min(n_pairs, pair_capacity) sorted pairs,
 *     key = frame * n_tiles + tile (tile = ty * tiles_x + tx), item =
 *     frame * n + gaussian, ascending (key, depth key, gaussian);
 *   depth_key / depth_item: the M = n * n_frames items sorted by their depth
 *     key (float32 bits of the camera-space z; 0xFFFFFFFF for culled items);
 *   item_count: tiles covered per item (0 = culled), item order;
 *   item_rect: [M][2] packed tile rectangles (x_lo | x_hi << 16,
 *     y_lo | y_hi << 16), item order;
 *   tile_ranges: [n_frames * n_tiles][2] [start, end) of every tile list in
 *     the pair arrays.
 * Every destination may be NULL.  Synchronises `stream` to read the pair
 * count. */
int gftorf_copy_lists(const void* ws, int64_t n, int32_t n_frames, const gftorf_config* cfg,
                      uint32_t* pair_key, uint32_t* pair_item, int64_t pair_capacity,
                      uint32_t* depth_key, uint32_t* depth_item, uint32_t* item_count,
                      uint32_t* item_rect, uint32_t* tile_ranges, void* stream);

/* L2 loss (paper Eq. 9, L2 part): for f < n_frames, with target frame
 * s = frame_index[f] (device int32 [n_frames], or NULL for s = f):
 *   loss += weight * mean((pred[f] - targets[s])^2)   over all f and elements,
 *   grad[f] = weight * 2 (pred[f] - targets[s]) / (n_frames * elems_per_frame).
 * pred, grad: [n_frames][elems_per_frame]; targets: [*][elems_per_frame];
 * loss: device float, ADDED to (clear it with gftorf_fill_f32). */
int gftorf_l2_loss_grad(const float* pred, const float* targets, const int32_t* frame_index,
                        int32_t n_frames, int64_t elems_per_frame, float weight,
                        float* grad, float* loss, void* stream);

/* One parameter group of gftorf_adam_step. */
typedef struct gftorf_adam_group {
    float* param;
    const float* grad;
    float* m;      /* first moment, same size, start at 0  */
    float* v;      /* second moment, same size, start at 0 */
    int64_t n;
    float lr;      /* learning rate (at step 1 when decaying)                 */
    float lr_final;        /* with decay_steps > 0: the rate from step decay_steps + 1 on */
    int32_t decay_steps;   /* 0: constant lr; else lr (lr_final / lr)^(min(t - 1, decay_steps) / decay_steps)
                              at 1-based step t (paper §4: the network's rate, 8e-4 to
                              1.6e-6 over 60K iterations), computed on the device from
                              the step counter, so a replayed graph follows the schedule */
    int32_t reserved;      /* must be 0 */
} gftorf_adam_group;

/* Adam (paper §4: beta = (0.9, 0.999), eps = 1e-15, per-group learning
 * rates).  Increments the device step counter *step (int32) and applies the
 * bias-corrected update with t = the new value.  groups: host array. */
int gftorf_adam_step(const gftorf_adam_group* groups, int32_t n_groups, int32_t* step,
                     float beta1, float beta2, float eps, void* stream);

/* Selects a batch of frames of a sequence from the device step counter, for
 * graph-replayed optimisation loops: with s = *step (read on the device),
 * frame b of the batch is seq[(n_batch * s + b) mod n_seq], its backgrounds
 * replaced by bg_table[(s mod n_bg)][b][0 .. 3 + n_quad) when bg_table is not
 * NULL (the paper's per-iteration random background, §4), and
 * frame_index[b] receives the sequence index.  All pointers are device. */
int gftorf_select_frames(gftorf_frame* frames, int32_t n_batch, const gftorf_frame* seq,
                         int32_t n_seq, const float* bg_table, int32_t n_bg, int32_t n_quad,
                         const int32_t* step, int32_t* frame_index, void* stream);

/* Fills n floats with `value` (a kernel, not a memset: safe in graphs). */
int gftorf_fill_f32(float* p, float value, int64_t n, void* stream);

/* Graph capture of everything the calling thread enqueues on `stream`
 * between begin and end (hipStreamBeginCapture, thread-local mode).
 * end instantiates the graph and returns an executable handle. */
int gftorf_graph_begin(void* stream);
int gftorf_graph_end(void* stream, void** graph_exec);
int gftorf_graph_launch(void* graph_exec, void* stream);
int gftorf_graph_destroy(void* graph_exec);

/* Per-kernel timing with HIP events, for benchmarks (not for graph capture).
 * Between begin and end every kernel the library launches is bracketed by
 * two events on its stream.  begin pre-creates 2 * max_launches events;
 * launches beyond that are not timed.  collect waits for the recorded events,
 * adds their durations to per-kernel totals and frees the slots; end collects,
 * copies up to max_entries totals to `out` (host) and switches timing off.
 * Profiling state belongs to the calling thread: a thread's begin times only
 * the launches that thread makes, and collect / end see only its records. */
typedef struct gftorf_profile_entry {
    char name[48];       /* kernel name                      */
    int64_t launches;    /* timed launches                   */
    double total_ms;     /* summed event-to-event durations  */
} gftorf_profile_entry;

int gftorf_profile_begin(int32_t max_launches);
int gftorf_profile_collect(void);
int gftorf_profile_end(gftorf_profile_entry* out, int32_t max_entries, int32_t* n_entries);

/* ---- Deformation network (paper §4, "MLP") ---------------------------------
 * delta x = MLP(enc_Lx(s_x x0), enc_Lt(s_t t)) for every (time, Gaussian) row,
 * rows in time-major order r = i_t n + k.
 *   enc_L(p): the blocks p, sin(pi p), cos(pi p), sin(2 pi p), cos(2 pi p), ...,
 *             sin(2^(L-1) pi p), cos(2^(L-1) pi p) of the coordinates of p;
 *   network:  h_0 = the encoding (3 (1 + 2 L_x) + 1 + 2 L_t <= 96 features),
 *             h_{l+1} = relu(W_l h_l + b_l) for l = 0 .. 7 (width 256),
 *             delta x = W_8 h_8 + b_8;
 *   params:   float32, for l = 0 .. 8 in order W_l [out][in] row-major, then
 *             b_l [out] (gftorf_mlp_param_count floats).
 * The products run on the matrix cores with bfloat16 operands (weights,
 * encodings, activations and back-propagated gradients rounded to nearest
 * even) and float32 accumulation; biases, outputs and gradients are float32.
 * Every call enqueues on `stream`, allocates nothing and does not
 * synchronise. */
typedef struct gftorf_mlp_config {
    int32_t n_freq_x;   /* L_x (paper: 10)                                        */
    int32_t n_freq_t;   /* L_t (paper: 10)                                        */
    int32_t width;      /* hidden units per layer: must be 256                    */
    int32_t depth;      /* hidden layers: must be 8                               */
    float pos_scale;    /* s_x (paper: 1 / unambiguous range = 2 f / c)           */
    float time_scale;   /* s_t                                                    */
} gftorf_mlp_config;

#define GFTORF_MLP_MAX_TIMES 64

/* Floats of the parameter vector of `cfg` (0 if cfg is invalid). */
int64_t gftorf_mlp_param_count(const gftorf_mlp_config* cfg);

/* Workspace bytes for n Gaussians at n_times times; with `training` it also
 * holds the activations, ReLU decisions and gradients gftorf_mlp_bwd reads
 * (about 9.5 KB per row).  0 if the arguments are invalid. */
size_t gftorf_mlp_workspace_size(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                                 int32_t training);

/* delta [n_times][3][n] (overwritten) for canonical centres x0 [3][n] at the
 * times `times` (host, n_times <= GFTORF_MLP_MAX_TIMES).  With `save` the
 * activations stay in ws for gftorf_mlp_bwd (ws sized with training = 1). */
int gftorf_mlp_fwd(const gftorf_mlp_config* cfg, const float* params, const float* x0, int64_t n,
                   const float* times, int32_t n_times, float* delta, int32_t save,
                   void* ws, size_t ws_bytes, void* stream);

/* Backward of the last gftorf_mlp_fwd with save = 1 on the same ws and
 * arguments: given d_delta [n_times][3][n], overwrites d_params (the
 * parameter layout) and, if not NULL, d_x0 [3][n] (the canonical centres
 * reach the network through s_x x0; summed over the times).  Deterministic:
 * no atomics; the weight gradients are summed over fixed row chunks in a
 * fixed order. */
int gftorf_mlp_bwd(const gftorf_mlp_config* cfg, const float* params, const float* x0, int64_t n,
                   const float* times, int32_t n_times, const float* d_delta, float* d_params,
                   float* d_x0, void* ws, size_t ws_bytes, void* stream);

/* The ReLU decisions of the hidden layers (paper §4, "MLP": which units of
 * h_1 .. h_depth are active, z > 0 as the forward decided it in its own
 * precision), for tests and diagnostics.  decisions is a device array of
 * bytes [n_times * n][depth][width], row t * n + k for time t and Gaussian k,
 * 1 = active, 0 = inactive (any non-zero byte reads as active when set).
 * gftorf_mlp_get_decisions copies out what the last gftorf_mlp_fwd with
 * save = 1 recorded in ws; gftorf_mlp_set_decisions replaces them, so that
 * the next gftorf_mlp_bwd on this ws gates its gradients with the given
 * pattern (the saved activations stay the forward's).  ws, n and n_times are
 * those of the training forward (ws sized with training = 1); the caller owns
 * decisions.  Asynchronous on the stream.  Errors: GFTORF_EINVAL (bad
 * configuration, NULL pointer, misaligned ws), GFTORF_ENOWS, GFTORF_EHIP. */
int gftorf_mlp_get_decisions(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                             uint8_t* decisions, void* ws, size_t ws_bytes, void* stream);
int gftorf_mlp_set_decisions(const gftorf_mlp_config* cfg, int64_t n, int32_t n_times,
                             const uint8_t* decisions, void* ws, size_t ws_bytes, void* stream);

/* The same with the times read on the device from frames[0 .. n_frames)
 * (.time of each descriptor), so a replayed graph follows the frames that
 * gftorf_select_frames wrote; n_frames <= GFTORF_MLP_MAX_TIMES.  The
 * backward with accumulate_x0 != 0 ADDS the centre gradient to d_x0 (e.g.
 * the rasterizer's gradient of the same centres) instead of overwriting. */
int gftorf_mlp_fwd_frames(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                          int64_t n, const gftorf_frame* frames, int32_t n_frames, float* delta,
                          int32_t save, void* ws, size_t ws_bytes, void* stream);
int gftorf_mlp_bwd_frames(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                          int64_t n, const gftorf_frame* frames, int32_t n_frames,
                          const float* d_delta, float* d_params, float* d_x0, int32_t accumulate_x0,
                          void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * inference forward of gftorf_mlp_fwd (save = 0) without a workspace
 * argument.  delta [n_times][3][n] (overwritten) for canonical centres
 * x0 [3][n] at the host `times` (n_times <= GFTORF_MLP_MAX_TIMES); same
 * kernels and same result, bit for bit, as gftorf_mlp_fwd with save = 0.
 * The bfloat16 weight copies it needs live in a static device array of
 * GFTORF_MLP_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 * until the process ends; a configuration whose weight copies do not fit is
 * rejected with GFTORF_ENOWS (the supported 8 x 256 network needs about
 * 1.9 MB).  The call allocates nothing, does not synchronise, and resolves
 * the array's device address once per GPU on its first call there.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (other streams, other threads) race and give undefined offsets.
 * Errors: GFTORF_EINVAL (bad configuration, NULL pointer, non-finite scale),
 * GFTORF_ENOWS, GFTORF_EHIP. */
#define GFTORF_MLP_NOALLOC_SCRATCH_BYTES (4u << 20)
int gftorf_mlp_fwd_noalloc(const gftorf_mlp_config* cfg, const float* params, const float* x0,
                           int64_t n, const float* times, int32_t n_times, float* delta,
                           void* stream);

/* Eq. 7 with the deformation network (paper §4): the network is evaluated at
 * integer timesteps only, and a raw frame between two of them takes the
 * straight line between the deformed positions.  With delta_steps
 * [n_steps][3][n] the network's offsets at the timesteps, frame f gets
 *   delta_frames[f] = w1 delta_steps[lo_f] + w2 delta_steps[hi_f],
 *   w1 = (t_hi - t) / (t_hi - t_lo), w2 = (t - t_lo) / (t_hi - t_lo)
 * from frames[f] (device; the rasterizer's descriptors), and
 * (lo_f, hi_f) = anchors[2 f], anchors[2 f + 1] (HOST int32 [n_frames][2],
 * each in [0, n_steps)).  A frame with t_hi <= t_lo takes delta_steps[lo_f].
 * The result is the `delta` of gftorf_gaussians.  n_frames <= 256. */
#define GFTORF_MAX_BLEND_FRAMES 256
int gftorf_blend_offsets(const float* delta_steps, int32_t n_steps, int64_t n,
                         const gftorf_frame* frames, int32_t n_frames, const int32_t* anchors,
                         float* delta_frames, void* stream);

/* Transpose of gftorf_blend_offsets: d_steps [n_steps][3][n] (overwritten) =
 * the gradient of sum(d_frames * delta_frames) with respect to delta_steps,
 * summed over frames in frame order (deterministic). */
int gftorf_blend_offsets_bwd(const float* d_frames, int32_t n_frames, int64_t n,
                             const gftorf_frame* frames, const int32_t* anchors, int32_t n_steps,
                             float* d_steps, void* stream);

const char* gftorf_strerror(int code);
const char* gftorf_last_error(void);
int gftorf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GFTORF_H */
