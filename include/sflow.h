/*
 * sflow.h - C ABI of the structure-flow predictor-update filter for AMD MI355X (gfx950).
 *
 * The filter estimates structure flow, the scene's 3-D velocity relative to the camera at
 * every pixel divided by its range (Adarve & Mahony, "Real-time Structure Flow",
 * arXiv 2406.18031, Section "Structure Flow", eq:homogeneous_flow; units rad/s), from a
 * stream of brightness images Y and inverse-depth maps rho (eq:inv_depth, reference range
 * 1 m).  Each frame runs the pyramidal predictor-update filter of Section "Filter
 * Architecture": an upwind finite-difference prediction of the previous flow and inverse
 * depth (Section "Numerical prediction"), then a per-pixel least-squares update from the
 * new image and depth (Section "State update"), smoothing and coarse-to-fine
 * reconstruction (eq:hflow_reconstruction).
 *
 * Conventions shared by every call
 *  - Images are on a pinhole grid: pixel (i, j) (row i, column j) looks along
 *    normalize(((j - cx)/fx, (i - cy)/fy, 1)) with x right, y down, z forward.
 *  - Image arguments are caller-owned DEVICE pointers (HIP memory, e.g. torch tensors),
 *    rows x cols, row-major, contiguous.  Element type is float32, or float16 when the
 *    context was created with storage = SF_FP16.  Host pointers are rejected.
 *  - All device work is enqueued on the HIP stream given to sf_create, in stream order, like
 *    hipMemcpyAsync: the caller must not modify an input until that stream has passed the
 *    call that consumed it.  Calls return without waiting for the device, except
 *    sf_get_state / sf_set_state, which synchronise the stream.
 *  - Every call validates all arguments before it enqueues anything: a call that returns an
 *    error leaves the context unchanged (except the sticky SF_ERR_HIP below).  Calls that
 *    allocate device memory (sf_create*, sf_set_camera*, sf_set_tile, sf_set_pass_steps,
 *    sf_net_create) allocate before they release anything, so SF_ERR_OOM leaves the context
 *    as it was too.  For tests, the environment variable SFLOW_FAIL_ALLOC=n makes the n-th
 *    device allocation, counted from the moment the variable took its current value, fail
 *    with SF_ERR_OOM.
 *  - A context may be used from one host thread at a time.
 *  - Return values are sf_status codes; nothing throws or aborts across the ABI.
 *    sf_last_error(ctx) gives a text for the last failure on that context.
 *  - A HIP failure (launch error, fault reported by the runtime) makes the context
 *    unusable: it and every later call return SF_ERR_HIP; destroy it.
 */
#ifndef SFLOW_H
#define SFLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sf_ctx_s* sf_ctx;

typedef enum {
    SF_OK = 0,
    SF_ERR_INVALID_ARG = -1, /* NULL/host pointer, bad size, dt <= 0 or not finite, ...     */
    SF_ERR_STATE = -2,       /* call not valid now (push before sf_set_camera, get before push) */
    SF_ERR_OOM = -3,         /* device allocation failed                                   */
    SF_ERR_HIP = -4,         /* a HIP runtime call failed; the context is unusable          */
    SF_ERR_UNSUPPORTED = -5, /* valid request this build does not implement                */
    SF_ERR_NUMERIC = -6      /* a stored flow value was not finite (sf_check_state)        */
} sf_status;

/* element type of images and stored state */
enum { SF_FP32 = 0, SF_FP16 = 1 };
/* update stage: the paper's least-squares update, or the learned correction */
enum { SF_UPDATE_PLAIN = 0, SF_UPDATE_LEARNED = 1 };

/* Readings of points the paper leaves ambiguous (bit flags; 0 = the default readings):
 *  SF_READ_DOMINANT_LITERAL  dominant optical flow as printed in Section "Numerical
 *                            prediction" (picks the neighbour of smaller magnitude); the
 *                            default follows the text (the larger one).
 *  SF_READ_SOURCE_LITERAL    the source term f<eta,w> with the full step in both the column
 *                            and the row half-step, as printed; the default applies half of it
 *                            in each, matching eq:hflow_propagation_discrete.
 *  SF_READ_NO_CFL_CLAMP      do not clamp the dominant flow to the stability bound of
 *                            eq:numerical_stability (|u_hat| <= N). */
enum {
    SF_READ_DOMINANT_LITERAL = 1u,
    SF_READ_SOURCE_LITERAL = 2u,
    SF_READ_NO_CFL_CLAMP = 4u
};

/* sf_get_flow kinds (finest level).  Output is always float32, planar: component-major
 * [components][rows][cols], contiguous. */
enum {
    SF_FLOW_W_RAD_S = 0,    /* 3 planes: structure flow w in rad/s (eq:homogeneous_flow)      */
    SF_FLOW_TANGENT_PX = 1, /* 2 planes: B^T P w / dmu in pixels per frame (eq:tangent_flow)   */
    SF_FLOW_NORMAL_PX = 2,  /* 1 plane : <eta, w> / dmu in pixels per frame (eq:normal_flow)   */
    SF_FLOW_RHO = 3,        /* 1 plane : filtered inverse depth, 1/m                          */
    SF_FLOW_W_FRAME = 4     /* 3 planes: structure flow in rad/frame (the filter's own unit)  */
};

#define SF_MAX_LEVELS 8

typedef struct {
    int32_t rows, cols;   /* finest grid, >= 2 each                                           */
    int32_t levels;       /* pyramid levels H in [1, SF_MAX_LEVELS] (Section "Filter
                             Architecture"); level h has ceil(rows/2^(h-1)) x ceil(cols/2^(h-1))
                             pixels and every level must be at least 2 x 2                      */
    float max_flow_px;    /* largest expected image motion per frame at the finest level, >= 0.
                             Level h integrates N_h = max(1, ceil(max_flow_px / 2^(h-1))) steps
                             (eq:numerical_stability)                                          */
    int32_t smooth_iters[SF_MAX_LEVELS]; /* 5x5 averaging passes after each level's solve,
                             finest first, in [0, 16]                                          */
    float alpha[5];       /* weights alpha_1..alpha_5 of the image, depth, temporal, depth
                             measurement and depth prior terms (eq:cost_top, eq:cost_invdepth);
                             gamma_1,2 = alpha_1,2 / dmu0^2 with dmu0 = 1/sqrt(fx_h^2 + 1) the
                             level's on-axis pixel spacing, gamma_3,4,5 = alpha_3,4,5.
                             All five zero selects the defaults {300, 1000, 1, 1, 1}.
                             Otherwise each must be finite and >= 0, with alpha_3 > 0 and
                             alpha_4 + alpha_5 > 0.                                           */
    int32_t storage;      /* SF_FP32 or SF_FP16 (images and state stored in half precision,
                             all arithmetic in float32)                                        */
    int32_t update;       /* SF_UPDATE_PLAIN or SF_UPDATE_LEARNED (then smooth_iters[0] <= 4,
                             the same for every stream of a batch, and sf_set_learned before
                             the first push)                                                   */
    uint32_t read_flags;  /* SF_READ_* bits                                                    */
} sf_config;

typedef struct {
    double fx, fy, cx, cy; /* pinhole intrinsics of the finest level, in pixels; fx, fy > 0   */
    /* Optional general grid (Section "Spherical image data structure"): NULL for the pinhole
     * grid of the intrinsics, or a HOST array of rows x cols x 3 doubles, the finest level's
     * unit directions (row-major, x right, y down, z forward; |eta| within 1e-6 of 1), e.g. a
     * Spherepix patch or a wide-angle camera's rays.  Level h then samples it at every
     * 2^(h-1)-th row and column; the tangent bases and spacings are derived from it as the
     * paper defines them (b1 toward the next column, b2 = eta x b1 toward the next row,
     * dmu = |P eta_next|) and kept in device tables (36 bytes per pixel per level, read by
     * every frame).  fx still sets the weights' scaling (dmu0 in sf_config.alpha) and the FP16
     * flow scale; cx, cy are not used.  Read during the call only. */
    const double* eta;
} sf_camera;

/* Create a filter context.  Allocates all device memory for the state (double-buffered),
 * the pyramid and work buffers.  hip_stream is a hipStream_t (NULL = default stream).
 * On success *out owns the context until sf_destroy. */
sf_status sf_create(const sf_config* cfg, void* hip_stream, sf_ctx* out);

/* Set the camera (Section "Spherical image data structure": the grid of unit directions,
 * its tangent bases and pixel spacing are derived from the intrinsics).  Resets the filter:
 * the next push is a first frame. */
sf_status sf_set_camera(sf_ctx ctx, const sf_camera* cam);

/* Push frame k+1: Y brightness (any float scale), rho inverse depth in 1/m (NaN = no
 * measurement, 0 = infinitely far, valid), dt seconds since the previous frame (> 0,
 * finite; ignored on the first frame).  The first frame after sf_set_camera initialises the
 * state (flow 0, inverse depth from rho with 0 where missing; Section "Ground truth
 * evaluation").  Later frames run prediction, update, smoothing and reconstruction; the
 * reconstruction launch holding the finest level is enqueued by the next call that needs it
 * (sf_get_flow, which runs it together with the output, or a push, state copy, tile or pass
 * change, update-input read), always on the context's stream and before that call's own work,
 * so the deferral is invisible to the caller. */
sf_status sf_push_frame(sf_ctx ctx, const void* Y, const void* rho, double dt);

/* sf_push_frame with the camera's inertial rates, host arrays of 3 doubles in the camera frame
 * (x right, y down, z forward), each taken as constant since the previous frame and each NULL
 * for zeros: omega, its angular velocity (rad/s); omega_dot, the rate of change of omega
 * (rad/s^2); acc, its linear acceleration relative to an inertial frame (m/s^2)
 * (Section "Structure Flow", eq:camvel_dot).  The prediction then keeps the source terms of
 * eq:hflow_conservation that the paper drops by eq:assumption (Section "State prediction"):
 * after each step of length 1/N (frames) the structure flow gains
 * 1/N (-2 W x w - W x (W x eta) - D x eta - rho A), with W = omega dt, D = omega_dot dt^2 and
 * A = acc dt^2, and the increment of a lower level gains 1/N (-2 W x dw).  The acceleration
 * enters with -rho A as the kinematics give it (w = -Omega x eta - rho v for a static scene,
 * dv/dt = -Omega x v + a; the printed field acceleration has +rho a), and -D x eta is the
 * derivative of -Omega x eta when omega changes (the paper takes it constant,
 * eq:totaldev_camangvel).  With all three NULL this is sf_push_frame, bitwise.
 * SF_ERR_INVALID_ARG for a non-finite rate. */
sf_status sf_push_frame_ex(sf_ctx ctx, const void* Y, const void* rho, double dt,
                           const double* omega, const double* omega_dot, const double* acc);

/* Write the finest-level result of the last push to out (device, float32, see SF_FLOW_*).
 * SF_ERR_STATE before the first push; zeros after only the first push. */
sf_status sf_get_flow(sf_ctx ctx, int32_t kind, void* out);

/* Bytes of the state blob of sf_get_state / sf_set_state. */
sf_status sf_state_size(sf_ctx ctx, size_t* bytes);

/* Watchdog of the state.  Every launch that stores a level's new flow (w at the top level,
 * dw below; Sections "State update" and "Numerical prediction") tests each stored value and sets
 * bit s of a device word when a value of stream s is NaN, infinite or, with FP16 storage,
 * beyond the FP16 range; this costs no synchronisation and a ballot per wave.  sf_check_state
 * synchronises the context stream, writes the word to *streams (bit s = stream s), clears it
 * and returns SF_ERR_NUMERIC (with the streams in sf_last_error) if it was set, else SF_OK.
 * The word is also cleared when the cameras are set (the state restarts).  Why: the
 * prediction's source term f<eta, w> lets the flow's normal component grow without bound where
 * the update observes it only weakly, so a long run of a scene can end in non-finite flow;
 * inputs with infinite values do the same.  A caller checks every so many frames and restarts
 * the stream (sf_set_camera) or restores a saved state (sf_set_state) when it fails. */
sf_status sf_check_state(sf_ctx ctx, uint64_t* streams);

/* Copy the whole filter state to / from HOST memory (synchronises the stream).  The blob is
 * a 32-byte header {uint32 magic 'SFST', uint32 version 1, int32 levels, int32 initialised,
 * double dt_prev, int64 frames} followed, for h = 1..H, by float32 planes of
 * rows_h x cols_h: w (3, rad/frame), dw (3, levels below the top only), rho, Yhat.
 * Used to resume a stream and to inject a state for single-frame checks.  sf_set_state
 * needs a camera to be set and a blob of exactly sf_state_size bytes for this
 * configuration. */
sf_status sf_get_state(sf_ctx ctx, void* host_blob, size_t bytes);
sf_status sf_set_state(sf_ctx ctx, const void* host_blob, size_t bytes);

/* Release the context and all its device memory (synchronises the stream first).
 * sf_destroy(NULL) is a no-op returning SF_OK. */
sf_status sf_destroy(sf_ctx ctx);

/* Text of the last error on ctx (or of the last failed sf_create when ctx is NULL).  The
 * pointer stays valid until the next call on the same context. */
const char* sf_last_error(sf_ctx ctx);

/* ---- batches of camera streams -------------------------------------------------------------
 * A batch context advances up to 64 independent camera streams together: every frame runs one
 * pyramid launch per pyramid depth, one fused level-step launch over every tile of every level
 * of every stream, and one reconstruction launch per lower level, for all streams at once.  Streams
 * may differ in size, levels, maximum flow, smoothing, weights and readings, but not in
 * storage.  sf_create is sf_create_batch with n = 1; the single-stream calls (sf_set_camera,
 * sf_push_frame, sf_get_flow, sf_state_size, sf_get_state, sf_set_state) return
 * SF_ERR_INVALID_ARG on a context of more than one stream. */
sf_status sf_create_batch(const sf_config* cfgs, int32_t n, void* hip_stream, sf_ctx* out);
sf_status sf_stream_count(sf_ctx ctx, int32_t* n);
/* cams: host array of n cameras, one per stream; resets every stream */
sf_status sf_set_cameras(sf_ctx ctx, const sf_camera* cams);
/* Y, rho: host arrays of n device pointers (one frame per stream); dt: host array of n */
sf_status sf_push_frames(sf_ctx ctx, const void* const* Y, const void* const* rho,
                         const double* dt);
/* sf_push_frames with inertial rates (see sf_push_frame_ex): omega, omega_dot, acc are host
 * arrays of 3 n doubles (stream s at [3 s, 3 s + 3)), each NULL for zeros */
sf_status sf_push_frames_ex(sf_ctx ctx, const void* const* Y, const void* const* rho,
                            const double* dt, const double* omega, const double* omega_dot,
                            const double* acc);
sf_status sf_get_flow_stream(sf_ctx ctx, int32_t stream, int32_t kind, void* out);
/* Every stream's output in one call: outs is a host array of n device pointers (NULL = skip
 * that stream), each as out of sf_get_flow for that stream.  The results are bitwise those of
 * sf_get_flow_stream; the streams' outputs are written by one or two launches. */
sf_status sf_get_flows(sf_ctx ctx, int32_t kind, void* const* outs);
sf_status sf_state_size_stream(sf_ctx ctx, int32_t stream, size_t* bytes);
sf_status sf_get_state_stream(sf_ctx ctx, int32_t stream, void* host_blob, size_t bytes);
/* on a batch of more than one stream, only after the first frame has been pushed */
sf_status sf_set_state_stream(sf_ctx ctx, int32_t stream, const void* host_blob, size_t bytes);

/* Tile shape of the fused level kernel for level h (1-based, all streams that have it):
 * output tiles of tw x th pixels; tw + 2*halo_h and th + 2*halo_h must not exceed 64, where
 * halo_h = max(n, 2) + 2 * smooth_iters[h-1] with n the steps of the level's last prediction
 * pass (N_h unless split, see sf_set_pass_steps; earlier passes use the built-in choice when
 * the shape does not fit them).  0, 0 restores the built-in choice.  For tuning. */
sf_status sf_set_tile(sf_ctx ctx, int32_t level, int32_t tw, int32_t th);

/* Prediction steps per level-step launch (default 8).  A level whose prediction takes more
 * steps N (N_h of Section "Numerical prediction") runs it in ceil(N / steps) launches, each
 * over tiles with a halo of only its own steps, handing the transported fields on in FP32
 * device buffers (allocated here; set-up work).  The result is bitwise the same for any value;
 * smaller values trade an extra launch for less redundant halo work, which pays when many
 * tiles are in flight (batches, large images, large flows).  Also lifts the limit on the
 * maximum flow: only the last pass's halo, max(steps, 2) + 2*smooth, must fit the region.
 * SF_ERR_UNSUPPORTED if some level's last pass would not fit. */
sf_status sf_set_pass_steps(sf_ctx ctx, int32_t steps);

/* ---- mapping a camera's frame onto a stream's grid ----------------------------------------
 * The paper maps each camera image and depth map onto its spherical grid before the filter runs
 * (Section "Experimental Validation"; Section "Spherical image data structure").  After
 * sf_set_source_camera names the pinhole camera (intrinsics, size; eta must be NULL) that
 * produces a stream's frames, sf_map_frame resamples one frame of that camera onto the stream's
 * finest grid (its camera's eta, or its pinhole grid): grid direction eta looks at source pixel
 * (u, v) = (fx eta_x / eta_z + cx, fy eta_y / eta_z + cy); brightness is interpolated bilinearly
 * with the source clamped to its edge; inverse depth (1/m, NaN = missing) bilinearly over the
 * valid neighbours, missing where they carry less than half of the weight or where the
 * direction is more than 1e-3 px outside the image or behind the camera.  Y_src, rho_src are
 * device images of the source size, Y_out, rho_out device images of the stream's finest size,
 * all in the context's storage type; enqueued on the context stream.  The outputs are what
 * sf_push_frame takes. */
sf_status sf_set_source_camera(sf_ctx ctx, int32_t stream, const sf_camera* src, int32_t rows,
                               int32_t cols);
sf_status sf_map_frame(sf_ctx ctx, int32_t stream, const void* Y_src, const void* rho_src,
                       void* Y_out, void* rho_out);

/* ---- inverse depth from a rectified stereo pair ----------------------------------------------
 * The paper's proposed extension (Section "Conclusions and Future Work"): take the depth
 * measurements from the disparity of a coupled stereo pair, so that the filter runs on image
 * data alone.  The left camera is the stream's pinhole camera (a stream with an eta grid is
 * SF_ERR_UNSUPPORTED); the right camera has the same intrinsics and orientation, its centre
 * `baseline` metres along the left camera's x axis (rectified pair).  A point at inverse range
 * rho along the left direction eta appears kappa rho pixels to the left on the same row,
 * kappa = fx baseline sqrt(x^2 + y^2 + 1), x = (j - cx)/fx, y = (i - cy)/fy.
 * sf_stereo_depth writes, per pixel of the finest level: the integer disparity in
 * [0, max_disparity] minimising the sum of absolute differences over a 5x5 window (rows and
 * columns clamped to the image; float32 sums over window rows then columns; the smallest on
 * ties), refined by `iterations` Gauss-Newton steps on the window's squared residuals with the
 * right image interpolated linearly along the row (kept in [0, max_disparity + 1]), as the
 * inverse depth d / kappa (1/m); NaN (missing) where the window's sum of squared row slopes of
 * the right image is below `texture`, its mean absolute residual above `residual`, or j - d < 0.
 * Images are device, rows x cols of the stream, in the context's storage type; enqueued on the
 * context stream.  The output is what sf_push_frame takes as rho.  Ranges: baseline > 0,
 * max_disparity in [0, 64], iterations in [0, 16], texture >= 0, residual > 0 (for images in
 * [0, 1]: 3, 2.5e-3 and 0.05 work well). */
sf_status sf_set_stereo(sf_ctx ctx, int32_t stream, double baseline, int32_t max_disparity,
                        int32_t iterations, double texture, double residual);
sf_status sf_stereo_depth(sf_ctx ctx, int32_t stream, const void* Y_left, const void* Y_right,
                          void* rho_out);

/* Kernel timing for measurement.  When enabled, every push records HIP events around each
 * kernel on the context stream; sf_kernel_times returns, per kernel kind (0 pyramid,
 * 1 level step, 2 reconstruction), the total milliseconds and launch counts since the
 * last reset (synchronises the stream). */
sf_status sf_set_timing(sf_ctx ctx, int32_t enable);
sf_status sf_kernel_times(sf_ctx ctx, double* ms3, int64_t* launches3, int32_t reset);

/* Frame graphs.  When enabled, every push after a stream's first frame replays a HIP graph
 * instead of enqueuing its launches one by one: the frame's launches (pyramid, level steps,
 * learned update, reconstruction) are captured once per state parity and per form of the
 * prediction (with or without inertial rates) on a private stream, and each push updates the
 * per-frame arguments of the pyramid and level-step nodes (input pointers, dt rescale, rates)
 * and launches the graph on the context stream.  Results are bitwise those of the launches
 * enqueued one by one.  Graphs are captured again after any change of cameras, tiles, pass
 * length or learned parameters.  Not used while kernel timing is on.  Disabling releases them
 * (synchronises the stream). */
sf_status sf_set_graph(sf_ctx ctx, int32_t enable);

/* Frame inputs produced on another stream.  sf_set_input_stream names the HIP stream on which
 * the caller produces (or copies in) the frames it pushes; NULL or the context stream restores
 * the default, where every launch of a push is ordered after the work already enqueued on the
 * context stream.  With another stream, a push orders the launches that read the frame's Y and
 * rho after the work enqueued so far on that stream only, and builds the frame's pyramid on a
 * stream of the library's own (default priority), so that it runs beside the previous frame's
 * level step and reconstruction instead of after them; the level step and every later launch
 * stay on the context stream, which waits for the pyramid.  The pyramid planes alternate
 * between two buffers from frame to frame, so no frame's pyramid overwrites one still being
 * read.  A frame's input buffers stay in use until the next push returns: that push makes the
 * input stream wait until the earlier frame's launches are done with them, so work enqueued on
 * the input stream afterwards may rewrite them (a caller reusing buffers keeps two sets).
 * Results are bitwise those of the default mode.  With frame graphs or kernel timing on, the
 * pyramid stays on the context stream (which then waits for the input stream).  The stream
 * must stay valid while it is set.  Synchronises the context stream. */
sf_status sf_set_input_stream(sf_ctx ctx, void* hip_stream);

/* ---- learned update ----------------------------------------------------------------------
 * An extension beyond the paper, which uses the least-squares update of Section "State
 * update" at every level.  With update = SF_UPDATE_LEARNED, at the finest level of every
 * stream a convolutional network (3x3 kernels, 9 -> 16 -> 16 -> 16 -> 3 channels, ReLU after
 * the first three layers, zero padding; BF16 operands, FP32 accumulation) corrects the output
 * flow: with x_ls the solution of the update and S the level's N_s passes of 5x5 averaging
 * (so that S(x_ls) is the level's new state), sf_get_flow reports the flow of
 * S(x_ls) + dmu * c, where c (3 values, pixels per frame) is the network's output.  The
 * filter's state, and so its recurrence, stay those of the plain update.  The network's
 * inputs per pixel are Y_prior - 1/2, Y_new - 1/2, 4 rho (0 where missing), x0 / dmu / 4 (3)
 * and x_ls / dmu / 4 (3), where Y_prior is the predicted smoothed image, Y_new the new one and
 * x0 the predicted field (the flow at a top level, the increment over the parent's flow
 * below it; Section "State update").
 * Per pixel, c is applied unless the least-squares cost of the step,
 * G1 (aY.c)^2 + G2 (aR.c)^2 + gamma_3 |c|^2 (in pixel units, the cost increase a step c away
 * from the minimum x_ls), exceeds `threshold` or is not finite (a "fallback": the plain
 * flow).  A threshold < 0 makes every pixel fall back, which gives exactly the plain
 * update.  sf_get_state / sf_set_state carry the state only, not the correction;
 * sf_set_state clears the stream's correction, so the flow read back is the state's.
 *
 * The parameters are FP32, SF_LEARNED_PARAMS values: per layer l = 0..3 the weights
 * W[3][3][cin][cout] (tap row dy+1, tap column dx+1, input channel, output channel;
 * out[p] = b + sum W[dy+1][dx+1][c][:] in[p + (dy, dx)][c]) followed by the bias b[cout]. */
#define SF_LEARNED_PARAMS 6387
#define SF_UPDATE_INPUT_PLANES 22

/* Load parameters (host, SF_LEARNED_PARAMS finite floats) and the fallback threshold (not
 * NaN; +inf never falls back); synchronises the stream.  SF_ERR_STATE on a plain context. */
sf_status sf_set_learned(sf_ctx ctx, const float* params, size_t n, float threshold);
/* Fallbacks and learned pixels since the last reset (synchronises the stream). */
sf_status sf_learned_stats(sf_ctx ctx, int64_t* fallbacks, int64_t* pixels, int32_t reset);
/* Training data of the last frame of one stream (finest level): writes
 * SF_UPDATE_INPUT_PLANES float32 planes of rows x cols to the device pointer out: the network
 * inputs (9, as the network reads them: rounded to BF16), x0 (3), x_ls (3), S(x_ls) (3), the
 * parent's reconstructed flow (3; 0 at a top level) and dmu (1).  Flows are in rad/frame, so the network output that reaches a flow w is
 * (w - parent - S(x_ls)) / dmu.  SF_ERR_STATE until an update has run after the camera or
 * the stream's state was last set. */
sf_status sf_get_update_inputs(sf_ctx ctx, int32_t stream, float* out);

/* ---- training the learned update's network --------------------------------------------------
 * A network object runs the network above on a fixed list of up to 64 images (sizes given at
 * creation, each at most 2^26 pixels, 2^27 in total), on the caller's HIP stream.  Image
 * tensors are device float32, the images one after the other, each planar [C][rows][cols]
 * (C = 9 for inputs, 3 for outputs and targets).  Every call synchronises the stream except
 * sf_net_forward. */
typedef struct sf_net_s* sf_net;
sf_status sf_net_create(const int32_t* rows, const int32_t* cols, int32_t n_images,
                        void* hip_stream, sf_net* out);
/* set the parameters (host) and reset the optimiser */
sf_status sf_net_set_params(sf_net net, const float* params, size_t n);
sf_status sf_net_get_params(sf_net net, float* params, size_t n);
sf_status sf_net_forward(sf_net net, const float* in, float* out);
/* One step: forward, the loss mean over all pixels of sqrt(|out - target|^2 + eps^2), its
 * gradient by backpropagation, and, when lr > 0, one Adam step (beta 0.9, 0.999, eps 1e-8)
 * on the parameters.  loss_out (host, 1 float) and grad_out (host, SF_LEARNED_PARAMS floats,
 * the gradient at the parameters before the step) may be NULL. */
sf_status sf_net_train_step(sf_net net, const float* in, const float* target, float lr,
                            float* loss_out, float* grad_out);
/* the loss's eps (pixels, > 0; default 1e-3: close to the endpoint error itself; about 1
 * makes the loss quadratic for errors below a pixel) */
sf_status sf_net_set_loss(sf_net net, float eps);
/* ---- the network's forward pass without allocation ---------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the forward pass of sf_net_forward on one image,
 * with no network object and no allocation of any kind.  Its work buffers live in a fixed
 * array of the library's device code (about 29 MiB, held on every GPU the call runs on until
 * the process ends), which limits the image to SF_NOALLOC_MAX_PIXELS pixels.
 *  params  device, SF_LEARNED_PARAMS float32 values in the layout of sf_set_learned (not
 *          checked for finiteness: non-finite parameters give non-finite outputs)
 *  in      device, float32 [9][rows][cols] contiguous (the inputs of sf_net_forward)
 *  out     device, float32 [3][rows][cols] contiguous
 * The work is enqueued on hip_stream (NULL = default stream) and not waited for.  The result is
 * bitwise that of sf_net_forward on a network holding the same parameters.  All calls on one
 * GPU share the one array: calls that overlap in time on the same GPU (other streams, other
 * threads) race and give undefined results; calls ordered on one stream are safe.
 * SF_ERR_INVALID_ARG for a size outside [1, SF_NOALLOC_MAX_PIXELS] or a pointer that is not a
 * device pointer (nothing is enqueued); the text is sf_net_last_error(NULL). */
#define SF_NOALLOC_MAX_PIXELS (1 << 18)
sf_status sf_net_forward_noalloc(const float* params, int32_t rows, int32_t cols,
                                 const float* in, float* out, void* hip_stream);
/* releases the network and its device memory (synchronises its stream); NULL is a no-op */
sf_status sf_net_destroy(sf_net net);
const char* sf_net_last_error(sf_net net);

/* ---- measurement -------------------------------------------------------------------------
 * A plain streaming copy of `bytes` bytes from src to dst (device pointers, 16-byte aligned,
 * not overlapping) on hip_stream, enqueued and not waited for: the yardstick for the HBM
 * bandwidth the device reaches (bytes read + bytes written over its duration), and a copy of
 * known size for scaling HBM byte counters.  SF_ERR_INVALID_ARG for host, misaligned or
 * overlapping pointers. */
sf_status sf_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SFLOW_H */
