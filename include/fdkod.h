/*
 * fdkod.h -- C ABI of the FDK-OD cone-beam backprojection library for AMD
 * MI355X (gfx950).
 *
 * FDK-OD ("optimal decomposition", Andriiashen and Kozhevnikov, 2017) splits
 * every N x N slice into 4^s squares (Sec. 2.1), bounds the part of every
 * detector row each square uses with eq. (1) evaluated at the square's
 * vertices (Sec. 2.1), crops and shifts that part so the square's centre
 * trajectory becomes one column, decimates it in angle from P to P' angles
 * (low-pass filter + downsampling, Sec. 2.1), and backprojects each square
 * from the decimated data (Sec. 2.2, eq. (6)-(8)).  The ramp filtering of the
 * FDK stage it starts from is the "initial convolution" of Sec. 3.
 *
 * Geometry and units
 *   Circular orbit, flat detector.  Units are voxels; the detector is a
 *   virtual detector through the rotation axis with the voxel pitch.  The
 *   source sits at distance R from the axis (the R of eq. (1)).  Angle
 *   beta_p = 2 pi p / P over 360 degrees; source at -R (cos b, sin b, 0).
 *   Voxel (i, j, l) sits at x = i - (N-1)/2, y = j - (N-1)/2,
 *   z = l - (N_z-1)/2.  Detector pixel (u, v) sits at a = u - (N-1)/2,
 *   b = v - (N-1)/2.
 *
 * Layouts (all device buffers, contiguous, 256-byte aligned)
 *   projections  float32 [P][N][N]       (p, v, u), u fastest
 *   filtered     store type [P][N][N]    same layout (fdkod_filter output)
 *   workspace    store type, decimated sub-sinograms of every square,
 *                fdkod_plan_info().workspace_bytes bytes (unused when s = 0):
 *                square q (q = by 2^s + bx) holds Y_q as [P'][N][W_q]
 *                (m, v, j), j fastest, from element offset
 *                N P' sum_{q' < q} W_q' 
 *   volume       float32 [N_z][N][N]     (l, j, i), x fastest
 *
 * Ownership and streams
 *   The caller owns every data buffer.  A plan owns only its small device
 *   tables.  Every enqueueing call (fdkod_bounds, fdkod_filter,
 *   fdkod_decompose, fdkod_reconstruct, fdkod_backproject) is asynchronous
 *   on the given stream, allocates nothing and never synchronises.  Only
 *   fdkod_plan_create synchronises (once).  A plan is read-only after
 *   creation; concurrent use on several streams needs separate workspaces.
 *
 * Errors
 *   Every call returns a status; nothing throws across the ABI.  Kernel
 *   faults are asynchronous and surface at the caller's next synchronisation.
 *   fdkod_last_error() returns a thread-local text for the last failure.
 */
#ifndef FDKOD_H
#define FDKOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdkod_plan_s* fdkod_plan_t;  /* opaque */
typedef void* fdkod_stream_t;               /* a hipStream_t; NULL = null stream */

typedef enum {
    FDKOD_OK = 0,
    FDKOD_E_ARG = 1,          /* null pointer, bad size or enum value */
    FDKOD_E_GEOMETRY = 2,     /* R <= (N-1)/sqrt(2), 2^s > N, skip > s */
    FDKOD_E_UNSUPPORTED = 3,  /* not a gfx950 device, or sizes beyond the kernels' tiles */
    FDKOD_E_NOMEM = 4,        /* plan table allocation failed */
    FDKOD_E_HIP = 5,          /* a HIP runtime call failed (see fdkod_last_error) */
    FDKOD_E_STATE = 6         /* call not valid for this plan */
} fdkod_status;

typedef enum { FDKOD_F32 = 0, FDKOD_F16 = 1, FDKOD_BF16 = 2 } fdkod_dtype;

/* Window of the angular decimation (Sec. 2.1, step 4):
 *  TRIANGLE  triangle of half-width one decimated step (the library's reading
 *            of the paper's unspecified small low-pass kernel); taps = 2.
 *  SINC      windowed sinc (an extension, a cheaper alternative to a learned
 *            filter): the ideal low-pass cut off at the decimated rate's
 *            Nyquist frequency, times a Hann window over `taps` decimated
 *            steps (even, 2..6; 0 selects 4), normalised per window; each
 *            projection feeds up to `taps` windows.  Needs P >= taps * D.
 *            The learned decimation adds its correction to it as to the
 *            triangle; not available to batches (FDKOD_E_UNSUPPORTED); the
 *            slab mode supports it. */
typedef enum { FDKOD_DECIM_TRIANGLE = 0, FDKOD_DECIM_SINC = 1 } fdkod_decim;

/* Rows of the decomposed data:
 *  DETECTOR  every detector row is cropped and decimated on its own, as in
 *            Sec. 2.1; the backprojection reads row z R / D(beta) + c_v (eq. (9)).
 *  CONE      cone-corrected rows (an extension beyond the paper): before the
 *            decimation, row v' of square q at angle beta is resampled from
 *            detector row (v' - c_v) R / D_c(beta) + c_v (linear in v; rows
 *            outside the detector read zero), D_c the depth of the square's
 *            centre, so a voxel's row coordinate z D_c / D + c_v varies little
 *            with beta and the angular decimation averages less of the z
 *            direction.  With s = 0 it equals DETECTOR.  Not available to the
 *            learned decimation, the slab mode and batches (FDKOD_E_UNSUPPORTED). */
typedef enum { FDKOD_ROWS_DETECTOR = 0, FDKOD_ROWS_CONE = 1 } fdkod_rows;

/* Interpolation of the crop's shift along u (Sec. 2.1, step 3):
 *  LINEAR  as in the paper;
 *  CUBIC   Keys' cubic convolution kernel with a = -1/2 (Catmull-Rom), four
 *          samples per cropped value, zero outside the detector (an
 *          extension: Sec. 2.2 notes that a more precise interpolation
 *          reduces smoothing).  The learned decimation reads its rows S
 *          with the same interpolation; not available to batches
 *          (FDKOD_E_UNSUPPORTED); the slab mode supports it. */
typedef enum { FDKOD_INTERP_LINEAR = 0, FDKOD_INTERP_CUBIC = 1 } fdkod_interp;

/* Problem statement, after Sec. 2.1: N, P, R, s, and the skipped
 * decimation stages k of Sec. 2.2 (D = 2^(s-k), P' = ceil(P / D)). */
typedef struct {
    int32_t n;      /* detector width = height = volume side in x, y; 2..4096 */
    int32_t nz;     /* volume slices; 0 means n */
    int32_t p;      /* projections over 360 degrees; 1..65536 */
    double r;       /* R of eq. (1), voxel units; must exceed (N-1)/sqrt(2) */
    int32_t s;      /* decomposition stages: 4^s squares; 2^s <= N; s = 0 is direct FDK */
    int32_t skip;   /* skipped decimation stages k, 0 <= k <= s */
    int32_t store;  /* fdkod_dtype of the filtered and decimated sinograms */
    int32_t decim;  /* fdkod_decim: window of the angular decimation */
    int32_t taps;   /* SINC: window length in decimated steps (2, 4, 6; 0 = 4); TRIANGLE: 0 or 2 */
    int32_t rows;   /* fdkod_rows */
    int32_t interp; /* fdkod_interp */
} fdkod_params;

/* Sizes and derived quantities of a plan (filled by fdkod_plan_info). */
typedef struct {
    int32_t squares;         /* 4^s */
    int32_t p_dec;           /* P' = ceil(P / D) */
    int32_t d;               /* D = 2^(s-k) */
    int32_t fft_len;         /* M, the ramp filter's FFT length (>= 2N-1) */
    int32_t max_width;       /* max over squares of W_q (local columns) */
    int32_t z_run;           /* voxels along z per backprojection thread */
    int64_t filtered_bytes;  /* P*N*N * sizeof(store) */
    int64_t workspace_bytes; /* sum_q W_q * P' * N * sizeof(store); 0 when s = 0 */
    int64_t volume_bytes;    /* N_z*N*N*4 */
    int64_t updates;         /* N*N*N_z*P', voxel-angle updates of one reconstruction */
} fdkod_info;

/* Validate parameters without touching a device.  Same checks and codes as
 * fdkod_plan_create's first step. */
fdkod_status fdkod_validate(const fdkod_params* prm);

/* Create a plan on `device`: validates, builds the angle, decimation and
 * ramp-filter tables on the host in FP64 (rounded to FP32), runs the bounds
 * kernel (eq. (1) at the square vertices, Sec. 2.1) and synchronises once to
 * size the workspace.  *out receives the plan; on failure *out is NULL. */
fdkod_status fdkod_plan_create(const fdkod_params* prm, int device, fdkod_plan_t* out);

/* Release a plan's device tables.  NULL is accepted. */
fdkod_status fdkod_plan_destroy(fdkod_plan_t plan);

/* Copy the plan's sizes into *info (host memory). */
fdkod_status fdkod_plan_info(fdkod_plan_t plan, fdkod_info* info);

/* Re-enqueue the bounds kernel (Sec. 2.1, eq. (1) at the vertices of every
 * square, for every original and decimated angle).  It rewrites the plan's
 * device tables with the values fdkod_plan_create computed.  Not thread-safe
 * against concurrent use of the same plan. */
fdkod_status fdkod_bounds(fdkod_plan_t plan, fdkod_stream_t stream);

/* Ramp filtering, the initial convolution of Sec. 3 (textbook FDK): cosine
 * pre-weight R / sqrt(R^2 + a^2 + b^2), then linear convolution of every
 * detector row with the spatial Ram-Lak kernel (unit spacing, zero outside
 * the detector), by FFT of length M in FP32.  proj: float32 [P][N][N];
 * filt: store type [P][N][N].  The buffers must not overlap. */
fdkod_status fdkod_filter(fdkod_plan_t plan, const float* proj, void* filt,
                          fdkod_stream_t stream);

/* Decomposition (Sec. 2.1, eq. (7)): for every square q, detector row v,
 * decimated angle m and local column j,
 *   Y_q[m][v][j] = sum_p w[m][p] * Lin(filt[p][v][.], a_c(beta_p) + u0_q + j)
 * with linear interpolation, zero outside the detector, and the triangle
 * decimation weights w.  Writes the workspace.  No-op when s = 0. */
fdkod_status fdkod_decompose(fdkod_plan_t plan, const void* filt, void* ws,
                             fdkod_stream_t stream);

/* Reconstruction (Sec. 2.2, eq. (6)): cone-weighted bilinear backprojection
 * of every square from its decimated data (s > 0, reads ws) or of the whole
 * slice from the filtered projections (s = 0, direct FDK, reads filt):
 *   f = (pi / P') sum_m U^-2 Bil(Y_q[m], v*, tau),  U = depth / R,
 * tau the local column of eq. (1)'s position, v* = b + (N-1)/2 (eq. (9)).
 * Overwrites every voxel of vol (float32 [N_z][N][N]). */
fdkod_status fdkod_reconstruct(fdkod_plan_t plan, const void* filt, const void* ws,
                               float* vol, fdkod_stream_t stream);

/* fdkod_decompose followed by fdkod_reconstruct on the same stream. */
fdkod_status fdkod_backproject(fdkod_plan_t plan, const void* filt, float* vol,
                               void* ws, fdkod_stream_t stream);

/* ------------------------------------------------------------------ tuning
 * Kernel shapes are chosen per plan: the backprojection's slices per thread
 * and LDS footprint / angles per stage, and the decimation's column chunks.
 * fdkod_plan_create picks a default that holds the plan's geometry (or the
 * entry of the file named by the environment variable FDKOD_TUNE_CACHE);
 * fdkod_tune measures the alternatives.                                    */
typedef struct {
    int32_t z_run;            /* slices per backprojection thread: 16 or 32 */
    int32_t tile_w, tile_h;   /* LDS footprint of a 16 x 16 x z_run block: 32/64 x 48/64 */
    int32_t angles_per_stage; /* angles staged in LDS per barrier: 1, 2 or 4 */
    int32_t decim_chunks;     /* 64-column chunks per decimation wavefront: 1, 2, 4 or 8 */
    float bp_ms;              /* backprojection time measured by fdkod_tune (else 0) */
    float decim_ms;           /* decimation time measured by fdkod_tune (else 0) */
} fdkod_tuning;

/* The plan's current kernel shapes. */
fdkod_status fdkod_get_tuning(fdkod_plan_t plan, fdkod_tuning* out);

/* Apply kernel shapes; E_UNSUPPORTED if the variant does not exist or its LDS
 * footprint cannot hold the plan's block footprint (the plan is unchanged). */
fdkod_status fdkod_set_tuning(fdkod_plan_t plan, const fdkod_tuning* t);

/* Autotuner: times every valid backprojection variant (fdkod_reconstruct)
 * and decimation chunking (fdkod_decompose) on the caller's buffers and
 * stream (one warm-up and three timed runs each), applies the fastest and
 * returns it.  Overwrites vol and ws.  Synchronises the stream; not for use
 * under graph capture.  When FDKOD_TUNE_CACHE names a file, the choice is
 * appended to it, keyed by device and plan parameters. */
fdkod_status fdkod_tune(fdkod_plan_t plan, const void* filt, void* ws, float* vol,
                        fdkod_stream_t stream, fdkod_tuning* out);

/* ---------------------------------------------------------------- cost model
 * Sec. 2.2 prices FDK-OD as reconstruction C1 N^4 / 2^s (eq. (6)) plus
 * decomposition C2 N^3 2^s (eq. (7)), with the optimum 2^s = sqrt(C1 N / C2)
 * (eq. (8)).  The library counts both terms exactly for a parameter set (host
 * arithmetic in FP64, no device): the voxel-angle updates N^2 N_z P' of the
 * reconstruction (N^2 N_z P for s = 0) and the cropped samples
 * (sum_q W_q) P N of the decomposition, W_q the squares' local grid widths
 * from eq. (1) at their vertices (0 for s = 0).                              */
fdkod_status fdkod_cost_counts(const fdkod_params* prm, int64_t* cropped, int64_t* updates);

/* The s in [0, s_max] (skip clipped to s) whose predicted time
 * c1_ms * updates + c2_ms * cropped is least, and that time (ms_out may be
 * NULL): eq. (8)'s optimum, taken over the exact counts; c1_ms / c2_ms are a
 * device's measured cost per update / per cropped sample. */
fdkod_status fdkod_choose_s(const fdkod_params* prm, int32_t s_max, double c1_ms, double c2_ms, int32_t* s_out,
                            double* ms_out);

/* ------------------------------------------------------------------ batches
 * Many volumes of different sizes reconstructed together (the decomposition of
 * Sec. 2.1 applied to every volume): one bounds launch over all volumes'
 * squares, one filter launch per FFT length over the volumes too small to fill
 * the GPU alone (larger ones keep a launch each), one grouped decimation launch
 * over all volumes' (square, row) tasks and one persistent backprojection
 * launch whose workgroups take (volume, square, 16 x 16 tile, slab) items from
 * a ticket queue, largest first.  The launch sequence can be captured in a
 * hipGraph. */
typedef struct fdkod_batch_s* fdkod_batch_t;

/* Create a batch of `count` plans (1..4096) on `device`; every plan is
 * validated and created as by fdkod_plan_create.  All must share the store
 * type.  Synchronises. */
fdkod_status fdkod_batch_create(const fdkod_params* prms, int32_t count, int device,
                                fdkod_batch_t* out);
fdkod_status fdkod_batch_destroy(fdkod_batch_t batch);

/* The plan of volume `index` (owned by the batch; do not destroy). */
fdkod_status fdkod_batch_plan(fdkod_batch_t batch, int32_t index, fdkod_plan_t* out);

/* Bind the device buffers of every volume (host arrays of `count` device
 * pointers, laid out as for the single-plan calls; ws[i] may be NULL when
 * volume i has s = 0).  Copies the pointer tables to the device
 * (synchronously) and invalidates a captured graph. */
fdkod_status fdkod_batch_bind(fdkod_batch_t batch, const float* const* proj, void* const* filt,
                              void* const* ws, float* const* vol);

/* Enqueue the grouped bounds and filters, the grouped decimation and the
 * persistent backprojection on `stream`.  Asynchronous, allocates nothing;
 * capture-safe (the ticket counter is cleared by a kernel, not a memset). */
fdkod_status fdkod_batch_run(fdkod_batch_t batch, fdkod_stream_t stream);

/* Capture fdkod_batch_run on `stream` (not the null stream) into a hipGraph
 * and instantiate it; fdkod_batch_replay launches it on any stream. */
fdkod_status fdkod_batch_capture(fdkod_batch_t batch, fdkod_stream_t stream);
fdkod_status fdkod_batch_replay(fdkod_batch_t batch, fdkod_stream_t stream);

/* Autotuner for the batch: times the persistent backprojection variants that
 * hold every volume's footprint and the decimation chunkings on the bound
 * buffers, applies the fastest (and invalidates a captured graph). */
fdkod_status fdkod_batch_tune(fdkod_batch_t batch, fdkod_stream_t stream, fdkod_tuning* out);

/* Work items of the persistent launch, its workgroups, and the direct-
 * equivalent voxel-angle updates of one run (sum over volumes N^2 N_z P). */
fdkod_status fdkod_batch_info(fdkod_batch_t batch, int64_t* items, int32_t* blocks,
                              int64_t* updates_eq);

/* Copy the bounds tables to host memory (any pointer may be NULL to skip):
 *   ac_p    float [4^s][P]   a_c(beta_p), centre trajectory at original angles
 *   ac_m    float [4^s][P']  a_c(beta'_m) at decimated angles
 *   amin_m  float [4^s][P']  min of eq. (1) over the square's vertices
 *   amax_m  float [4^s][P']  max of eq. (1) over the square's vertices
 *   u0      int32 [4^s]      local column origin (detector index offset)
 *   width   int32 [4^s]      W_q, local columns
 *   rect    int32 [4^s][4]   x0, x1, y0, y1 voxel index ranges (half-open)
 * Synchronises with the plan's device. */
fdkod_status fdkod_get_bounds(fdkod_plan_t plan, float* ac_p, float* ac_m, float* amin_m,
                              float* amax_m, int32_t* u0, int32_t* width, int32_t* rect);

/* ---------------------------------------------------------------------------
 * Learned decimation filter.  Sec. 2.1 leaves the low-pass filter of the
 * angular decimation open (the quality depends on its implementation).  This
 * filter adds a trained correction R to the plan's decimation T (the
 * triangle, or the windowed sinc) of every square q and detector row v:
 *
 *   Y_q[m][v][j] = T[m][v][j] + R[m][v][j],   R = conv2(ReLU(conv1(S)))
 *   conv1: H_k(p, j) = b1_k + sum_{a,b<5} W1[k][a][b] S((p + (a-2) d) mod P, j + b - 2)
 *   R(m, j) = b2 + sum_{k,a,b<5} W2[k][a][b] A_k((c(m) + (a-2) d) mod P, j + b - 2)
 *
 * S(p, j) = Lin(filt[p][v][.], a_c(beta_p) + u0_q + j) is the cropped and
 * shifted full-rate sub-sinogram (zero outside the columns [0, W_q)); with
 * the cubic shift Lin is Keys' cubic convolution, as in the decimation;
 * A = ReLU(H) on [0, W_q) and zero outside, c(m) = floor(m P / P' + 1/2) mod P
 * the original angle nearest to beta'_m, d = max(1, D / 4), k < 16 channels.
 * Parameters: FDKOD_LEARNED_PARAMS BF16 values on the device, in the order
 * W1 [16][5][5], b1 [16], W2 [16][5][5], b2.  Both convolutions multiply BF16
 * operands (S, the weights, the activations) with FP32 accumulation.  With
 * W2 = 0 and b2 = 0 the result is the plan's decimation.  Requires s > 0,
 * detector rows and W_q <= 252 for every square (FDKOD_E_UNSUPPORTED
 * otherwise).
 * ------------------------------------------------------------------------- */
#define FDKOD_LEARNED_PARAMS 817

/* fdkod_decompose followed by the learned correction: ws receives Y. */
fdkod_status fdkod_learned_decompose(fdkod_plan_t plan, const void* filt, void* ws,
                                     const uint16_t* weights, fdkod_stream_t stream);

/* Training: grad (float32 [FDKOD_LEARNED_PARAMS], overwritten) receives the
 * gradient of sum_{q,m,v,j} R[m][v][j] dws[m][v][j] with respect to the
 * parameters.  dws: float32, the workspace layout (workspace_bytes / element
 * size elements).  The BF16 roundings of the forward pass are held fixed.
 * Workgroup partial sums are added in a fixed order: the same inputs give the
 * same bits on every call.  Calls that overlap on one plan (two streams)
 * race on the plan's partial-sum buffer. */
fdkod_status fdkod_learned_backward(fdkod_plan_t plan, const void* filt, const float* dws,
                                    const uint16_t* weights, float* grad, fdkod_stream_t stream);

/* Transpose of fdkod_reconstruct for s > 0: dws (float32, workspace layout,
 * overwritten) receives, for every voxel with value resid and every decimated
 * angle, resid * (pi / P') U^-2 spread over the four samples of its bilinear
 * interpolation.  resid: float32 [N_z][N][N].  Deterministic: each FP32
 * contribution is rounded to a multiple of 2^-e and the multiples are summed
 * exactly in int64 (e chosen per call from max |resid| so that no sum can
 * overflow; the step 2^-e is below 2^-60 of the largest possible sum), then
 * every entry is rounded once to FP32; a resid that holds a value that is
 * not finite gives NaN.  The plan holds the int64 sums: the first call
 * allocates them (8 bytes per workspace element), a later call that needs
 * more grows them (hipFree waits for the device), and calls that overlap on
 * one plan race on them.  Plans with cone-corrected rows (FDKOD_ROWS_CONE)
 * return FDKOD_E_UNSUPPORTED. */
fdkod_status fdkod_reconstruct_adjoint(fdkod_plan_t plan, const float* resid, float* dws,
                                       fdkod_stream_t stream);

/* The learned filter on a band of detector rows (the slab mode below; a band
 * holds the rows eq. (9) maps a slab of slices to), for training on slabs:
 * the same results, row for row, as the whole-volume calls on those rows.
 * Buffers: filt_band store type [P][nrows][N]; ws_band / dws_band the
 * workspace blocks [P'][nrows][W_q] of square q from element offset
 * nrows P' sum_{q' < q} W_q' (store type / float32); resid_slab float32
 * [nzs][N][N], slices [z0, z0 + nzs).  fdkod_reconstruct_adjoint_slab is the
 * transpose of fdkod_reconstruct_slab: FDKOD_E_ARG when the band misses a row
 * the slab samples. */
fdkod_status fdkod_learned_decompose_band(fdkod_plan_t plan, const void* filt_band, int32_t v0, int32_t nrows,
                                          void* ws_band, const uint16_t* weights, fdkod_stream_t stream);
fdkod_status fdkod_learned_backward_band(fdkod_plan_t plan, const void* filt_band, int32_t v0, int32_t nrows,
                                         const float* dws_band, const uint16_t* weights, float* grad,
                                         fdkod_stream_t stream);
fdkod_status fdkod_reconstruct_adjoint_slab(fdkod_plan_t plan, const float* resid_slab, int32_t v0, int32_t nrows,
                                            int32_t z0, int32_t nzs, float* dws_band, fdkod_stream_t stream);

/* Squared-error residual on the current device: resid = 2 (f - ref) and
 * *loss = sum (f - ref)^2 (float64, on the device), over count floats. */
fdkod_status fdkod_sq_residual(const float* f, const float* ref, float* resid, double* loss,
                               int64_t count, fdkod_stream_t stream);

/* The same with a weight w: resid = 2 w (f - ref), *loss = w sum (f - ref)^2
 * (training on slabs of different energy weights each slab's squared error,
 * e.g. by the inverse of its target's energy). */
fdkod_status fdkod_sq_residual_weighted(const float* f, const float* ref, float* resid, double* loss,
                                        int64_t count, float weight, fdkod_stream_t stream);

/* One AdamW step on the current device over count float32 master weights
 * (bias-corrected moments m1, m2; decoupled weight decay), then their BF16
 * copy w_bf16 (round to nearest even).  step counts from 1. */
fdkod_status fdkod_adamw_step(float* master, float* m1, float* m2, const float* grad,
                              uint16_t* w_bf16, int32_t count, int32_t step, float lr, float beta1,
                              float beta2, float eps, float weight_decay, fdkod_stream_t stream);

/* ---------------------------------------------------------------------------
 * Low-memory reconstruction by slabs.  Sec. 2.2: eq. (9) gives the detector
 * rows a slice uses, so only a band of rows of every projection has to be
 * resident, and the decomposition and reconstruction of a part of the volume
 * need only the matching part of the data.
 *
 * A slab is the output slices [z0, z0 + nzs).  Its band is the detector rows
 * [v0, v0 + nrows) that eq. (9) maps the slab's voxels to at any angle (depth
 * between R - (N-1)/sqrt(2) and R + (N-1)/sqrt(2)), the two rows of each
 * bilinear sample and one row of margin on each side, widened to even row
 * boundaries and clipped to the detector.  Band buffers hold only those rows:
 *   projection band  float32 [P][nrows][N]
 *   filtered band    store type [P][nrows][N]
 *   workspace band   store type, square q's block [P'][nrows][W_q] from
 *                    element offset nrows P' sum_{q' < q} W_q'
 *   volume slab      float32 [nzs][N][N]
 * The band calls compute for those rows and slices exactly what the
 * whole-volume calls compute (bit for bit when v0 is even, as
 * fdkod_band_rows returns it, and z0 is a multiple of the plan's z_run; the
 * filter transforms detector rows 2k and 2k + 1 together).  Asynchronous on
 * `stream`; they allocate nothing.
 * ------------------------------------------------------------------------- */

/* The band of slab [z0, z0 + nzs) (host arithmetic, FP64). */
fdkod_status fdkod_band_rows(fdkod_plan_t plan, int32_t z0, int32_t nzs, int32_t* v0, int32_t* nrows);

/* fdkod_filter on the rows [v0, v0 + nrows) held by proj_band. */
fdkod_status fdkod_filter_band(fdkod_plan_t plan, const float* proj_band, int32_t v0, int32_t nrows,
                               void* filt_band, fdkod_stream_t stream);

/* fdkod_decompose of the rows [v0, v0 + nrows); no-op when s = 0. */
fdkod_status fdkod_decompose_band(fdkod_plan_t plan, const void* filt_band, int32_t v0, int32_t nrows,
                                  void* ws_band, fdkod_stream_t stream);

/* fdkod_reconstruct of slices [z0, z0 + nzs) from a band (ws_band when s > 0,
 * filt_band when s = 0).  FDKOD_E_ARG when the band misses a row the slab
 * samples. */
fdkod_status fdkod_reconstruct_slab(fdkod_plan_t plan, const void* filt_band, const void* ws_band,
                                    int32_t v0, int32_t nrows, int32_t z0, int32_t nzs, float* vol_slab,
                                    fdkod_stream_t stream);

/* Device bytes of the work buffer fdkod_reconstruct_streamed needs for slabs
 * of nzs slices (rounded up to a multiple of z_run): two projection bands,
 * one filtered and one workspace band, two volume slabs. */
fdkod_status fdkod_streamed_bytes(fdkod_plan_t plan, int32_t nzs, int64_t* bytes);

/* The whole reconstruction from host memory, slab by slab: host_proj float32
 * [P][N][N] and host_vol float32 [N_z][N][N] are host buffers (page-locked
 * for overlap).  Each slab's band is copied in on copy_stream while the
 * previous slab is filtered, decomposed and reconstructed on `stream`, and
 * each finished slab is copied out on copy_stream.  copy_stream may be NULL
 * (everything on `stream`).  work: device buffer of fdkod_streamed_bytes.
 * Synchronous: returns when host_vol is complete.  Creates and destroys its
 * own events; allocates no device memory. */
fdkod_status fdkod_reconstruct_streamed(fdkod_plan_t plan, const float* host_proj, float* host_vol,
                                        int32_t nzs, void* work, int64_t work_bytes, fdkod_stream_t stream,
                                        fdkod_stream_t copy_stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * fdkod_backproject_noalloc is fdkod_backproject with the workspace taken
 * from a fixed device array inside the library instead of a caller buffer:
 * the same decimation and backprojection kernels, the same result.  The array
 * holds FDKOD_NOALLOC_SCRATCH_BYTES bytes on every GPU the library runs on,
 * from the time the library's device code is loaded there until the process
 * ends.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); the caller passes the filtered projections and the volume
 * as for fdkod_backproject.  Plans whose workspace (fdkod_plan_info
 * workspace_bytes) exceeds the array return FDKOD_E_UNSUPPORTED.  s = 0
 * (direct FDK) needs no workspace.  All calls on one GPU share its array and
 * keep the last call's contents: calls that overlap in time on one GPU (on
 * several streams or host threads) race and give undefined results.  The
 * first call on a device looks up the array's device address (synchronously,
 * with that device made current and the caller's current device restored).
 * ------------------------------------------------------------------------- */
#define FDKOD_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

fdkod_status fdkod_backproject_noalloc(fdkod_plan_t plan, const void* filt, float* vol,
                                       fdkod_stream_t stream);

/* Checked builds (the library compiled with FDKOD_CHECKS defined): counts of
 * events that the plan's geometry is meant to rule out, per kind, summed over
 * every launch on the current device since the last reset:
 *   [0] backprojection z runs whose detector rows fall outside the block's
 *       staged footprint (they contribute zero)
 *   [1] backprojection columns outside the staged footprint (clamped)
 *   [2] decimation reads beyond the staged row segment
 *   [3] reserved (zero)
 * counts: host array of n (1..4) int64 values; reset != 0 clears the counters
 * after reading.  Synchronises the current device.  Unchecked builds return
 * FDKOD_E_UNSUPPORTED. */
fdkod_status fdkod_check_counts(int64_t* counts, int32_t n, int32_t reset);

/* Static text for a status code. */
const char* fdkod_status_str(fdkod_status st);

/* Thread-local text describing the last failure on this thread ("" if none). */
const char* fdkod_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t fdkod_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDKOD_H */
