/* ld.h -- C ABI of the MI355X lane-detection library (libld.so).
 *
 * The library runs, on one AMD Instinct MI355X (gfx950), the per-frame hot path of the
 * stereo lane detector of Fan & Dahnoun, "Real-Time Stereo Vision-Based Lane Detection
 * System" (arXiv 1807.02752): from a left grey image and its disparity map to lane
 * positions.  Every step runs in hand-written HIP kernels; nothing comes back to the host
 * between steps.
 *
 * Conventions shared by every call
 *  - Every function returns ld_status; no exception or abort crosses the ABI.
 *  - Image buffers are DEVICE memory holding `batch` frames stacked vertically:
 *    batch * height rows of `pitch` bytes each, frame b starting at row b * height.
 *    Pixel (u, v) of frame b is at byte (b * height + v) * pitch + u * elem_size.
 *  - Output buffers are DEVICE memory owned by the caller, unless stated otherwise.
 *    Nullable outputs are skipped when NULL.
 *  - Calls are asynchronous on `hip_stream` (a hipStream_t; NULL = the default stream).
 *    Only argument checks are synchronous: a bad argument returns LD_E_INVAL and
 *    enqueues nothing.  Inputs must stay alive until the enqueued work completes.
 *  - A frame object (ld_frame) owns its device scratch and the state carried between
 *    steps (road profile, V_p tables, edge lists, energies).  Use one host thread per
 *    frame object at a time; calls on one frame object must use one stream, or the caller
 *    must order the streams.
 *  - Per-frame failures of the method are not errors: they are reported in
 *    ld_lanes.flags (LD_FLAG_*) and as NaN rows of the V_p tables.
 *  - Coordinates: u = column 0..width-1, v = row 0..height-1, v_max = height - 1.
 */
#ifndef LD_H
#define LD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LD_OK = 0,
    LD_E_INVAL = -1,   /* bad argument (null/unaligned pointer, size out of range, ...) */
    LD_E_NOMEM = -2,   /* device scratch could not be allocated / not admitted by the budget */
    LD_E_HIP = -3,     /* a HIP runtime call failed (also deferred kernel errors, see ld_sync) */
    LD_E_STATE = -4,   /* a step was called before the step it depends on */
    LD_E_BUSY = -5     /* the server's queue for this resolution class is full: retry later */
} ld_status;

/* Disparity pixel formats.  0 marks an invalid (rejected) pixel in every format; an F32
 * pixel is also invalid if it is not finite or not positive. */
typedef enum {
    LD_DISP_U8 = 0,     /* uint8, disparity in px */
    LD_DISP_F32 = 1,    /* float32, subpixel disparity in px */
    LD_DISP_U16Q4 = 2   /* uint16, disparity in 1/16 px */
} ld_disp_format;

/* Per-frame flags reported in ld_lanes.flags. */
enum {
    LD_FLAG_NOROAD = 1,     /* no road profile could be fitted, or fewer than 8 road rows */
    LD_FLAG_NOVP = 2,       /* the V_px fit failed */
    LD_FLAG_NOCONS_Y = 4,   /* road-profile RANSAC ended without reaching the inlier fraction */
    LD_FLAG_NOCONS_X = 8,   /* V_px RANSAC ended without reaching the inlier fraction */
    LD_FLAG_FALLBACK = 16   /* the pruned search fell back to the full search */
};

#define LD_MAX_LANES 16

/* Parameters of the method.  ld_params_default() fills the constants printed in the paper
 * (Sec. 2.2-2.4) and the readings taken where it is silent. */
typedef struct ld_params {
    int32_t chi;           /* V_px band half-height, Sec. 2.3.2: 25 */
    int32_t tau_y_max;     /* v-disparity DP jump bound, Eq. vpy_estimation: 6 */
    int32_t tau_x_max;     /* V_px DP jump bound, Eq. dense_vpx_estimation: 5 (max 5) */
    int32_t lambda_y;      /* DP smoothness weights (not given in the paper): 1, 1 */
    int32_t lambda_x;
    double tr_y;           /* RANSAC inlier tolerances, Sec. 2.2 and 2.3.3: 4, 16 */
    double tr_x;
    int32_t eps_num;       /* RANSAC exit fraction eps = eps_num / eps_den = 99/100 */
    int32_t eps_den;
    double varpi;          /* road tolerance |D - f(v)| <= varpi, Sec. 2.3.1: 3 */
    int32_t edge_t;        /* Sobel magnitude threshold: 100 */
    double sigma_g;        /* width of w_g, Eq. sigma_g: 3.5 */
    int32_t nu;            /* M_0 box half-sizes (columns, rows), Sec. 2.4: 1, 3 (fixed) */
    int32_t varsigma;
    int32_t n_hyp;         /* RANSAC samples scored per round (not given): 64 (1..64) */
    int32_t max_rounds;    /* RANSAC round cap (not given): 16 (1..64) */
    double rho_lpv;        /* lane threshold: E < rho_lpv * min E (not given): 0.25 */
    int32_t d_nms;         /* minimum lane separation in px; 0 -> max(8, width/64) */
    int32_t weight_squared;/* 0: w_g exponent as printed; 1: squared (Gaussian) reading */
    int32_t vote;          /* 0: q = G_x w_g (Eq. sigma_g); 1: the authors' prior vote named at
                              the opening of Sec. 2.4, |grad(e)| cos(theta_e - theta_Vp), with
                              theta_e the tangent (-G_y, G_x) and theta_Vp the ray from V_p(v)
                              to the pixel (an A/B variant; the rest of the path unchanged) */
    uint64_t seed;         /* Philox key word 0 of the RANSAC samples */
} ld_params;

/* Lanes of one frame.  u_start is the column of the lane on row v_max (it may lie outside
 * the image: candidates span -width/2 .. 1.5*width), sorted ascending. */
typedef struct ld_lanes {
    int32_t n;                      /* number of lanes, 0..LD_MAX_LANES */
    int32_t flags;                  /* LD_FLAG_* */
    int32_t v_h;                    /* first road row (height if none) */
    int32_t v_end;                  /* top row reached by the lane tracks */
    int32_t u_start[LD_MAX_LANES];
    float energy[LD_MAX_LANES];     /* candidate energy of each lane (negative) */
} ld_lanes;

typedef struct ld_frame_s* ld_frame;

/* Fill p with the defaults described above. */
void ld_params_default(ld_params* p);

/* Create a frame object for `batch` frames of width x height pixels whose disparity is in
 * format `fmt` with bins 0..d_max.  Limits: 8 <= width <= 4096, 8 <= height <= 4096,
 * 1 <= batch <= 65535, 1 <= d_max <= 1023, width * height * (2 chi + 1) < 2^27 (the row DP
 * holds its energies in 32 bits; 1920 x 1080 with chi = 25 fits).  p may be NULL (defaults).  The scratch is
 * allocated on the current HIP device (LD_E_NOMEM if it does not fit). */
ld_status ld_frame_create(int32_t width, int32_t height, int32_t batch, int32_t fmt, int32_t d_max,
                          const ld_params* p, ld_frame* out);

/* Free a frame object (synchronises its last stream first).  NULL is accepted. */
ld_status ld_frame_destroy(ld_frame f);

/* Process only the first n frames (1 <= n <= batch) in the following calls.  Default:
 * batch. */
ld_status ld_frame_set_active(ld_frame f, int32_t n);

/* Step 1 (Sec. 2.2): v-disparity histogram, DP path on it, road profile beta by RANSAC
 * (Alg. "beta estimation"), V_py(v) (Eq. vpy_equation) and the road rows.
 *  disp, disp_pitch : disparity frames (see above), pitch >= width * elem_size.
 *  stream_ids       : nullable device array of n uint64, Philox key word 1 per frame
 *                     (NULL: 0).
 *  frame_idx        : nullable device array of n int64, Philox counter word 0 per frame
 *                     (NULL: the frame's index in the batch).
 *  vdisp_out        : nullable device int32 n x height x (d_max+1), row-major m_y(v, d).
 *  beta_out         : nullable device double n x 3, road profile f(v) = b0 + b1 v + b2 v^2
 *                     (NaN if no fit). */
ld_status ld_vdisp(ld_frame f, const void* disp, int64_t disp_pitch, const uint64_t* stream_ids,
                   const int64_t* frame_idx, int32_t* vdisp_out, double* beta_out, void* hip_stream);

/* Step 2 (Sec. 2.3): Sobel gradient on the road surface, sparse V_px votes
 * (Eq. sparse_vpx_estimation), band accumulation (Alg. "Dense V_px accumulation"), DP path
 * (Eq. dense_vpx_estimation) and V_px by RANSAC (Alg. "gamma estimation",
 * Eq. vpx_estimation).  Needs a prior ld_vdisp on this frame object (else LD_E_STATE).
 *  grey, grey_pitch : uint8 grey frames, pitch >= width, height * pitch < 2^31 - 4096.
 *  disp, disp_pitch : the same disparity frames as given to ld_vdisp.
 *  stream_ids, frame_idx : as in ld_vdisp (they key the V_px RANSAC samples).
 *  seed_gamma       : nullable device double n x 5, a raw-basis quartic in v used as
 *                     RANSAC hypothesis 0 (a learned or tracked seed); a row whose first
 *                     coefficient is NaN carries no seed.
 *  vp_out           : nullable device double n x height x 2, (V_px, V_py) per row, NaN
 *                     outside the road rows. */
ld_status ld_vp_ransac(ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp, int64_t disp_pitch,
                       const uint64_t* stream_ids, const int64_t* frame_idx, const double* seed_gamma,
                       double* vp_out, void* hip_stream);

/* Step 3 (Sec. 2.4): weights w_g (Eq. sigma_g), M_0, M_1 and the energy of every lane
 * candidate (Eq. lane_energy along Eq. lane_visualisation).  Needs a prior ld_vp_ransac.
 *  cand_mask  : nullable device uint8 n x (2*width); 0 prunes a candidate (its energy is
 *               reported as 0 and it cannot be a lane).  NULL = the full search.
 *  energy_out : nullable device float n x (2*width); candidate i starts at column
 *               i - width/2 on row v_max. */
ld_status ld_lane_energy(ld_frame f, const uint8_t* cand_mask, float* energy_out, void* hip_stream);

/* Step 4 (Alg. "Lane position validation"): local minima of the energies, threshold and
 * suppression of nearby weaker minima; lane curves by iterating Eq. lane_visualisation.
 * Needs a prior ld_lane_energy.
 *  lanes_out  : n ld_lanes, device or host-pinned memory (written by a kernel).
 *  curves_out : nullable device float n x LD_MAX_LANES x height, u of each lane per row,
 *               NaN outside [v_end, v_max]. */
ld_status ld_peaks(ld_frame f, ld_lanes* lanes_out, float* curves_out, void* hip_stream);

/* All steps in order: ld_vdisp + ld_vp_ransac + ld_lane_energy (full search) + ld_peaks. */
ld_status ld_detect(ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp, int64_t disp_pitch,
                    const uint64_t* stream_ids, const int64_t* frame_idx, ld_lanes* lanes_out, float* curves_out,
                    void* hip_stream);

/* Bilateral pre-filter of the grey images ahead of the gradient (Sec. 2.3.1, Eq.
 * bilateral_filter with its spatial weight w_s and range weight w_r): each output pixel is
 * sum w_s w_r I / sum w_s w_r over the (2 rho + 1)^2 window around it, w_s = exp(-(du^2 + dv^2)
 * / sigma_s^2), w_r = exp(-(dI / 255)^2 / sigma_r^2), window pixels outside the frame excluded,
 * rounded half up to u8.  The arithmetic is fixed so the rounding is reproducible: FP32 weight
 * tables (each the FP64 exponential of the float sigmas, rounded to float), FP32 sums in window
 * order (rows top to bottom, each left to right; numerator by fused multiply-add), IEEE quotient.
 * Pass `out` as the grey image of ld_vp_ransac / ld_detect / ld_detect_pruned to run the paper's
 * pipeline with the filter.  The paper uses rho 5 (11 x 11), sigma_s 300, sigma_r 0.3.
 *  grey, grey_pitch : device uint8 n x height x grey_pitch (n = active frames), >= width.
 *  out, out_pitch   : device uint8 n x height x out_pitch, >= width; must not overlap grey.
 *  rho              : 1..5.   sigma_s, sigma_r : finite, > 0.
 *  road_rows        : 0 filters every row; 1 only rows v_h - 1 .. height - 1 of frames with a
 *                     road (all that the later steps read of the grey image), after ld_vdisp on
 *                     f (LD_E_STATE before it); the other rows of out are not written.
 * LD_E_INVAL for invalid arguments or overlapping images; nothing is enqueued then. */
ld_status ld_bilateral(ld_frame f, const uint8_t* grey, int64_t grey_pitch, uint8_t* out, int64_t out_pitch,
                       int32_t rho, float sigma_s, float sigma_r, int32_t road_rows, void* hip_stream);

/* Lane tracking across frames.  The paper names a tracking algorithm as future work (Sec. 4)
 * and defines none; this one filters each lane's start column on row v_max:
 *  - predict every track, x_hat = x + dx;
 *  - a frame flagged LD_FLAG_NOROAD or LD_FLAG_NOVP has no detections;
 *  - assign detections (ld_lanes.u_start) to predicted tracks greedily, the closest pair
 *    |u - x_hat| first (ties: lower track slot, then lower lane index), pairs within `gate`;
 *  - matched: r = u - x_hat, x = x_hat + alpha r, dx = dx + beta r, hits + 1, misses = 0;
 *    unmatched: x = x_hat, misses + 1, dropped once misses > max_misses (the rest keep order);
 *  - unmatched detections start tracks (x = u, dx = 0, hits = 1, id = next_id++) while fewer
 *    than LD_MAX_LANES tracks live.
 * FP64 in the order written.  A track with hits >= confirm is a confirmed lane. */
typedef struct ld_track_state {
    int32_t n;                        /* live tracks, in slot order */
    int32_t next_id;                  /* id the next new track gets */
    int64_t frames;                   /* frames folded in */
    int32_t id[LD_MAX_LANES];
    int32_t hits[LD_MAX_LANES];       /* frames with a detection since the track's birth */
    int32_t misses[LD_MAX_LANES];     /* consecutive frames without one */
    double x[LD_MAX_LANES];           /* filtered start column on row v_max */
    double dx[LD_MAX_LANES];          /* filtered rate, columns per frame */
} ld_track_state;                     /* all zero: a stream without tracks */

typedef struct ld_track_params {
    double alpha;                     /* (0, 1]  (0.5) */
    double beta;                      /* [0, 1]  (0.1) */
    double gate;                      /* > 0, columns (24) */
    int32_t confirm;                  /* >= 1 (3): hits that confirm a track */
    int32_t max_misses;               /* >= 0 (5) */
} ld_track_params;

void ld_track_params_default(ld_track_params* tp);

/* Fold the lanes of the active frames of f into their streams' tracker states, one frame per
 * state: frame b updates states[state_index[b]] (state_index: nullable device int32 per
 * frame, identity when NULL).  The indices of one call must be distinct (frames of one stream
 * go to successive calls, in frame order); a negative index skips the frame.
 *  lanes  : device ld_lanes per frame (from ld_peaks / ld_detect / ld_detect_pruned).
 *  states : device ld_track_state array, updated in place.
 * LD_E_INVAL for NULL pointers or parameters out of range. */
ld_status ld_track(ld_frame f, const ld_lanes* lanes, ld_track_state* states, const int32_t* state_index,
                   const ld_track_params* tp, void* hip_stream);

/* Disparity maps of rectified stereo pairs (Sec. 2.1): NCC block matching on memorised block
 * statistics (Eq. ncc_1, Eq. sigma_l_1, Eq. sigma_r_1; the paper forms them from integral
 * images, the sweep here from running column sums, the same integers), search range
 * propagation row by row from the bottom (Eq. srp), left-right consistency check (Alg. "LRC
 * check").  A pixel is matched when its (2 rho + 1)^2 block lies in the image; disparity 0 means
 * no match, so the search runs over 1..d_max (the frame object's d_max, <= 255); a candidate
 * counts when the other image's block lies in the image and neither block is flat.  The cost is
 * (n P - S_l S_r) / (sqrt(n Q_l - S_l^2) sqrt(n Q_r - S_r^2)) (S block sums, Q sums of squares, P
 * the sum of products, n = (2 rho + 1)^2): integers exactly, the quotient in FP64 in that order;
 * the largest cost wins, ties to the smaller disparity.  The bottom matched row searches
 * 1..d_max; row v the union of [l - tau, l + tau] over the matched neighbours u-1..u+1 of row
 * v+1 with l > 0, or 1..d_max when none has one.  The right map is the same search from the
 * right image (the left block at x + d).  The checked map keeps l(u, v) when u - l >= 0 and
 * |l(u, v) - l_right(u - l, v)| <= tr_lrc, else 0.  The paper uses rho 3, tau 1, tr_lrc 3.
 *  left, right       : device uint8 n x height x pitch (n = active frames), pitches >= width.
 *  disp_out          : device uint8 n x height x disp_pitch: the checked map (an LD_DISP_U8
 *                      disparity for ld_vdisp / ld_detect).
 *  disp_lf, disp_rt  : device uint8 n x height x width each: the left and right maps (the
 *                      check needs both).
 *  rho 1..5, tau 0..255, tr_lrc >= 0.  LD_E_INVAL otherwise, or when the sweep's rows do not fit
 *  in LDS (width above about 2800 at rho 3). */
ld_status ld_stereo(ld_frame f, const uint8_t* left, int64_t left_pitch, const uint8_t* right, int64_t right_pitch,
                    int32_t rho, int32_t tau, int32_t tr_lrc, uint8_t* disp_out, int64_t disp_pitch, uint8_t* disp_lf,
                    uint8_t* disp_rt, void* hip_stream);

/* Scratch of ld_detect_noalloc, per GPU (64 MiB). */
#define LD_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* ld_detect for callers that cannot allocate device memory (work recorded under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the same kernels and results as
 * ld_frame_create + ld_detect + ld_frame_destroy with these sizes and parameters, but the
 * scratch is a fixed device array of LD_NOALLOC_SCRATCH_BYTES built into the library (each
 * GPU the library runs on holds its own copy from the first call there until the process
 * ends).  No device or host memory is allocated and nothing is freed.
 *  width, height, batch, fmt, d_max, p : as in ld_frame_create (LD_E_INVAL outside its
 *                     limits).  The frame object's scratch for these sizes must fit the
 *                     array, else LD_E_NOMEM and nothing is enqueued: about 6.1 MiB per
 *                     1242 x 375 frame (d_max 128; batch <= 10), 27.2 MiB per 1920 x 1080
 *                     frame (d_max 255; batch <= 2), 1.7 MiB per 640 x 192 frame.
 *  grey ... hip_stream : as in ld_detect.
 * The array keeps the last call's contents; every call on one GPU shares it, so calls that
 * may overlap on a GPU (other streams, other host threads) must be ordered by the caller:
 * overlapping calls race and their results are undefined.  The first call on a device
 * looks up that device's copy (a lock is taken then; later calls only read it). */
ld_status ld_detect_noalloc(int32_t width, int32_t height, int32_t batch, int32_t fmt, int32_t d_max,
                            const ld_params* p, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                            int64_t disp_pitch, const uint64_t* stream_ids, const int64_t* frame_idx,
                            ld_lanes* lanes_out, float* curves_out, void* hip_stream);

/* Wait for the frame object's last stream; a failure of enqueued work surfaces here as
 * LD_E_HIP. */
ld_status ld_sync(ld_frame f);

/* Static description of a status code. */
const char* ld_status_string(ld_status s);

/* Introspection: copy one piece of the device state of frame `b` into `dst` (device or
 * host memory, `bytes` bytes available), asynchronously on hip_stream.  Returns LD_E_INVAL
 * if `bytes` is too small.  Layouts (per frame):
 *   LD_STATE_INFO      int32[8]: flags, v_h, v_end, n_my, n_edges, n_votes, R, n_mx
 *   LD_STATE_MY_PATH   int32[2 * (d_max+1)]: x (row v) then y (disparity d) of the n_my
 *                      points of the v-disparity DP path that carry votes
 *   LD_STATE_BETA      ld_fit (see below)
 *   LD_STATE_GAMMA     ld_fit
 *   LD_STATE_TABLES    double[6 * height]: f, f', V_py, V_px, A_v, B_v (one row each;
 *                      A_v, B_v are the track coefficients u_v = B_v u_{v+1} + A_v)
 *   LD_STATE_ROWCOUNT  int32[height]: road edges per row
 *   LD_STATE_EDGES     ld_edge[height * width]: per-row edge buckets (row v at v * width)
 *   LD_STATE_MX_PATH   int32[height]: DP column c_v (0..2W-1) on road rows, -1 elsewhere
 *   LD_STATE_ENERGY    double[2 * width]
 *   LD_STATE_TRACE     int32[2 * 3 * max_rounds]: per RANSAC round (best hypothesis,
 *                      its inlier count, points in the round), beta then gamma
 *   LD_STATE_LANE_BITS uint8[4 * 16 * width]: network decisions of the last
 *                      ld_cnn_forward / ld_detect_pruned, band k at k * 16 * width
 *                      (ld_detect_pruned without the candidate mask, dilate < 0, evaluates
 *                      only the 60-column tiles whose band rows hold a voting road edge,
 *                      the only pixels it reads; the other tiles hold 0)
 *   LD_STATE_PRUNE     int32[16] of the last ld_detect_pruned: bands, fallback bits (1 plain
 *                      V_px search, 2 plain energies, 4 no seed, 8 window edge touched),
 *                      seed column c_s (-1 none), window lo, hi, pooled marking votes,
 *                      per-band argmax column [4] (-1 none), per-band votes [4], kept
 *                      candidates, 0
 *   LD_STATE_CAND_MASK uint8[2 * width]: candidate mask of the last ld_detect_pruned that pruned
 *     candidates (dilate >= 0); all ones before the first such call */
enum {
    LD_STATE_INFO = 0, LD_STATE_MY_PATH = 1, LD_STATE_BETA = 2, LD_STATE_GAMMA = 3, LD_STATE_TABLES = 4,
    LD_STATE_ROWCOUNT = 5, LD_STATE_EDGES = 6, LD_STATE_MX_PATH = 7, LD_STATE_ENERGY = 8, LD_STATE_TRACE = 9,
    LD_STATE_LANE_BITS = 10, LD_STATE_PRUNE = 11, LD_STATE_CAND_MASK = 12
};

/* A robust polynomial fit: coefficients in the variable s = (v - center) / 2^kshift, and
 * the same polynomial in raw v (reporting). */
typedef struct ld_fit {
    int32_t ok, flags, center, kshift, rounds, n_survivors;
    double coef[5];
    double raw[5];
} ld_fit;

/* One road edge pixel: column, Sobel gradient and V_px vote column (0..2W-1, -1 none). */
typedef struct ld_edge {
    int16_t u, gx, gy, bin;
} ld_edge;

ld_status ld_frame_read(ld_frame f, int32_t what, int32_t b, void* dst, int64_t bytes, void* hip_stream);

/* Kernel timing (tracing aid).  ld_frame_profile(f, 1) waits for the frame's last stream,
 * clears the accumulated times and brackets every following kernel launch with a pair of
 * HIP events recorded on the launch stream; 0 turns it off.  ld_frame_kernel_times waits
 * for the recorded events and writes, for the first n of the eleven kernels (0 v-disparity
 * histogram, 1 v-disparity DP + RANSAC, 2 edges and votes, 3 V_px accumulator and row DP,
 * 4 energies, 5 peaks, 6 network decisions, 7 seed, 8 windowed V_px DP, 9 candidate mask
 * and fallback check, 10 V_px RANSAC), the total milliseconds and launch counts (calls_out
 * nullable) since profiling was enabled. */
ld_status ld_frame_profile(ld_frame f, int32_t enable);
ld_status ld_frame_kernel_times(ld_frame f, double* ms_out, int64_t* calls_out, int32_t n);

/* ---------------------------------------------------------------------------------------
 * Learned candidate pruning (not part of the paper's method).
 *
 * A convolutional network, 3x3 convolutions 4 -> 16 -> 16 -> 1 channels with ReLU after the
 * first two and zero padding, looks at n_bands bands of 16 road rows per frame (band k, k = 0
 * at the bottom, starts at row (H-16) - ((R-16) k) / n_bands, R = H - v_h road rows; frames
 * with fewer than 16 road rows have no band).  Its 4 inputs per pixel are I/255,
 * sqrt(G_x^2 + G_y^2)/1020, atan2(G_y, G_x)/pi with the Sobel pair of the lane detector, and
 * the disparity residual clamp((D - f(v))/varpi, -4, 4) (-4 where D is invalid).  Its output
 * logit z scores "lane marking"; a pixel counts as marking when sigmoid(z) >= theta.  Weights
 * are FP32 masters with BF16 copies feeding MFMA tiles that accumulate in FP32.
 *
 * Parameters, LD_CNN_PARAMS floats in this order: w1[3][3][4][16] (row offset, column
 * offset, input, output), b1[16], w2[3][3][16][16], b2[16], w3[3][3][16][1], b3[1].
 *
 * Training (ld_cnn_train_step) runs the forward pass, the loss
 *   L = inv_norm * sum over labelled pixels of  pos_weight * y * softplus(-z) + (1 - y) * softplus(z),
 * the backward pass and, when lr > 0, one Adam step (beta1 0.9, beta2 0.999, eps 1e-8); the
 * gradient is reduced over the workgroups in a fixed order, so a step is deterministic.
 * Labels (u8, batch x n_bands x 16 x width): 1 marking, 0 not, 255 ignored.
 */
typedef struct ld_cnn_s* ld_cnn;

#define LD_CNN_PARAMS 3057

typedef struct ld_cnn_config {
    int32_t n_bands;      /* bands of 16 rows per frame, 1..4 (default 1) */
    float theta;          /* marking probability threshold, (0, 1) (0.5) */
    int32_t delta_x;      /* half width of the V_px search window around the seed, 1..127 (127) */
    int32_t dilate;       /* candidates kept on each side of a candidate whose track hits
                             marking, 0..64; -1 (default) keeps every candidate */
    int32_t min_votes;    /* fewest marking votes that make a seed (8) */
    int32_t max_batch;    /* frames per training step (sizes the gradient scratch) (32) */
    int32_t max_width;    /* widest frame trained on (1920) */
    int32_t seed_ransac;  /* 1: hypothesis 0 of the V_px RANSAC is the line through the band
                             estimates; 0 (default): RANSAC as in the plain search */
} ld_cnn_config;

void ld_cnn_config_default(ld_cnn_config* c);
/* params: host, LD_CNN_PARAMS floats, nullable (all zero).  Runs on the current device. */
ld_status ld_cnn_create(const ld_cnn_config* c, const float* params, ld_cnn* out);
ld_status ld_cnn_destroy(ld_cnn n);
/* Host copies of the FP32 master weights; set also clears the optimiser state. Synchronous. */
ld_status ld_cnn_set_params(ld_cnn n, const float* params);
ld_status ld_cnn_get_params(ld_cnn n, float* params);

/* Checkpoint (training resume).  ld_cnn_save writes, synchronously, one header line of JSON
 *   {"format": "ld_cnn_checkpoint", "version": 1, "params": 3057, "step": <Adam steps taken>,
 *    "dtype": "float32", "arrays": ["master", "adam_m", "adam_v"], "config": {...the ld_cnn_config}}
 * followed by the FP32 master weights, the Adam first and second moments (LD_CNN_PARAMS
 * little-endian float32 each, in that order).  ld_cnn_load creates a network on the current
 * device from such a file: weights, moments and step restored, so the next ld_cnn_train_step
 * continues the run exactly; the configuration is the file's, or *cfg when cfg is not NULL.
 * LD_E_INVAL for a file that cannot be opened or written, or whose header, parameter count or
 * size does not match (checked before any device call). */
ld_status ld_cnn_save(ld_cnn n, const char* path);
ld_status ld_cnn_load(const char* path, const ld_cnn_config* cfg, ld_cnn* out);

/* Network decisions for the active frames of f into f's band buffer (needs ld_vdisp on f;
 * LD_E_STATE otherwise).  prob_out: nullable device float batch x n_bands x 16 x width,
 * sigmoid(z) (0 where a frame has no band).  The frame format must have varpi > 0. */
ld_status ld_cnn_forward(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                         int64_t disp_pitch, float* prob_out, void* hip_stream);

/* Training labels from a finished plain detection of f (ld_detect / ld_peaks with curves):
 * 1 where a band pixel of row v lies within radius + radius_per_disp * f(v) columns of a
 * detected lane curve (f: the road disparity of the row, so that the label covers the marking
 * at every distance), else 0; 255 on frames without bands.  lanes: device batch entries;
 * curves: device batch x 16 x height. */
ld_status ld_cnn_labels(ld_cnn n, ld_frame f, const ld_lanes* lanes, const float* curves, float radius,
                        float radius_per_disp, uint8_t* labels_out, void* hip_stream);

/* One training step over the active frames of f (needs ld_vdisp on f).  loss_out (nullable,
 * device float) and grad_out (nullable, device LD_CNN_PARAMS floats) receive the loss and
 * gradient at the weights before the update.  LD_E_INVAL if active frames x n_bands x
 * ceil(width / 60) exceeds max_batch x n_bands x ceil(max_width / 60). */
ld_status ld_cnn_train_step(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                            int64_t disp_pitch, const uint8_t* labels, float pos_weight, float inv_norm, float lr,
                            float* loss_out, float* grad_out, void* hip_stream);

/* The whole path with the network narrowing the search, for the active frames of f:
 *  1. ld_vdisp, edges and votes as in ld_detect, the network's band decisions (with
 *     dilate < 0 only on the 60-column tiles of a band that hold a voting road edge);
 *  2. seed: the votes of marking edges in the bands, histogrammed per band; the pooled
 *     histogram's argmax c_s (ties to the smaller column) centres the window
 *     [c_s - delta_x, c_s + delta_x] of V_px columns; with seed_ransac, RANSAC hypothesis 0
 *     is the line through the argmax columns (at the ninth row of each band) of the lowest
 *     and the highest band with at least min_votes votes (a constant with one such band);
 *  3. the band accumulator and row DP inside that window, then RANSAC of the V_px fit;
 *  4. candidate mask: candidate i is kept if its track, evaluated on the band rows as
 *     u_v = fma(a_v, u_start, b_v) with a_{v_max} = 1, b_{v_max} = 0,
 *     a_v = B_v a_{v+1}, b_v = fma(B_v, b_{v+1}, A_v), column floor(u_v + 0.5), meets a
 *     marking pixel; kept candidates are dilated by `dilate`;
 *  5. energies of the kept candidates (0 for the others) and peaks.
 * seed_gamma (nullable device n x 5, as in ld_vp_ransac: a stream's previous fit) is hypothesis 0
 * of the V_px RANSAC of every frame for which step 2 drew no seed line (seed_ransac off, or a
 * fallback frame).
 * Fallback to the plain search (LD_FLAG_FALLBACK) for a frame: no seed (fewer than
 * min_votes marking votes, or a frame narrower than 128 columns), or the window path
 * touches an inner window edge -> plain
 * accumulator, DP and unseeded RANSAC; no lane, or a lane next to a pruned candidate ->
 * energies of every candidate and peaks again. */
ld_status ld_detect_pruned(ld_frame f, ld_cnn n, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                           int64_t disp_pitch, const uint64_t* stream_ids, const int64_t* frame_idx,
                           const double* seed_gamma, ld_lanes* lanes_out, float* curves_out, void* hip_stream);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of frames from many camera streams.
 *
 * The server owns, per resolution class, up to `inflight` batch engines (a frame object of
 * max_batch frames, device staging for the inputs, its own HIP stream and, if enabled, one
 * captured HIP graph of the whole path at the full batch whose empty slots are masked).
 * Admission: an engine is created when its device bytes fit both hbm_budget (with the other
 * engines) and the device's free memory (hipMemGetInfo, keeping 512 MiB spare): at
 * ld_server_create round-robin over the classes up to `inflight` per class, and later, at a
 * poll, for a class whose requests wait with no idle engine; a class that has no engine and no
 * room takes the place of idle engines of classes with nothing queued.  Requests of a class
 * without an engine wait in its queue until one is admitted.  ld_server_submit only queues a
 * request (FIFO per class; LD_E_BUSY when max_queue requests wait; LD_E_NOMEM only for a class
 * whose single engine exceeds hbm_budget).  ld_server_poll (non-blocking) collects finished
 * batches and starts new ones: a batch takes queued requests in order, skipping a stream that
 * already has a frame in flight (each stream's frames run in submission order), up to
 * max_batch, as soon as an engine of the class is idle, so requests that arrive while others
 * run join the next free engine.  Input frames are copied on the engine's own stream at the
 * start of their batch, so they must be complete (and stay alive) by the ld_server_submit call
 * that hands them over, until their result is returned.
 * Per-stream state stays in device memory: the last V_px fit (seed of the next frame's
 * RANSAC hypothesis 0 when seed_from_state is set) and a frame counter; Philox keys are
 * (seed, stream id) and counters use the stream's frame index, never the batch slot, so a
 * frame's result does not depend on what it was batched with.
 */
typedef struct ld_server_s* ld_server;

#define LD_MAX_CLASSES 4

typedef struct ld_server_config {
    int32_t n_classes;                      /* 1..LD_MAX_CLASSES */
    int32_t width[LD_MAX_CLASSES];
    int32_t height[LD_MAX_CLASSES];
    int32_t fmt[LD_MAX_CLASSES];            /* ld_disp_format */
    int32_t d_max[LD_MAX_CLASSES];
    int32_t max_batch[LD_MAX_CLASSES];      /* frames per engine launch, >= 1 */
    int32_t n_streams;                      /* stream ids 0..n_streams-1 */
    int32_t inflight;                       /* engines per class, 1..8 */
    int32_t max_queue;                      /* waiting requests per class, >= 1 */
    int32_t use_graphs;                     /* 1: replay a captured graph per engine */
    int32_t seed_from_state;                /* 1: seed V_px RANSAC with the stream's last fit (also in
                                               the pruned path, for frames without a seed line) */
    int32_t track;                          /* 1: fold every frame's lanes into its stream's tracker
                                               state (ld_track, default parameters); read it with
                                               ld_server_tracks */
    int64_t hbm_budget;                     /* bytes of device memory the engines may use */
    ld_cnn cnn;                             /* nullable: run ld_detect_pruned with this network
                                               (plain fallback per frame); read only, must
                                               outlive the server */
} ld_server_config;

/* One finished request.  Times are host seconds (steady clock) at submit and at the poll
 * that observed completion. */
typedef struct ld_server_result {
    int64_t request;
    int32_t stream_id;
    int32_t cls;
    int64_t frame_idx;                      /* the stream's frame counter for this frame */
    double t_submit;
    double t_done;
    ld_lanes lanes;
} ld_server_result;

/* Create a server on the current HIP device (p may be NULL: defaults). */
ld_status ld_server_create(const ld_server_config* cfg, const ld_params* p, ld_server* out);
/* Wait for all in-flight work and free everything.  NULL is accepted. */
ld_status ld_server_destroy(ld_server s);
/* Queue one frame of stream stream_id in class cls.  grey/disp are device buffers of one
 * frame (rows of the given pitches) that the caller keeps alive until the request's result
 * has been returned by ld_server_poll.  req_out (nullable) receives the request id. */
ld_status ld_server_submit(ld_server s, int32_t stream_id, int32_t cls, const uint8_t* grey, int64_t grey_pitch,
                           const void* disp, int64_t disp_pitch, int64_t* req_out);
/* Collect up to max_results finished requests (host memory) and start batches for queued
 * requests on idle engines.  Never blocks on the device. */
ld_status ld_server_poll(ld_server s, ld_server_result* results, int32_t max_results, int32_t* n_out);
/* Numbers of requests waiting in queues and in flight. */
ld_status ld_server_pending(ld_server s, int32_t* queued, int32_t* inflight);
/* Engines created per class and the device bytes they hold. */
ld_status ld_server_engines(ld_server s, int32_t* per_class /* LD_MAX_CLASSES */, int64_t* bytes);

/* Tracker state of one stream (config track = 1; LD_E_STATE otherwise), copied to host memory
 * `out` once the batches in flight have finished: it holds every frame of the stream that has
 * reached a batch (the server keeps at most one frame per stream in flight, so a stream's
 * frames are folded in order).  Blocks the calling thread. */
ld_status ld_server_tracks(ld_server s, int32_t stream_id, ld_track_state* out);

#ifdef __cplusplus
}
#endif

#endif /* LD_H */
