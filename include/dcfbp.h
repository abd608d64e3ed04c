/*
 * dcfbp.h -- C ABI of the MI355X (gfx950) Defrise-Clack shift-variant FBP library.
 *
 * The library computes, per cone-beam view lambda, the chain of the paper's
 * eq. 12 (Ye et al., "DRACO: Differentiable Reconstruction for Arbitrary CBCT
 * Orbits", Sec. 2.3-2.4):
 *
 *     f = A3d^T w_d A2d^T D w_red w_sino D A2d w_cos g
 *
 * split into four stages, each with its exact transpose:
 *
 *   dc_weight_radon   g  -> R  = A2d(w_cos g)                 (eq. 7, before D)
 *   dc_filter         R  -> H  = D( M c_geo (D R) )            (eqs. 7, 10, 11)
 *   dc_detector_bp    H  -> gF = A2d^T H                       (eq. 8 / 11, w_d folded)
 *   dc_cone_bp        gF -> f  = sum_v (D/U)^2 bilinear(gF_v)  (eq. 5 with w_d, ReLU)
 *
 * Discretisation (identical to the float64 reference it is tested against):
 *   detector pixel (i,j) at x_i = (i-(nu-1)/2) du, y_j = (j-(nv-1)/2) dv in the
 *   detector frame (origin at the detector centre, l_z = l_x x l_y towards the
 *   source, Fig. 1); Radon angles mu_k = k pi/n_theta (range pi, Table 2),
 *   bins s_m = (m-(n_s-1)/2) ds; A2d^T = pixel-driven linear interpolation of each
 *   sinogram row summed over mu with weight pi/n_theta; A2d = its transpose times
 *   du dv/ds; D = zero-padded central difference along s;
 *   c_geo = -|D t.n_mu + s t.l_z| / (4 pi^2 D^2) with t = a'(lambda) dlambda, the
 *   collapse of w_sino * w_red (eqs. 7, 10) for theta = (D n_mu + s l_z)/sqrt(s^2+D^2);
 *   the detector weight w_d = x^2+y^2+D^2 (eq. 11) and eq. 5's 1/|x-a|^2 combine at
 *   each voxel's exact projection into D^2/U^2, U = (a-x).l_z; bilinear
 *   interpolation with zero outside the detector.
 *
 * Layouts (contiguous, row-major, last index fastest):
 *   g, gF, Gg, GgF : [V][nv][nu]     R, H, M, GM, GR, GH : [V][n_theta][n_s]
 *   f, Gf          : [nz][ny][nx]    ([S][nz][ny][nx] for a plan of S samples)
 * Every stage call takes pointers to the FULL per-view arrays and processes the
 * view range [v0, v0+nv); volumes are shared by all views.
 *
 * Calling convention for every stage call: device pointers, enqueued on `stream`,
 * asynchronous, no allocation, no host synchronisation; base pointers 16-byte
 * aligned.  Errors are returned as dc_status before anything is enqueued (shape,
 * dtype, alignment, view range); dc_last_error() gives a thread-local message.
 * A fault inside a kernel surfaces at the caller's next synchronisation.
 * Ownership: the caller owns every array; the plan owns its small device
 * tables (immutable after creation), a scratch word per view and per sample that
 * dc_weight_radon, dc_detector_bp_adjoint and dc_cone_bp_adjoint use for their
 * fixed-point scales, and one volume-sized float32 buffer per sample into which
 * dc_cone_bp_adjoint rewrites the (ReLU-masked) gradient in z-bricks of 16
 * voxels (nz rounded up to a multiple of 16); stage calls on one plan
 * must therefore be ordered on one stream (use one plan per concurrent stream).  Plans must be created before any stream
 * capture that uses them; stage calls enqueue kernels only (no memset, no
 * allocation), so they can be captured into a graph.
 * Determinism: every stage returns bit-identical results for identical inputs
 * (the scattering stages accumulate in fixed point with integer atomics).
 */
#ifndef DCFBP_H
#define DCFBP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DC_OK = 0, DC_EINVAL = 1, DC_ESHAPE = 2, DC_EDTYPE = 3, DC_EALIGN = 4,
  DC_EHIP = 5, DC_ENOTSUP = 6, DC_ENOMEM = 7
} dc_status;

/* storage type of R, H, gF and their gradients; arithmetic is always float32 */
typedef enum { DC_F32 = 0, DC_BF16 = 1, DC_F16 = 2 } dc_dtype;

/* ANALYTIC: W = M * c_geo (M replaces 1/n, eq. 8/9);  RAW: W = M (the whole
 * redundancy weight of eq. 10 is the learned parameter, as the paper trains it) */
typedef enum { DC_WEIGHT_ANALYTIC = 0, DC_WEIGHT_RAW = 1 } dc_wmode;

typedef struct {
  int32_t nu, nv;          /* detector columns (along l_x) and rows (along l_y) */
  double  du, dv;          /* pixel pitch, mm */
  int32_t n_theta, n_s;    /* Radon grid: angles over [0, pi) and s bins */
  double  ds;              /* s bin width, mm */
  int32_t nx, ny, nz;      /* volume size */
  double  vx, vy, vz;      /* voxel size, mm */
  double  ox, oy, oz;      /* volume centre in world coordinates, mm */
} dc_grid;

/* One view (Fig. 1): source a, detector centre O, in-plane unit vectors l_x, l_y
 * (l_z = l_x x l_y points to the source; the source must lie on the detector
 * normal through O), and the orbit tangent already scaled by the view spacing,
 * t = a'(lambda) dlambda (mm).  All in world mm. */
typedef struct {
  double src[3], det_center[3], ex[3], ey[3], tangent[3];
} dc_view;

typedef struct dc_plan_s* dc_plan;

/* Host-only geometry check (no GPU needed): positive sizes and pitches,
 * orthonormal detector axes, source on the detector normal through its centre
 * (relative 1e-6), every voxel-box corner strictly in front of the source
 * (U > 0).  Returns DC_OK, DC_EINVAL or DC_ESHAPE. */
dc_status dc_validate(const dc_grid* grid, const dc_view* views, int32_t n_views);

/* Builds a plan on the current HIP device: copies grid and views, derives the
 * per-view projection tables in float64 and uploads them (small allocations made
 * here, never in a stage call).  flags must be 0.  *out is set only on DC_OK. */
dc_status dc_plan_create(const dc_grid* grid, const dc_view* views, int32_t n_views,
                         uint32_t flags, dc_plan* out);
/* Batched plan: n_samples scans that share one grid, each with its own orbit
 * (eq. 12 applied to every scan; the views of different scans never mix).  The
 * views of sample s are views[first_view[s] .. first_view[s+1]) (first_view has
 * n_samples + 1 entries, starts at 0, ends at n_views, strictly increasing).
 * Per-view arrays (g, R, M, H, gF and their gradients) hold all samples' views
 * back to back; volumes (f, Gf, f_relu) hold one [nz][ny][nx] block per sample,
 * in sample order, so every stage call serves all samples with one launch per
 * kernel (the cone stages too: over scans of different evaluation forms each
 * workgroup takes its scan's own form).  A view range [v0, v0+nv) may span samples: dc_cone_bp writes the
 * volumes of the samples it meets (for nv = 0, the sample holding view v0, the
 * last one when v0 = n_views) and leaves the others untouched; dc_cone_bp_adjoint
 * reads each view's own sample volume.  dc_plan_create is n_samples = 1. */
dc_status dc_plan_create_batched(const dc_grid* grid, const dc_view* views, int32_t n_views,
                                 const int32_t* first_view, int32_t n_samples, uint32_t flags,
                                 dc_plan* out);
dc_status dc_plan_destroy(dc_plan plan);

/* Work shapes of the kernels (the plan's knobs).  Every value gives the same
 * results up to float32 rounding: splat_angles, fp_tile_u (integer sums) and
 * interp_angles (the same sums in the same order) give bit-identical outputs;
 * interp_tile_u changes the float32 rounding of pixel positions, and bp_block_y
 * that of the cone BP only where one block's detector footprint is too large to
 * stage in LDS and its taps take the direct form.
 *   splat_angles   sinogram rows one weighted-Radon / detector-Radon workgroup holds
 *                  in LDS, 1..8 (0 on input: as many as fit 80 KiB);
 *   interp_tile_u  detector-BP pixel tile width, 32 or 64 (tile height 64);
 *   interp_angles  detector-BP angles staged per chunk, 16, 32 or 64;
 *   bp_block_y     cone-BP voxel block rows, 16 or 32 (block 16 x rows x 8);
 *   fp_tile_u      cone-FP detector tile width, 16, 20 or 24 (tile height 64).
 * A plan starts with 0 / 64 / 32 / 32 / 20, the values tuned by hand on the
 * 256^3 volume, 512^2 detector, 360 x 725 sinogram workload. */
typedef struct {
  int32_t splat_angles, interp_tile_u, interp_angles, bp_block_y, fp_tile_u;
} dc_knobs;
dc_status dc_plan_get_knobs(dc_plan plan, dc_knobs* out);
/* Re-derives the plan's tables for other knobs.  DC_EINVAL for a value the
 * kernels are not built for, DC_ENOTSUP when the geometry does not fit it (LDS);
 * the plan is unchanged on failure.  Allocates, and synchronises the device before
 * releasing the old tables: call it, like dc_plan_create, outside stream capture
 * and with no stage call on this plan in flight on another thread. */
dc_status dc_plan_set_knobs(dc_plan plan, const dc_knobs* knobs);
/* The autotuner: times every candidate value of each knob on the plan's own
 * geometry and sets the fastest.  Each stage is timed (on `stream`, one warm-up and
 * three timed runs, the fastest kept) over up to four runs of 32 consecutive views
 * spread over the plan; the knobs held so far are timed first and a candidate
 * replaces them only if it is more than 2% faster.  Inputs are seeded synthetic
 * ones in temporary device buffers
 * allocated and freed inside the call: dc_weight_radon for splat_angles,
 * dc_detector_bp for interp_tile_u x interp_angles, dc_cone_bp for bp_block_y and
 * dc_cone_bp_adjoint (with a ReLU mask) for fp_tile_u.
 *   - DCFBP_KNOBS (environment), e.g. "splat=7,itile=64,iangles=32,bprows=32,fptile=20":
 *     these knobs are set without timing (unnamed ones keep their current value);
 *   - DCFBP_TUNE_CACHE (environment): a text file of earlier results, one line per
 *     geometry key (a 64-bit hash of the grid, every view, the scan split, the GPU's
 *     architecture name and compute-unit count); a hit sets the cached knobs without
 *     timing, a miss tunes and appends a line.
 * *chosen (nullable) receives the knobs set; ms (nullable, 4 doubles) the chosen
 * knobs' measured times of the four stages over the sampled views (0 when not
 * timed).  *source (nullable) is set to 0 (timed), 1 (cache) or 2 (environment).
 * Synchronises the device; call it outside stream capture.  flags must be 0. */
dc_status dc_plan_autotune(dc_plan plan, uint32_t flags, hipStream_t stream, dc_knobs* chosen, double* ms,
                           int32_t* source);

/* The bounds and kernel forms a plan over these views would use, computed on the
 * host only (no device, no allocation): the same float64 derivation as
 * dc_plan_create, for a one-scan plan.  They decide the safety and accuracy of
 * the fixed-point stages (dc_weight_radon and dc_detector_bp_adjoint accumulate
 * pixel terms per (angle, bin); dc_cone_bp_adjoint voxel terms per detector cell):
 * each term is rounded to an integer number of units, the largest term of a view
 * (splat: max |w_cos g| or |GgF| over the view's pixels) or of the call (cone FP:
 * max |Gf| times the view's bound on (D/U)^2) taking qmax units, and a sum of at
 * most max_terms such integers never leaves 32 bits.  So every output's absolute
 * error is at most (number of terms it sums) x 1/2 unit, relative to that
 * largest term: the stages are exact transposes up to this rounding, which is
 * small against large outputs but not against outputs far below the largest
 * term.  Returns DC_OK, or the dc_validate / dc_plan_create status and message. */
typedef struct {
  int32_t splat_angles;      /* sinogram rows one splat workgroup holds in LDS */
  int32_t splat_max_terms;   /* bound on the pixels whose bin floor(t) is one bin, on one angle */
  int32_t splat_checked;     /* 1 if a pixel may fall outside bins [-1, n_s): the range-checked splat */
  int32_t interp_window;     /* detector-BP window: sinogram intervals staged per angle and pixel tile */
  int32_t interp_local;      /* 1 if that window takes the fixed-point position tap form (wide windows) */
  int32_t cone_max_terms;    /* bound on the voxel centres projecting into one detector cell of one view */
  int32_t bp_stage;          /* footprint rows each cone-BP thread stages per view (0: taps from memory) */
  int32_t cone_form;         /* 0: reciprocal per voxel, 1: 1/U quadratic in z, 2: z-invariant columns */
  int32_t bp_block[3];       /* cone-BP voxel block (x, y, z) */
  int32_t interp_tile[2];    /* detector-BP pixel tile (u, v) */
  float   splat_qmax;        /* units of the largest splat term */
  float   cone_qmax;         /* units of the largest cone-FP term */
  int32_t bp_pitch;          /* pixels between the cone BP's staged footprint rows: 64 or 128 (0: taps from memory) */
} dc_bounds;
dc_status dc_plan_bounds(const dc_grid* grid, const dc_view* views, int32_t n_views, dc_bounds* out);
/* Thread-local text of the last error (empty string if none). */
const char* dc_last_error(void);
/* Size queries used by bindings: views, samples, and the grid the plan was built with. */
int32_t dc_plan_n_views(dc_plan plan);
int32_t dc_plan_n_samples(dc_plan plan);
dc_status dc_plan_grid(dc_plan plan, dc_grid* out);

/* Stage 1, eq. 7 (integrate first): R[v] = (du dv/ds) sum_p w_cos(p) g[v](p) Lambda((s_p,k - s_m)/ds),
 * w_cos = D/sqrt(x^2+y^2+D^2).  g float32; R stored as tR. */
dc_status dc_weight_radon(dc_plan plan, const float* g, void* R, dc_dtype tR,
                          int32_t v0, int32_t nv, hipStream_t stream);
/* dc_weight_radon for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): the same stage, bit for bit,
 * with its per-view fixed-point scale words in a static device array of 65536
 * words (256 KiB) that each GPU holds until the process ends, instead of the
 * plan's scratch.  Nothing is allocated in the call.  At most 65536 views per
 * call (DC_ESHAPE beyond).  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other plans, other
 * threads) race and must be ordered by the caller.  The array is cleared by a
 * kernel at the start of each call. */
dc_status dc_weight_radon_noalloc(dc_plan plan, const float* g, void* R, dc_dtype tR,
                                  int32_t v0, int32_t nv, hipStream_t stream);
/* Exact transpose of dc_weight_radon: Gg[v] = w_cos (du dv/ds) interp(GR[v]).  Gg float32, overwritten. */
dc_status dc_weight_radon_adjoint(dc_plan plan, const void* GR, dc_dtype tR, float* Gg,
                                  int32_t v0, int32_t nv, hipStream_t stream);

/* Stage 2, eqs. 7, 10, 11: Q = D R, P = W Q, H = D P, W per mode (see dc_wmode). M float32. */
dc_status dc_filter(dc_plan plan, const void* R, dc_dtype tR, const float* M, dc_wmode mode,
                    void* H, dc_dtype tH, int32_t v0, int32_t nv, hipStream_t stream);
/* Transpose of dc_filter w.r.t. R and gradient w.r.t. M given GH = dL/dH:
 *   GP = D^T GH (= -D GH),  GM (+)= GP * (D R) * c_geo   (c_geo = 1 in RAW mode),
 *   GR = D^T (W * GP).
 * GM (float32) and GR (float32) may each be NULL to skip; accumulate_GM != 0 adds into GM. */
dc_status dc_filter_adjoint(dc_plan plan, const void* GH, dc_dtype tH, const void* R, dc_dtype tR,
                            const float* M, dc_wmode mode, float* GM, int32_t accumulate_GM,
                            float* GR, int32_t v0, int32_t nv, hipStream_t stream);

/* Stage 3, eq. 8 / 11: gF[v](i,j) = (pi/n_theta) sum_k lerp(H[v][k], s = x_i cos mu_k + y_j sin mu_k). */
dc_status dc_detector_bp(dc_plan plan, const void* H, dc_dtype tH, void* gF, dc_dtype tF,
                         int32_t v0, int32_t nv, hipStream_t stream);
/* Exact transpose of dc_detector_bp (the detector Radon): GH[v] = (pi/n_theta) splat(GgF[v]). */
dc_status dc_detector_bp_adjoint(dc_plan plan, const void* GgF, dc_dtype tF, void* GH, dc_dtype tH,
                                 int32_t v0, int32_t nv, hipStream_t stream);

/* Stage 4, eq. 5 with w_d folded: f(x) (+)= sum_{v in range} (D/U)^2 bilinear(gF[v], proj_v(x)).
 * accumulate != 0 adds to f; relu != 0 applies max(., 0) to the result (set it
 * only on the call that completes the view sum, paper Sec. 2.4).
 * The plan evaluates each sample's projections (here and in dc_cone_bp_adjoint)
 * in one of three forms chosen from its geometry: per voxel column when no view's
 * depth U or detector u coordinate varies along z (detector v axis along z); with
 * 1/U taken along z as its quadratic Taylor polynomial about a segment's middle
 * when U changes by at most 5e-4 of itself per voxel step; with a
 * reciprocal per voxel otherwise.  The forms agree to float32 rounding, and each
 * is deterministic. */
dc_status dc_cone_bp(dc_plan plan, const void* gF, dc_dtype tF, float* f, int32_t accumulate,
                     int32_t relu, int32_t v0, int32_t nv, hipStream_t stream);
/* Exact transpose of dc_cone_bp (cone-beam forward projection of Gf):
 * GgF[v](p) = sum_x (D/U)^2 Gf'(x) bilinear-weight(x -> p), Gf' = Gf * [f_relu > 0]
 * when f_relu (the ReLU output of the forward) is non-NULL, else Gf.  GgF overwritten. */
dc_status dc_cone_bp_adjoint(dc_plan plan, const float* Gf, const float* f_relu, void* GgF,
                             dc_dtype tF, int32_t v0, int32_t nv, hipStream_t stream);

/* The Gaussian filter layer after the weight layer (Sec. 3.1; the paper uses
 * sigma = 20, 121 taps): Ms = G_mu G_s M per view, the separable 2D Gaussian over
 * the (mu, s) grid with taps exp(-t^2 / (2 sigma^2)) normalised over
 * t = -radius..radius and mirror padding (the edge sample is not repeated) along
 * both axes; views are not mixed.  M, Ms float32 [V][n_theta][n_s]; Ms may alias M.
 * Needs sigma > 0, 1 <= radius <= 255, radius < n_theta and radius < n_s
 * (DC_EINVAL / DC_ESHAPE otherwise), and radius + 1 + 16 (n_theta + 2 radius + 4)
 * <= 40960 (one workgroup's 160 KiB of LDS; e.g. n_theta <= 2432 at radius 60;
 * DC_ENOTSUP otherwise). */
dc_status dc_smooth_weights(dc_plan plan, const float* M, float* Ms, double sigma, int32_t radius,
                            int32_t v0, int32_t nv, hipStream_t stream);
/* Exact transpose of dc_smooth_weights: GM = G_s^T G_mu^T GMs (the backward of the
 * layer).  GM float32, overwritten; GM may alias GMs.  Same limits. */
dc_status dc_smooth_weights_adjoint(dc_plan plan, const float* GMs, float* GM, double sigma, int32_t radius,
                                    int32_t v0, int32_t nv, hipStream_t stream);

/* Projection data from a voxel volume (the paper trains on simulated projections,
 * Sec. 3.3): g[v](i,j) = Siddon's exact line integral of the piecewise-constant
 * volume f (value f[z][y][x] on voxel [x-1/2, x+1/2] vx ... around each centre)
 * along the segment from the source of view v to the centre of pixel (i, j).
 * vol float32 [nz][ny][nx] ([S][nz][ny][nx] for a batched plan: each view reads its
 * own sample's volume); g float32 [V][nv][nu], views [v0, v0+nv) overwritten. */
dc_status dc_project(dc_plan plan, const float* vol, float* g, int32_t v0, int32_t nv, hipStream_t stream);

/* One analytic piece of a source orbit of radius sid around the origin, for the
 * Crofton weight.  Views [start, start + count) of the plan sample it at
 * parameters tau_k = p0 + k p1:
 *   DC_SEG_CIRCLE   a = sid (cos tau, sin tau, 0)            p0 = lambda_0, p1 = dlambda
 *   DC_SEG_ARC      a = sid (cos tau, 0, sin tau)            p0 = phi_0, p1 = dphi
 *   DC_SEG_LINE     a = (sid, 0, tau)                        p0 = z_0, p1 = dz
 *   DC_SEG_SINUSOID a = sid (cos phi cos tau, cos phi sin tau, sin phi),
 *                   phi = phi_max cos(freq tau), tau over one turn   p0 = theta_0, p1 = dtheta
 * closed = 1 for a curve that closes on itself (no end taper).  A sinusoid must
 * be closed, and a closed circle or sinusoid must span one turn (count p1 = 2 pi). */
typedef enum { DC_SEG_CIRCLE = 1, DC_SEG_ARC = 2, DC_SEG_LINE = 3, DC_SEG_SINUSOID = 4 } dc_seg_kind;
typedef struct {
  int32_t kind, start, count, closed;
  double p0, p1, phi_max, freq;
} dc_orbit_segment;

/* The smooth Crofton redundancy weight of eq. 9 (Defrise & Clack's smooth
 * replacement of 1/n, Sec. 2.4) on the plan's Radon grid:
 *   M[v][k][m] = |a'(tau_v) . theta|^m_exp c(tau_v) / sum_alpha |a'(tau_alpha) . theta|^m_exp c(tau_alpha),
 *   theta = (D n_mu_k + s_m l_z) / sqrt(s_m^2 + D^2),
 * the sum running over every orbit parameter tau_alpha whose source point lies in
 * the plane through a(tau_v) with normal theta.  a' is the tangent per view step
 * (p1 a'(tau)); c = 1 on closed segments, and on open ones a raised-cosine ramp
 * over the fraction `taper` of the parameter range at each end, floored at
 * c_floor.  Where the sum is at most 1e-18 |a'(tau_v)|^m_exp (a plane tangent to
 * the orbit wherever it meets it), M = 1 / max(1, number of crossings).
 * Crossings are solved in closed form on circles, arcs and lines.  On a sinusoid
 * the plane function is sampled at fine * count points tau_j = p0 + (j + 1/2) 2 pi / (fine count),
 * every sign change (a zero sample counts on both sides, and the interval
 * across the end of the turn) is refined by 80 bisection steps, and the
 * crossing is the midpoint of the final interval.
 * segs (host) partition the plan's views in order; one scan per plan
 * (n_samples = 1, else DC_ENOTSUP); at most 16 segments; m_exp >= 1,
 * 0 < taper <= 0.5, 0 < c_floor <= 1, fine >= 1 (DC_EINVAL otherwise).
 * M float32 [V][n_theta][n_s], views [v0, v0+nv) overwritten.  work: device
 * buffer of dc_crofton_workspace_bytes() bytes owned by the caller (the sampled
 * sinusoid points). */
size_t dc_crofton_workspace_bytes(const dc_orbit_segment* segs, int32_t n_segs, int32_t fine);
dc_status dc_crofton_weights(dc_plan plan, const dc_orbit_segment* segs, int32_t n_segs, double sid, int32_t m_exp,
                             double taper, double c_floor, int32_t fine, float* M, int32_t v0, int32_t nv,
                             void* work, size_t work_bytes, hipStream_t stream);

/* Poisson noise on projection data (the simulated data of Sec. 3.3): for each
 * element q of the line integrals p, lambda = photons exp(-mu p[q]) expected
 * photons, a count N ~ Poisson(lambda), and out[q] = -ln(max(N, 1) / photons) / mu.
 * The random numbers are those of the counter-based generator Philox4x64-10
 * (Salmon et al., SC 2011) keyed (seed, 0): element e = e0 + q draws the blocks of
 * counter (e, j, 0, 0), j = 0, 1, ..., each 64-bit word x giving the uniform
 * ((x >> 11) + 1/2) 2^-53.  N is drawn by inversion for lambda < 10 and by
 * Hoermann's transformed rejection (PTRS, 1993) otherwise, every decision in
 * float64; results depend only on (seed, e, p[q], photons, mu), not on the launch.
 * p, out float32 [n] (out may alias p); counts (nullable) int64 [n] receives N.
 * Needs 0 < photons <= 1e12 and mu > 0 (DC_EINVAL).  Not tied to a plan. */
dc_status dc_poisson_noise(const float* p, float* out, int64_t* counts, size_t n, double photons, double mu,
                           uint64_t seed, uint64_t e0, hipStream_t stream);

/* One Adam step (AdamW when weight_decay > 0) of a float32 parameter array: the
 * paper trains the weight M with AdamW (Sec. 3.1).  In one pass,
 *   M <- M (1 - lr weight_decay);  m <- b1 m + (1 - b1) G;  v <- b2 v + (1 - b2) G^2;
 *   M <- M - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * with t = *step, a float32 on the device (>= 1) that the caller advances before
 * the call, so the update can be captured in a graph.  M, m, v [n] updated in
 * place, G [n] read; all float32, 16-byte aligned.  The hyperparameters are float64: 1 - b and
 * the bias corrections are formed in float64 before rounding.  Needs 0 <= b1, b2 < 1,
 * eps > 0, finite lr and weight_decay >= 0 (DC_EINVAL).  Not tied to a plan. */
dc_status dc_adam_step(float* M, const float* G, float* m, float* v, size_t n, const float* step, double lr,
                       double b1, double b2, double eps, double weight_decay, hipStream_t stream);

/* The structural term of the training loss (eq. 13), read as the standard 3D SSIM:
 * Gaussian window of standard deviation 1.5 and 11 taps per axis, C1 = (0.01 L)^2,
 * C2 = (0.03 L)^2 with L = data_range, mean over the positions where the whole
 * window lies inside the volume.  x, y float32 [nz][ny][nx], every side >= 11.
 * *ssim (one float on the device) receives the mean; grad_x (nullable) receives
 * d SSIM / d x, overwritten.  work: device buffer of at least
 * dc_ssim_workspace_bytes(nz, ny, nx) bytes owned by the caller; the mean is
 * reduced in a fixed order, so results are bit-reproducible.  Not tied to a plan. */
size_t dc_ssim_workspace_bytes(int32_t nz, int32_t ny, int32_t nx);
dc_status dc_ssim(const float* x, const float* y, int32_t nz, int32_t ny, int32_t nx, float data_range,
                  float* ssim, float* grad_x, void* work, size_t work_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DCFBP_H */
