/*
 * dgr.h -- C ABI of libdgr.so, the MI355X (gfx950) hot path of Discretized
 * Gaussian Representation (DGR) CT reconstruction (Wu et al., arXiv
 * 2411.04844).
 *
 * The library turns a set of 3-D Gaussians into a voxel volume (sec. 4.1-4.2,
 * Fast Volume Reconstruction, Alg. 1), projects the volume along X-ray paths
 * (sec. 4.3, P_hat = T(V); sec. 3, y = Ax), and provides the exact adjoints of
 * both, so that a projection-domain loss can be differentiated with respect to
 * every Gaussian parameter.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Memory: every array argument is a DEVICE pointer (HIP), contiguous and
 *   row-major, binary32 unless stated.  The caller allocates and owns every
 *   buffer, including the workspace `ws`; the library keeps no device state
 *   between calls and never allocates device memory.  The one exception is
 *   dgr_voxelize_backward_noalloc, whose records live in a fixed 32 MiB
 *   device array that each GPU it runs on holds until the process ends.
 * - Streams: `stream` is a hipStream_t (NULL = the default stream).  Every call
 *   only enqueues work and returns, except those that hand results to the
 *   host and therefore synchronise `stream`: dgr_voxelize_plan, dgr_densify,
 *   dgr_fd_l1_f64 and dgr_check.
 * - Workspaces are 256-byte aligned.  The workspace of the voxelization calls
 *   (dgr_voxelize_plan, dgr_voxelize, dgr_voxelize_f64, dgr_bin) carries a
 *   pair-overflow flag from one call to the next: zero-fill it once before its
 *   first use.  Other workspaces need no initial contents.
 * - Outputs are overwritten, never accumulated into.
 * - Errors: argument checks happen on the host before anything is enqueued;
 *   on failure nothing is launched and a status other than DGR_OK is
 *   returned.  dgr_last_error() gives a thread-local description.  No call
 *   aborts or throws.  A pair-capacity overflow found on the device is
 *   recorded in the workspace; the affected volume is filled with NaN and
 *   dgr_check() (or the next dgr_voxelize_plan) reports DGR_ERR_CAPACITY.
 * - Calls that share a workspace must not overlap; distinct workspaces may
 *   be used concurrently on different streams.
 *
 * Coordinates
 * -----------
 * World points are (x, y, z).  A grid of dims (nx, ny, nz) has its lower faces
 * at lo[] and voxel size 1/inv_h[a] on axis a; voxel (i, j, k) has its centre
 * at lo + (idx + 1/2)/inv_h and is stored at [k][j][i] (x fastest).  The
 * continuous voxel coordinate of a point p is u = (p - lo)*inv_h - 1/2, so
 * voxel centres sit at integers (the integer grid of the paper's Discretize
 * and Align step, sec. 4.1).
 */
#ifndef DGR_H
#define DGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DGR_OK = 0,
    DGR_ERR_INVALID_ARG = 1, /* null pointer, bad size or unsupported shape       */
    DGR_ERR_WORKSPACE = 2,   /* workspace too small or not 256-byte aligned        */
    DGR_ERR_CAPACITY = 3,    /* more (tile, Gaussian) pairs than the workspace holds */
    DGR_ERR_HIP = 4          /* a HIP runtime call failed; see dgr_last_error()    */
} dgr_status;

/* Voxel grid.  dims[a] in [1, 16384]; inv_h[a] > 0. */
typedef struct {
    int32_t dims[3];
    float lo[3];
    float inv_h[3];
} dgr_grid;

/* Truncation of each Gaussian to an axis-aligned box of voxel centres
 * (sec. 4.1, Gaussian Effect Confinement; Alg. 1 validity mask).
 * k_sigma > 0: per-Gaussian box |i_a - u_a| <= k_sigma*sqrt(Sigma_aa)*inv_h_a.
 * k_sigma <= 0: the paper's fixed cuboid floor(u) +- box_half on every axis.
 * The box is clamped to the grid.  Its integer bounds are defined by one
 * binary32 sequence (every operation correctly rounded, no fused
 * multiply-add, in this order):
 *   n2 = ((w*w + x*x) + y*y) + z*z;  m = sqrt(n2);  q_hat = q/m  (n2 = 0: R = I)
 *   R = rotation of q_hat (row a = image components), a_j = R[a][j]*s_j,
 *   S_aa = (a_0*a_0 + a_1*a_1) + a_2*a_2,  r = (k_sigma*sqrt(S_aa))*inv_h_a,
 *   u = (mu_a - lo_a)*inv_h_a - 0.5,  lo = ceil(u - r),  hi = floor(u + r),
 *   then lo clamped to [0, dims], hi to [-1, dims-1]; empty iff lo > hi.    */
typedef struct {
    float k_sigma;
    int32_t box_half;
} dgr_trunc;

#define DGR_PARALLEL 0
#define DGR_CONE 1
#define DGR_FAN 2

/* Acquisition geometry.  The paper leaves the projection T abstract
 * (sec. 4.3); the operator here is the trilinear ray march
 *   P_hat[r] = length_scale * step * sum_{k in Z} Vbar(c_r + k*step*d_r),
 * with d_r the unit ray direction, c_r the point of the ray nearest the world
 * origin and Vbar the trilinear interpolant of the volume on voxel centres,
 * zero outside the grid.
 * views: DEVICE pointer, binary32 [n_views][12] =
 *   { a[3], det[3], e_u[3], e_v[3] }  (world units)
 * a is the ray direction (DGR_PARALLEL), the source position (DGR_CONE) or
 * the source position of the central row (DGR_FAN: row iv has its own
 * source a + (iv-(nv-1)/2)*e_v, so each detector row is a 2-D fan beam in
 * its own plane -- a stack of fan-beam slices, the geometry of the paper's
 * fan-beam sparse-view and limited-angle experiments, sec. 5.1, Tabs. 2-3);
 * detector pixel (iu, iv) is centred at det + (iu-(nu-1)/2)*e_u +
 * (iv-(nv-1)/2)*e_v.  Projections are stored [n_views][nv][nu].
 * DGR_FAN is meant for e_v orthogonal to e_u and to det - a (each row's fan
 * then lies in a plane orthogonal to e_v); the operator is defined for any
 * vectors, and views that break this are handled exactly but without the
 * detector-footprint culling, so they run slower.                         */
typedef struct {
    int32_t kind;
    int32_t n_views, nu, nv;
    const float *views;
    float step;         /* march step, world units, > 0        */
    float length_scale; /* multiplies every line integral      */
} dgr_geometry;

/* ---- voxelization (sec. 4.2 Fast Volume Reconstruction, Alg. 1) -------- */

/* Bytes of workspace that dgr_voxelize / dgr_voxelize_plan / dgr_bin need for
 * n Gaussians and up to max_pairs (8^3 tile, Gaussian) pairs.  0 on bad
 * arguments. */
size_t dgr_voxelize_workspace(int64_t n, int64_t max_pairs, const dgr_grid *grid);

/* Counts the (tile, Gaussian) pairs of the truncation boxes and returns the
 * count in *n_pairs_host.  Synchronises `stream`.  Also reports an overflow
 * left in `ws` by an earlier dgr_voxelize (DGR_ERR_CAPACITY, after writing
 * the new count).  ws must hold dgr_voxelize_workspace(n, 0, grid) bytes. */
dgr_status dgr_voxelize_plan(const float *mu, const float *scale, const float *quat, int64_t n,
                             const dgr_grid *grid, const dgr_trunc *trunc, int64_t *n_pairs_host,
                             void *ws, size_t ws_bytes, void *stream);

/* V(p) = sum_g density_g * exp(-1/2 (p-mu_g)^T Sigma_g^-1 (p-mu_g)) over the
 * voxel centres p inside each Gaussian's box (sec. 4.1 eq. for V(p); Alg. 1).
 * mu [n][3], scale [n][3] (> 0, world units), quat [n][4] (w, x, y, z, any
 * norm; zero = identity), density [n]; Sigma = R diag(scale^2) R^T.
 * volume [nz][ny][nx] is overwritten.  Contributions to each voxel are added
 * in ascending Gaussian index, so results are run-to-run deterministic.
 * The pair capacity is whatever ws holds beyond dgr_voxelize_workspace(n,0). */
dgr_status dgr_voxelize(const float *mu, const float *scale, const float *quat,
                        const float *density, int64_t n, const dgr_grid *grid,
                        const dgr_trunc *trunc, float *volume, void *ws, size_t ws_bytes,
                        void *stream);

/* Gradient of a scalar loss with respect to the Gaussian parameters, given
 * dL/dV (dvolume, [nz][ny][nx]); boxes are held fixed (the box edges are not
 * differentiated).  Outputs dmu [n][3], dscale [n][3], dquat [n][4],
 * ddensity [n] are overwritten.  ws >= dgr_voxelize_backward_workspace(n). */
size_t dgr_voxelize_backward_workspace(int64_t n);
dgr_status dgr_voxelize_backward(const float *mu, const float *scale, const float *quat,
                                 const float *density, int64_t n, const dgr_grid *grid,
                                 const dgr_trunc *trunc, const float *dvolume, float *dmu,
                                 float *dscale, float *dquat, float *ddensity, void *ws,
                                 size_t ws_bytes, void *stream);

/* dgr_voxelize_backward without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, kernels and results as
 * dgr_voxelize_backward (bit for bit); the 64-byte per-Gaussian records go to
 * a fixed device array of dgr_voxelize_backward_noalloc_max() = 524,288
 * Gaussians (above the 500K cap of the density control, Alg. 2), 32 MiB per
 * GPU, kept until the process ends.  Nothing in it needs initial contents: a
 * call overwrites the first n records before reading them.  n beyond the
 * maximum returns DGR_ERR_INVALID_ARG and launches nothing.  The call itself
 * allocates nothing; its first call on a device looks up that device's array
 * address (the device current at the call must be the stream's).  Every call on
 * one GPU shares the array: calls that overlap in time on one GPU (different
 * streams, or host threads) race and give wrong gradients. */
int64_t dgr_voxelize_backward_noalloc_max(void);
dgr_status dgr_voxelize_backward_noalloc(const float *mu, const float *scale, const float *quat,
                                         const float *density, int64_t n, const dgr_grid *grid,
                                         const dgr_trunc *trunc, const float *dvolume, float *dmu,
                                         float *dscale, float *dquat, float *ddensity, void *stream);

/* ---- projection (sec. 4.3, P_hat = T(V)) and its adjoint --------------- */

/* Bytes of workspace that dgr_project / dgr_project_l1 / dgr_backproject need. */
size_t dgr_project_workspace(const dgr_grid *grid, const dgr_geometry *geom);

/* proj [n_views][nv][nu] = T(volume). */
dgr_status dgr_project(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                       float *proj, void *ws, size_t ws_bytes, void *stream);

/* Fused projection and L1 data term (sec. 4.3 objective, L1 part):
 * *loss (device scalar) = mean_r |P_hat_r - target_r| and
 * dproj_r = sign(P_hat_r - target_r)/M, sign(0) = 0, M = n_views*nu*nv.
 * P_hat itself is not stored.  The loss is summed in a fixed order. */
dgr_status dgr_project_l1(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                          const float *target, float *loss, float *dproj, void *ws,
                          size_t ws_bytes, void *stream);

/* volume [nz][ny][nx] = T^T(proj): the exact transpose of dgr_project.
 * Deterministic: the per-voxel sums are 64-bit fixed-point integers, so they
 * do not depend on the order of the adds.  The fixed-point unit follows
 * max|proj| and the geometry: where a per-view bound on the weight one voxel
 * can receive (computed on the device from the view vectors) allows it, two
 * voxels share one 64-bit LDS word as 32-bit halves and each sum of one
 * ray's samples in one cell is rounded to the nearest unit, at most 2^-21
 * of max|proj| length_scale step (2^-22.5 for the 256^3 / 512^2 cone scan);
 * otherwise one voxel per word with a power-of-two unit of about 2^-27 of
 * it, truncated.  The march step, in voxels of every axis, must lie between
 * 0.12 and 3.9 (at most 256 samples of one ray in a brick of 20 x 20 x 6
 * voxels, advances below 4 voxels); DGR_ERR_INVALID_ARG otherwise. */
/* bound[n_views] (DEVICE, binary32): for each view, the bound that
 * dgr_backproject uses for the weight one voxel can receive from that view's
 * rays (the rays through the eight cells around the voxel times the largest
 * weight sum one ray can give it, rounded up), in units of one projection
 * value times length_scale * step; 3e38 where no bound is found.  The
 * largest over the views picks the fixed-point tile (packed when at most
 * 512).  Asynchronous; for inspection and tests. */
dgr_status dgr_backproject_weight_bound(const dgr_grid *grid, const dgr_geometry *geom, float *bound,
                                        void *stream);

dgr_status dgr_backproject(const float *proj, const dgr_grid *grid, const dgr_geometry *geom,
                           float *volume, void *ws, size_t ws_bytes, void *stream);

/* ---- exact-path projection (Siddon) and its transpose ------------------- */

/* proj[r] = length_scale * sum over voxels of |ray_r inside voxel| * volume,
 * the voxels being constant-valued cells [lo + i h, lo + (i+1) h] (an
 * alternative to the trilinear march for the abstract projector T of
 * sec. 4.3; Siddon's exact radiological path).  The rays are the same lines
 * as in dgr_project (any geometry kind; geom->step is not used).  Each ray
 * is walked in binary64 and each segment between consecutive cell-plane
 * crossings goes to the cell holding its midpoint.  proj [n_views][nv][nu]
 * is overwritten.  No workspace. */
dgr_status dgr_project_siddon(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                              float *proj, void *stream);

/* volume = transpose of dgr_project_siddon applied to proj, summed in a
 * binary64 workspace with hardware binary64 atomics (the order of the adds
 * varies, at the 1e-16 level) and rounded to binary32.  ws >=
 * dgr_backproject_siddon_workspace(grid) bytes (8 per voxel), 256-byte
 * aligned. */
size_t dgr_backproject_siddon_workspace(const dgr_grid *grid);
dgr_status dgr_backproject_siddon(const float *proj, const dgr_grid *grid, const dgr_geometry *geom,
                                  float *volume, void *ws, size_t ws_bytes, void *stream);

/* ---- optimiser (sec. 5.1 Implementation Details: Adam) ------------------ */

/* One Adam step in place over n entries, projected onto param >= lower:
 * m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * param = max(param - lr * (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps), lower);
 * step >= 1; lower = -INFINITY for a plain step. */
dgr_status dgr_adam(float *param, const float *grad, float *m, float *v, int64_t n, float lr,
                    float b1, float b2, float eps, int64_t step, float lower, void *stream);

/* ---- reconstruction support: FDK, initialisation, PSNR -------------------- */

/* FDK reconstruction (Feldkamp; the paper initialises Gaussian positions from
 * an FBP/FDK volume, Fig. 4 caption, and uses FDK as a baseline, Tab. 1) of a
 * full circular cone-beam scan on a flat detector covering `arc` radians in
 * n_views equal steps (arc = 2*pi): cosine weighting, Ram-Lak ramp filter
 * along detector rows (spacing |e_u| R/D at the isocentre), and voxel-driven
 * backprojection with weight (dbeta/2)(R/U)^2, divided by length_scale.
 * With a DGR_FAN geometry the same steps use each row's own source, which
 * makes it slice-by-slice fan-beam FBP: the cosine weight sees only the
 * in-row offset, and a voxel is read from the row whose fan plane holds it,
 * row position ((x - a).m)/(e_v.m) with m = (det - a) x e_u (e_v must not
 * lie in the fan plane), linear between rows.  proj [n_views][nv][nu] -> volume [nz][ny][nx] (overwritten).  geom
 * must be DGR_CONE or DGR_FAN with nu <= 8192 (a filtered row is staged in
 * LDS in binary64).  Returns DGR_ERR_INVALID_ARG otherwise; all pointers are
 * DEVICE pointers. */
size_t dgr_fdk_workspace(const dgr_grid *grid, const dgr_geometry *geom);
dgr_status dgr_fdk(const float *proj, const dgr_grid *grid, const dgr_geometry *geom, float arc,
                   float *volume, void *ws, size_t ws_bytes, void *stream);

/* Bytes of workspace for dgr_psnr and dgr_fit_density_scale. */
size_t dgr_reduce_workspace(void);

/* PSNR of x against ground truth gt (App. C.1): out (DEVICE binary64 [3]) =
 * { 10 log10(MAX^2 / MSE), MSE, MAX } with MAX = max(gt), MSE over n. */
dgr_status dgr_psnr(const float *x, const float *gt, int64_t n, double *out, void *ws,
                    size_t ws_bytes, void *stream);

/* Initial Gaussians drawn from a volume (e.g. the FDK volume): voxels above
 * thresh_frac * max(volume) are drawn with probability proportional to their
 * value, with replacement; sample i takes the voxel whose cumulative-weight
 * interval (x fastest) holds uniforms[i][0] * W, mean = voxel centre +
 * (uniforms[i][1..3] - 1/2) voxel, isotropic scale `scale`, identity
 * rotation, density = volume value.  uniforms [n][4] in [0, 1) (DEVICE). */
size_t dgr_init_workspace(const dgr_grid *grid);
dgr_status dgr_init_from_volume(const float *volume, const dgr_grid *grid, float thresh_frac,
                                int64_t n, const float *uniforms, float scale, float *mu,
                                float *scale_out, float *quat, float *density, void *ws,
                                size_t ws_bytes, void *stream);

/* Least-squares intensity scale: kappa = <p1, target> / <p1, p1> over m
 * entries (binary64 sums); density[n] *= kappa; *kappa (DEVICE binary64, may
 * be null) receives kappa. */
dgr_status dgr_fit_density_scale(const float *p1, const float *target, int64_t m, float *density,
                                 int64_t n, double *kappa, void *ws, size_t ws_bytes, void *stream);

/* ---- adaptive density control (Alg. 2) ------------------------------------- */
/* A Gaussian set with its Adam moments (DEVICE, binary32): mu/scale [n][3],
 * quat [n][4], density [n]; m_* and v_* the first and second moments. */
typedef struct dgr_gaussians {
    float *mu, *scale, *quat, *density;
    float *m_mu, *m_scale, *m_quat, *m_density;
    float *v_mu, *v_scale, *v_quat, *v_density;
} dgr_gaussians;

/* Thresholds: iters = iterations accumulated in acc; tau = minimum averaged
 * position gradient to clone or split; tau_prune = near-zero gradient that
 * prunes; theta = scale separating clone (<=) from split (>) (the paper:
 * 0.005 of the body diagonal); size_vox = box edge in voxels (prune when the
 * largest scale exceeds 3 x size voxels); n_max = cap on the set's size. */
typedef struct dgr_densify_params {
    int32_t iters;
    float tau, tau_prune, theta, size_vox;
    int64_t n_max;
} dgr_densify_params;

/* acc[g] += ||dmu[g]||_2 (dmu [n][3]), after each iteration's backward. */
dgr_status dgr_accumulate_grad_norm(const float *dmu, int64_t n, float *acc, void *stream);

/* One pass of Alg. 2 from src (n Gaussians) into dst (capacity >= n_max; the
 * arrays of src and dst must not overlap).  avg = acc / iters (binary32);
 * sigma = largest scale.  Clone: avg >= tau, sigma <= theta; split: avg >=
 * tau, sigma > theta; each limited to the room left under n_max, largest avg
 * first (ties: lower index), clones before splits.  A clone and its original
 * carry half the density (the copy's moments start at zero); a split
 * Gaussian is replaced by two with means mu + R diag(s) z_k (normals
 * [n][2][3], standard normal draws supplied by the caller), scales s/2^(1/3),
 * zero moments.  Other Gaussians are pruned if avg <= tau_prune, density <= 0
 * or sigma > 3 size_vox / min(inv_h).  dst holds the survivors in index order
 * (0, 1 or 2 entries per source Gaussian).  Synchronising: *n_out (HOST) is
 * the new count, counts (HOST) = {cloned, split, pruned}. */
size_t dgr_densify_workspace(int64_t n);
dgr_status dgr_densify(const dgr_gaussians *src, int64_t n, const float *acc, const float *normals,
                       const dgr_grid *grid, const dgr_densify_params *params,
                       const dgr_gaussians *dst, int64_t *n_out, int64_t counts[3], void *ws,
                       size_t ws_bytes, void *stream);

/* ---- the paper's full objective (sec. 4.3, App. D.1) ------------------------ */
/* L = w1 L1(P_hat, P) + w2 L_SSIM(P_hat, P) + w3 L_TV(V), the paper's weights
 * being 0.6, 0.2, 1.  L1 = mean |P_hat - P|; L_SSIM = 1 - mean over every view
 * and pixel of the SSIM map (App. C.2 formula) of each 2-D view, with local
 * statistics from an 11 x 11 Gaussian window (sigma 1.5, normalised, zero
 * padding outside the detector), C1 = (0.01 R)^2, C2 = (0.03 R)^2;
 * L_TV = mean over voxels of the absolute forward differences along x, y, z. */

/* Projection terms: proj, target [n_views][nv][nu] (DEVICE); range R > 0, or
 * <= 0 to use max(target).  Writes loss (DEVICE binary32 [3]) = {w1 L1 +
 * w2 L_SSIM, L1, L_SSIM} and dproj = dL/dP_hat (overwritten).  SSIM moments,
 * maps and their blur are binary64. */
size_t dgr_projection_loss_workspace(int32_t n_views, int32_t nv, int32_t nu);
dgr_status dgr_projection_loss(const float *proj, const float *target, int32_t n_views, int32_t nv,
                               int32_t nu, float w_l1, float w_ssim, float range, float *loss,
                               float *dproj, void *ws, size_t ws_bytes, void *stream);
/* Volume term: loss (DEVICE binary32 [1]) = L_TV(volume); dvolume +=
 * w_tv dL_TV/dV (accumulated into the caller's dL/dV; sign(0) = 0). */
size_t dgr_tv_workspace(void);
dgr_status dgr_tv(const float *volume, const dgr_grid *grid, float w_tv, float *loss, float *dvolume,
                  void *ws, size_t ws_bytes, void *stream);

/* ---- learned initialisation: a 3-D U-Net on the matrix cores -------------- */
/* Not part of DGR (the paper initialises its Gaussians from an FBP/FDK volume,
 * Fig. 4 caption, or at random): a network that maps a one-channel volume to
 * per-voxel density, log-scale and occupancy-logit fields from which an
 * initial Gaussian set is drawn; the plain initialisation stays the fallback.
 *
 * Network (base width B = 32, volume extents multiples of 8 in [8, 1024]):
 *   enc1 = relu(conv3(x; 1->B)),  enc2 = relu(conv3(pool(enc1); B->2B)),
 *   enc3 = relu(conv3(pool(enc2); 2B->4B)), bott = relu(conv3(pool(enc3); 4B->8B)),
 *   dec3 = relu(conv3([up(bott), enc3]; 12B->4B)),
 *   dec2 = relu(conv3([up(dec3), enc2]; 6B->2B)),
 *   dec1 = relu(conv3([up(dec2), enc1]; 3B->B)),  out = head(dec1; B->3).
 * conv3: 3x3x3 cross-correlation, zero padding 1; tap t = 9(dz+1)+3(dy+1)+(dx+1)
 * multiplies x[z+dz][y+dy][x+dx].  pool: 2x2x2 mean.  up: nearest 2x.  [a, b]:
 * channel concatenation.  head: 1x1x1 convolution.
 * Parameters (binary32, flat): for enc1, enc2, enc3, bott, dec3, dec2, dec1 in
 * turn W[27][Cout][Cin] then b[Cout]; then head W[3][B], b[3] (2,904,707 values).
 * Activations and activation gradients are bfloat16, products accumulate in
 * binary32.  Volumes are [nz][ny][nx] (x fastest); dims = {nx, ny, nz}; out
 * is [nz][ny][nx][3] = (density, log-scale, occupancy logit).
 * All pointers are DEVICE pointers; ws is 256-byte aligned and holds the
 * activations: dgr_unet_backward must follow dgr_unet_forward with the same
 * params, input, dims and ws on the same stream. */
int64_t dgr_unet_param_count(int32_t base);  /* -1 if base is not 32 */
size_t dgr_unet_workspace(const int32_t dims[3], int32_t base);  /* 0 if unsupported */
dgr_status dgr_unet_forward(const float *params, const float *input, const int32_t dims[3],
                            int32_t base, float *out, void *ws, size_t ws_bytes, void *stream);
/* grad (binary32, flat like params) = d sum(dout * out) / d params. */
dgr_status dgr_unet_backward(const float *params, const float *input, const int32_t dims[3],
                             int32_t base, const float *dout, float *grad, void *ws,
                             size_t ws_bytes, void *stream);
/* Training loss over n voxels, target [n][3] = (t_d, t_s, t_o), t_o in [0, 1]:
 * L = mean (o_d - t_d)^2 + mean t_o (o_s - t_s)^2 + mean (softplus(o_o) - t_o o_o);
 * *loss (DEVICE binary32) and dout = dL/dout [n][3]. */
size_t dgr_unet_loss_workspace(void);
dgr_status dgr_unet_loss(const float *out, const float *target, int64_t n_voxels, float *loss,
                         float *dout, void *ws, size_t ws_bytes, void *stream);

/* 2x2x2 mean of a binary32 volume [nz][ny][nx] (dims even) into
 * [nz/2][ny/2][nx/2]: the network is trained at twice the voxel size of the
 * reconstruction grid and reads the pooled FDK volume. */
dgr_status dgr_pool2_f32(const float *in, const int32_t dims[3], float *out, void *stream);

/* Training targets on `grid` from a converged Gaussian set (mu, scale [n][3])
 * and its voxelization `volume`: target[v] = (volume[v] / input_scale,
 * mean over the Gaussians whose mean lies in v of log(geometric-mean scale in
 * voxels) or 0, 1 if there is such a Gaussian else 0).  Sums are fixed point
 * (deterministic). */
size_t dgr_unet_targets_workspace(const dgr_grid *grid);
dgr_status dgr_unet_targets(const float *mu, const float *scale, int64_t n, const dgr_grid *grid,
                            const float *volume, float input_scale, float *target, void *ws,
                            size_t ws_bytes, void *stream);

/* Initial Gaussians drawn from the network's output out [V][3] on `grid`:
 * voxel weight sigmoid(o_o), drawn with replacement by inverse CDF as in
 * dgr_init_from_volume (uniforms [n][4]), mean = voxel centre +
 * (uniforms[i][1..3] - 1/2) voxel, isotropic scale exp(o_s) voxels clamped
 * to [0.25, 8], identity rotation, density max(o_d, 0) * input_scale. */
size_t dgr_init_from_unet_workspace(const dgr_grid *grid);
dgr_status dgr_init_from_unet(const float *out, const dgr_grid *grid, int64_t n,
                              const float *uniforms, float input_scale, float *mu, float *scale,
                              float *quat, float *density, void *ws, size_t ws_bytes, void *stream);

/* One conv3 layer on the matrix cores (the network's building block).
 * x: bfloat16 [nz][ny][nx][x_stride] (channels 0..cin-1 read); w: bfloat16
 * [27][cout][cin]; bias: binary32 [cout] or NULL; y: bfloat16
 * [nz][ny][nx][y_stride] (channels 0..cout-1 written, rounded to nearest
 * even), relu != 0 clamps at zero.  cin, cout multiples of 32; strides
 * multiples of 8; x, w, y 16-byte aligned. */
dgr_status dgr_conv3_forward(const uint16_t *x, int32_t x_stride, const int32_t dims[3],
                             int32_t cin, const uint16_t *w, const float *bias, int32_t cout,
                             int32_t relu, uint16_t *y, int32_t y_stride, void *stream);
/* Backward of y = conv3(x; w) + b for dy (bfloat16 [nz][ny][nx][cout]):
 * dw (binary32 [27][cout][cin]), db (binary32 [cout]) and dx (bfloat16
 * [nz][ny][nx][cin]).  w is binary32 here (rounded to bfloat16 inside);
 * cin, cout multiples of 32 with cout <= 256. */
size_t dgr_conv3_grad_workspace(const int32_t dims[3], int32_t cin, int32_t cout);
dgr_status dgr_conv3_backward(const uint16_t *x, int32_t x_stride, const int32_t dims[3],
                              int32_t cin, const float *w, const uint16_t *dy, int32_t cout,
                              float *dw, float *db, uint16_t *dx, void *ws, size_t ws_bytes,
                              void *stream);

/* ---- binary64 path for finite-difference gradient checks ------------------ */

/* The volume of dgr_voxelize evaluated in binary64 (parameters promoted
 * exactly from binary32), volume [nz][ny][nx] binary64, overwritten.  Same
 * boxes and workspace as dgr_voxelize. */
size_t dgr_voxelize_f64_workspace(int64_t n, int64_t max_pairs, const dgr_grid *grid);
dgr_status dgr_voxelize_f64(const float *mu, const float *scale, const float *quat,
                            const float *density, int64_t n, const dgr_grid *grid,
                            const dgr_trunc *trunc, double *volume, void *ws, size_t ws_bytes,
                            void *stream);

/* Finite differences of the mean-L1 projection loss (sec. 4.3) for n_jobs
 * (Gaussian, component, step) jobs.  Component 0-2 = mean x,y,z, 3-5 = scale,
 * 6-9 = quaternion w,x,y,z, 10 = density.  The job's Gaussian keeps its
 * truncation box; only rays crossing it change, so the kernel sums, over
 * those rays, |res + A dV| - |res| with res = A V - target computed in
 * binary64 from `volume` (dgr_voxelize_f64) and dV the binary64 change of the
 * Gaussian on its box for +h and -h.  out [n_jobs][2] (DEVICE, binary64):
 * the loss changes L(+h) - L and L(-h) - L, each the sum over views (in view
 * order) of the per-view sums, divided by M = n_views*nu*nv.  job_gid,
 * job_comp, job_h are HOST arrays.  box_cap bounds the voxels of any job's
 * box (larger boxes give NaN).  Synchronises `stream`. */
size_t dgr_fd_l1_f64_workspace(int64_t n, int32_t n_jobs, int64_t box_cap, const dgr_geometry *geom);
dgr_status dgr_fd_l1_f64(const double *volume, const dgr_grid *grid, const dgr_geometry *geom,
                         const float *target, const float *mu, const float *scale, const float *quat,
                         const float *density, int64_t n, const dgr_trunc *trunc,
                         const int32_t *job_gid, const int32_t *job_comp, const double *job_h,
                         int32_t n_jobs, int64_t box_cap, double *out, void *ws, size_t ws_bytes,
                         void *stream);

/* ---- inspection ---------------------------------------------------------- */

/* Truncation boxes int32 [n][6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z). */
dgr_status dgr_bbox(const float *mu, const float *scale, const float *quat, int64_t n,
                    const dgr_grid *grid, const dgr_trunc *trunc, int32_t *box, void *stream);

/* The sorted (tile, Gaussian) pair list used by dgr_voxelize:
 * pairs uint32 [P][2] = (tile, gid) ascending, tile = (tz*Ty + ty)*Tx + tx
 * with T_a = ceil(dims_a/8); tile_begin uint32 [Tx*Ty*Tz + 1].  Needs
 * P <= capacity of ws; P comes from dgr_voxelize_plan. */
dgr_status dgr_bin(const float *mu, const float *scale, const float *quat, int64_t n,
                   const dgr_grid *grid, const dgr_trunc *trunc, uint32_t *pairs,
                   uint32_t *tile_begin, void *ws, size_t ws_bytes, void *stream);

/* Synchronises `stream` and reports a capacity overflow recorded in a
 * voxelization workspace (DGR_ERR_CAPACITY) or DGR_OK.  Clears the flag. */
dgr_status dgr_check(void *ws, void *stream);

const char *dgr_status_string(dgr_status status);
const char *dgr_last_error(void);

/* Library version, for the binding's load check. */
int32_t dgr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DGR_H */
