/*
 * pics.h -- C ABI of libpics.so: the preconditioned conjugate gradient (PCG)
 * inner solve of Split Bregman for parallel-imaging + compressed-sensing MRI,
 * with the block-circulant-with-circulant-blocks (BCCB) preconditioner of
 * Koolstra, van Gemert, Boernert, Webb and Remis, "Accelerating CS in Parallel
 * Imaging Reconstructions Using an Efficient and Effective Circulant
 * Preconditioner" (arXiv 1710.01758).  Built for AMD MI355X (gfx950).
 *
 * Problem (paper, Theory, Eq. original):
 *   x^ = argmin mu/2 sum_i ||R F S_i x - y_i||^2 + ||D_x x||_1 + ||D_y x||_1 + ||W x||_1
 * solved by Split Bregman (Algorithm 1), whose step 5 is A x = b (Eq. system):
 *   A = mu sum_i (R F S_i)^H R F S_i + lambda (D_x^H D_x + D_y^H D_y) + gamma W^H W,
 * preconditioned by M^{-1} = F^H diag(k)^{-1} F with k = diag(F A F^H)
 * (Eqs. K, precon, Kdiag).
 *
 * Conventions shared by every entry point
 *   - complex data are interleaved float32 pairs (re, im), "c64".
 *   - an image is [m][n], row-major, n contiguous; axis 0 (length m) is the
 *     phase-encode axis that a line mask selects.  F is the unitary 2D DFT,
 *     DC at [0][0] (no fftshift).
 *   - a context holds a batch of nslices independent slices; image-shaped
 *     buffers pack the slices one after another (slice s starts at element
 *     sum_{s'<s} m_s' n_s'), coil-shaped buffers pack [nc_s][m_s][n_s] per
 *     slice, masks pack uint8[m_s] (line masks) or uint8[m_s][n_s] (2D
 *     masks) per slice.
 *     pics_sizes() returns the packed totals.
 *   - every data pointer is a device pointer owned by the caller; sizes are
 *     element counts.  The context borrows `sens` and `masks` until
 *     pics_destroy() and owns its workspace, allocated by pics_create and by
 *     the set-up calls below; the calls that do the work (apply_A,
 *     apply_Minv, pcg_solve, split_bregman_recon, ...) allocate nothing:
 *       - the iteration-lock table and the per-solve history of
 *         split_bregman_recon are sized for 64 solves (n_outer x n_inner) by
 *         pics_create; pics_reserve enlarges them (a reconstruction with more
 *         solves is refused with PICS_ERR_INVALID until then);
 *       - the coil-split partial sums (G x image-packed c64) are allocated by
 *         pics_autotune or pics_set_option when they choose a split G > 1
 *         (apply_A_noalloc uses a static array instead).
 *     A split_bregman_recon that replays outer iterations from a HIP graph
 *     instantiates that graph on its first call with a given output buffer,
 *     tolerance and preconditioner (the HIP runtime then sets up the graph's
 *     resources); later calls with the same arguments replay it.
 *   - calls are ordered on the stream given at creation and asynchronous
 *     unless they return host results (those synchronise that stream).
 *     One host thread per context at a time; separate contexts (each on
 *     its own stream) may be driven from separate host threads at once.
 *   - return value: 0 = OK, > 0 = warning, < 0 = error (see PICS_*).  Errors
 *     detected on the host are reported before anything is launched; the
 *     library never aborts.  pics_last_error() gives a message.
 */
#ifndef PICS_H
#define PICS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PICS_OK 0
#define PICS_WARN_MAXIT 1        /* a PCG solve stopped at maxit without reaching tol */
#define PICS_WARN_FALLBACK 2     /* learned spectrum rejected (k <= 0 or not finite); circulant used */
#define PICS_ERR_INVALID (-1)    /* bad argument (null pointer, size, parameter) */
#define PICS_ERR_UNSUPPORTED (-2)/* size without an FFT plan, mask kind or wavelet not available */
#define PICS_ERR_NONFINITE (-3)  /* non-finite scalar inside PCG */
#define PICS_ERR_BREAKDOWN (-4)  /* p^H A p <= 0 inside PCG */
#define PICS_ERR_NOT_POSITIVE (-5)/* circulant spectrum k has a non-positive entry */
#define PICS_ERR_HIP (-6)        /* HIP runtime error */
#define PICS_ERR_STATE (-7)      /* call needs a preconditioner that was not built */

#define PICS_MASK_LINES 0        /* uint8[m]: k-space row u sampled (all of axis 1) */
#define PICS_MASK_2D 1           /* uint8[m][n]: any sampling pattern (Methods, Undersampling, second scheme) */

#define PICS_WAVELET_NONE 0
#define PICS_WAVELET_HAAR 1
#define PICS_WAVELET_DB4 2       /* 8-tap Daubechies, 4 vanishing moments, periodised */

#define PICS_PRECOND_NONE 0
#define PICS_PRECOND_JACOBI 1    /* diag(A)^{-1} (paper, Results: no gain) */
#define PICS_PRECOND_CIRCULANT 2 /* F^H diag(k)^{-1} F, Eq. precon */
#define PICS_PRECOND_LEARNED 3   /* circulant with k multiplied by a caller-given correction */

#define PICS_TERM_DATA 1         /* mu sum_i (R F S_i)^H R F S_i */
#define PICS_TERM_TV 2           /* lambda (D_x^H D_x + D_y^H D_y), periodic backward differences */
#define PICS_TERM_GAMMA 4        /* gamma W^H W = gamma I (W unitary) */
#define PICS_TERM_ALL 7
#define PICS_TERM_WAVELET_EXPLICIT 8 /* with PICS_TERM_GAMMA: evaluate gamma W^H W x through the wavelet
                                        analysis and synthesis instead of gamma x (apply_A only) */

/* One slice.  m, n in {64, 128, 192, 224, 256, 320, 512, 1024}; ncoils >= 1;
 * levels: wavelet levels (each level needs even extents); mu, lambda,
 * gamma >= 0 and finite (Split Bregman needs lambda, gamma > 0: its shrink
 * thresholds are 1/lambda and 1/gamma, Algorithm 1 steps 6-8). */
typedef struct pics_desc {
  int32_t m, n, ncoils;
  int32_t mask_kind;
  int32_t wavelet, levels;
  double mu, lambda, gamma;
} pics_desc;

typedef struct pics_ctx pics_ctx;

/* Create a context for nslices slices.  sens: packed coil sensitivities
 * S_i (c64, [nc][m][n] per slice; the paper normalises them so that
 * sum_i |S_i|^2 = 1, Methods, Coil sensitivity maps); masks: packed binary
 * masks R.  stream: a hipStream_t (NULL = default stream).
 * Returns PICS_ERR_INVALID / PICS_ERR_UNSUPPORTED for descriptors it cannot
 * serve, PICS_ERR_HIP if allocation fails. */
int pics_create(pics_ctx** ctx, int32_t nslices, const pics_desc* descs, const void* sens, const uint8_t* masks,
                void* stream);
int pics_destroy(pics_ctx* ctx);

/* Packed element counts: image-shaped (c64 elements), coil-shaped (c64
 * elements) and mask bytes. */
int pics_sizes(const pics_ctx* ctx, int64_t* image_elems, int64_t* coil_elems, int64_t* mask_bytes);

/* Room for split_bregman_recon runs of up to max_solves = n_outer x n_inner
 * solves (iteration-lock schedule and per-solve history, 3 x max_solves x
 * nslices int32); pics_create reserves 64.  A set-up call: it synchronises
 * the stream and allocates when max_solves exceeds the current room, and does
 * nothing otherwise.  PICS_ERR_INVALID outside 1 .. 2^20. */
int pics_reserve(pics_ctx* ctx, int32_t max_solves);

/* Build the preconditioner (paper, Efficient Implementation of the
 * Preconditioner, Eqs. d and diagonalelements; Table 1 lists its cost):
 * k = mu k_c + lambda k_d + gamma, k_c(j) = (1/N^2) sum_l r(l) P(l - j) with
 * P = sum_i |DFT(s_i)|^2, k_d the symbol of the periodic Laplacian.
 * kind: PICS_PRECOND_*.  correction: float per pixel (image-packed),
 * required for LEARNED (k <- k * correction), else ignored.  khat_out:
 * optional float per pixel receiving k.  Synchronises the stream.  Returns
 * PICS_ERR_NOT_POSITIVE if k has an entry <= 0 (e.g. gamma = 0 with the DC
 * line unsampled); for LEARNED a rejected correction falls back to the
 * circulant k with PICS_WARN_FALLBACK. */
int build_preconditioner(pics_ctx* ctx, int32_t kind, const float* correction, float* khat_out);

/* y = A x for every slice (Eq. system); terms selects PICS_TERM_* parts
 * (PICS_TERM_WAVELET_EXPLICIT routes the gamma term through W and W^H).
 * x and y image-packed c64, must not alias.  Line masks use one fused
 * kernel (the data term factors into axis-0 transforms); 2D masks use
 * row / column / row passes of full 2D transforms through the context's
 * coil-shaped workspace.  With 2D masks k_c is the 2D cross-correlation,
 * computed with FP32 FFTs. */
int apply_A(pics_ctx* ctx, const void* x, void* y, int32_t terms);

/* apply_A for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same operator and terms as apply_A (x, y as there), with every column
 * tile's coil loop split over min(coil_groups, coil count of the size group)
 * workgroups whose partial data terms (coil_groups x image-packed c64) go to
 * a static device array of the library, PICS_NOALLOC_SCRATCH_BYTES per GPU,
 * instead of the context's grow-only split table; coil_groups = 1 is the
 * fused single pass and touches no scratch.  Slices with 2D masks run as in
 * apply_A, through the context's coil workspace.  Allocates nothing and does
 * not synchronise; the array's device address is looked up by pics_create
 * (once per GPU) and the array is held until the process ends.
 * PICS_ERR_INVALID if coil_groups is outside 1..64 or the split needs more
 * than PICS_NOALLOC_SCRATCH_BYTES (8 bytes x image elements x split); nothing
 * is launched then.  Every call on one GPU shares the array, which keeps the
 * last call's partial sums (each is written before it is read, so nothing
 * needs to start at zero): calls that overlap on one GPU (other streams,
 * contexts or host threads) race and must be ordered by the caller. */
#define PICS_NOALLOC_SCRATCH_BYTES (32 << 20)
int apply_A_noalloc(pics_ctx* ctx, const void* x, void* y, int32_t terms, int32_t coil_groups);

/* z = M^{-1} r = F^H diag(k)^{-1} F r (Eq. precon); needs a CIRCULANT or
 * LEARNED build.  r and z image-packed c64, must not alias. */
int apply_Minv(pics_ctx* ctx, const void* r, void* z);

/* Unnormalised 2D DFT of every slice: out = sum exp(-+2 pi i (u i / m + v j / n)) in.
 * inverse = 0: forward (minus sign), 1: inverse (plus sign, no 1/N). */
int pics_fft2(pics_ctx* ctx, const void* in, void* out, int32_t inverse);

/* Orthonormal periodised wavelet transform W (inverse = 0) or W^H
 * (inverse = 1) per slice, Mallat layout, `levels` levels (paper, Theory:
 * W unitary).  in and out image-packed c64, must not alias. */
int pics_wavelet(pics_ctx* ctx, const void* in, void* out, int32_t inverse);

/* Solve A x = b by PCG with the preconditioner of the last build (none if
 * never built): paper, Complexity section (left preconditioning; equivalent
 * to standard PCG for Hermitian positive definite A and M).  x holds x0 on
 * entry and the solution on exit.  Stops per slice when the recursive
 * residual satisfies ||r|| <= tol ||b|| or after maxit iterations
 * (iteration = one product A p).  maxit_per_slice (host, nslices entries,
 * optional) overrides maxit per slice; with tol = 0 it fixes the iteration
 * count exactly.  Vectors are FP32, inner products and alpha / beta FP64.
 * Host outputs (optional, nslices entries each): iterations, final relative
 * residual, status (1 converged, 0 stopped at the cap, < 0 error).
 * Returns PICS_WARN_MAXIT if a slice stopped at the cap with tol > 0. */
int pcg_solve(pics_ctx* ctx, const void* b, void* x, double tol, int32_t maxit, const int32_t* maxit_per_slice,
              int32_t* iters_host, double* relres_host, int32_t* status_host);

/* Split Bregman reconstruction (Algorithm 1) of every slice from zero-filled
 * k-space y (coil-packed c64; samples outside the mask are ignored).
 * x^[1] = root sum of squares of the coil images; n_outer outer and n_inner
 * inner iterations; each step-5 solve is pcg_solve with the current
 * preconditioner, warm-started from the latest x.  lock_iters (host,
 * optional, [n_outer * n_inner][nslices]) fixes the PCG iteration count of
 * each solve (tol ignored).  x_out: image-packed c64 result.  pcg_iters
 * (host, optional, [n_outer * n_inner][nslices]) receives the counts. */
int split_bregman_recon(pics_ctx* ctx, const void* kspace, int32_t n_outer, int32_t n_inner, double tol,
                        int32_t maxit, const int32_t* lock_iters, void* x_out, int32_t* pcg_iters);

/* Coil compression (Methods, Coil compression): per slice the covariance
 * C = sum over k-space samples of y y^H of the slice's coil data, its
 * eigenvectors U by descending eigenvalue (cyclic Jacobi in FP64 on the GPU),
 * and the nvirt most dominant virtual coils y_v = U_v^H y and S_v = U_v^H S
 * of the data and of the context's coil maps.  kspace: coil-packed c64 as
 * for split_bregman_recon; kspace_out, sens_out: caller-owned, packed with
 * nvirt coils per slice (nvirt m_s n_s c64 elements for slice s, slices in
 * order) -- a new context over sens_out with ncoils = nvirt reconstructs the
 * compressed problem.  eig_out (host, optional): the eigenvalues of every
 * slice, descending, concatenated (ncoils_s per slice).  Uses the context's
 * coil workspace; at most 32 coils per slice (PICS_ERR_UNSUPPORTED);
 * 1 <= nvirt <= ncoils of every slice (PICS_ERR_INVALID).  Synchronises the
 * stream when eig_out is given. */
int pics_coil_compress(pics_ctx* ctx, const void* kspace, int32_t nvirt, void* kspace_out, void* sens_out,
                       double* eig_out);

/* Options.
 * PICS_OPT_POLL_CHUNK: PCG iterations enqueued between host convergence polls
 *   (first poll; later polls double it, up to 32).  Default 2.
 * PICS_OPT_GRAPH_BUDGET: split_bregman_recon runs a whole reconstruction
 *   (initialisation and every outer iteration) from one captured HIP graph
 *   whose PCG solves carry a fixed number of iterations, this many for every
 *   solve but the first (kernels of converged slices exit at entry).  If a
 *   solve needs more, the reconstruction is redone host-polled, so results
 *   never depend on the budgets; the context then raises the budget that was
 *   short (to 2, then doubling).  0 disables the graph (every solve
 *   host-polled).  Default 1.
 * PICS_OPT_GRAPH_FIRST_BUDGET: the graph's budget for the first solve (from
 *   the root-sum-of-squares start), 1 .. 256, doubled after a shortfall.
 *   Default 8.
 * PICS_OPT_COIL_GROUPS: split every column tile's coil loop over this many
 *   workgroups (clamped to each group's coil count), overriding the
 *   autotuner; 1 = no split (the default before pics_autotune).  The split
 *   applies to the size group's slice with the most coils; a slice with
 *   fewer coils takes only as many workgroups as keep each at or below that
 *   slice's coils per workgroup.  A split above 1 runs with the default
 *   column tiles.
 * PICS_OPT_COL_TILE: columns per workgroup of the line-mask operator for
 *   every size group, overriding the autotuner: 0 = the default (16 up to
 *   length 320, 4 at 512, 8 at 1024) or one of the two alternatives of each
 *   length (8 and 32 at 64, 128 and 224; 8 and 4 at 192, 256 and 320; 8 and
 *   2 at 512; 4 and 2 at 1024), at most 256 tiles per slice;
 *   PICS_ERR_INVALID otherwise.  A width other than the default resets the
 *   coil split to 1.
 * PICS_OPT_CONCURRENT_GROUPS: 1 (default) runs the per-size-group kernels of
 *   a batch with several slice sizes on side streams of the context (forked
 *   from and joined back to the caller's stream with events, also under
 *   graph capture); 0 runs them one group after the other on the caller's
 *   stream.  Results are identical either way. */
#define PICS_OPT_POLL_CHUNK 1
#define PICS_OPT_GRAPH_BUDGET 2
#define PICS_OPT_COIL_GROUPS 3
#define PICS_OPT_CONCURRENT_GROUPS 4
#define PICS_OPT_COL_TILE 5
#define PICS_OPT_GRAPH_FIRST_BUDGET 6
int pics_set_option(pics_ctx* ctx, int32_t key, int64_t value);

/* ---------------------------------------------------------------------------
 * Learned correction of the circulant spectrum (not in the paper).
 *
 * A small CNN maps per-slice features to a positive correction c of k; the
 * LEARNED preconditioner is F^H diag(1/(k c)) F.  It is trained to minimise
 * E_z ||M_c^{-1} A z - z||^2 / E_z ||z||^2 over random probes z, which per
 * frequency j is d_j^2 G_j - 2 d_j H_j + Z_j (d = 1/(k c)) with the probe
 * statistics G = E|F A z|^2, H = E Re(conj(F A z) F z), Z = E|F z|^2.
 *
 * Network: six 3x3 convolutions with circular padding and ReLU,
 * (cin, cout, dilation) = (6,32,1) (32,32,1) (32,32,2) (32,32,4) (32,32,8)
 * (32,16,1), then a 1x1 convolution 16 -> 1 giving o; c = max(softplus(o),
 * 1e-3).  Flat FP32 parameter order: per 3x3 layer W[cout][cin][3][3] then
 * bias[cout]; then w[16], bias[1] (43105 values).  Activations bf16 on the
 * matrix cores, FP32 weights, accumulation and optimiser state.
 * Features: float [slice][6][64][64] on the fft-shifted 64 x 64 frequency
 * grid (DC at (32, 32)): sampled fraction, log(coil energy / mean),
 * log(k / mean), log10(mu/1e-3), log10(lambda/4e-3), log10(gamma/4e-3);
 * slices must have m and n multiples of 64.
 * ------------------------------------------------------------------------- */
typedef struct pics_net pics_net;

/* Feature planes of every slice of ctx from its masks, coil maps and the
 * spectrum khat (image-packed float, e.g. build_preconditioner's khat_out).
 * PICS_ERR_UNSUPPORTED if a slice's m or n is not a multiple of 64. */
int pics_features(pics_ctx* ctx, const float* khat, float* features);

/* Probe statistics G, H, Z (image-packed float, unitary DFT scaling) of A over
 * nprobes probes (image-packed c64 each, back to back). */
int pics_probe_stats(pics_ctx* ctx, const void* probes, int32_t nprobes, float* G, float* H, float* Z);

/* Network with room for batches of up to batch_max slices; stream = hipStream_t. */
int pics_net_create(pics_net** net, int32_t batch_max, void* stream);
int pics_net_destroy(pics_net* net);
int64_t pics_net_param_count(void);
/* Host copies of the flat parameters / the last gradient. */
int pics_net_set_params(pics_net* net, const float* params_host);
int pics_net_get_params(pics_net* net, float* params_host);
int pics_net_get_grad(pics_net* net, float* grad_host);

/* o = network(features[index[b]]) for b < batch (index: device int32, NULL =
 * identity); o: float [batch][64][64] on the shifted grid. */
int pics_net_forward(pics_net* net, int32_t batch, const int32_t* index, const float* features, float* o);

/* Loss (mean over the batch) and its gradient (kept in the network) for the
 * slices index[0..batch): features [slice][6][64][64]; k, G, H, Z
 * [slice][64][64] (unshifted).  Synchronises the stream; loss_host optional. */
int pics_net_loss_grad(pics_net* net, int32_t batch, const int32_t* index, const float* features, const float* k,
                       const float* G, const float* H, const float* Z, double* loss_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradient. */
int pics_net_adam_step(pics_net* net, float lr);

/* Correction map c for every slice of ctx (image-packed float), from the
 * slice features: network output interpolated periodically-bilinearly from
 * the 64 x 64 shifted grid to m x n, unshifted.  Feed it to
 * build_preconditioner(PICS_PRECOND_LEARNED). */
int pics_net_correction(pics_net* net, pics_ctx* ctx, const float* features, float* correction);

/* Autotuner.  Per group of equal-size slices, times the fused operator for
 * each launch shape -- the default column tiles with each way of splitting a
 * tile's coil loop over 1, 2, 3, 4, 6, 8 or 12 workgroups (the split adds the
 * groups' partial sums in a second pass, in fixed order), and the two
 * alternative tile widths of the length (PICS_OPT_COL_TILE) without a split
 * -- and keeps the fastest for every later call.  Choices are cached per (GPU
 * arch, CU count, m, n, largest coil count, slices) in $PICS_TUNE_CACHE
 * (default ~/.cache/pics_autotune.txt).  Synchronises the stream; allocates
 * the partial-sum workspace when a split is chosen.
 * flags: PICS_TUNE_FORCE re-times even if cached; PICS_TUNE_NO_WRITE keeps
 * the cache file unchanged. */
#define PICS_TUNE_FORCE 1
#define PICS_TUNE_NO_WRITE 2
int pics_autotune(pics_ctx* ctx, int32_t flags);
/* Chosen coil split per size group (in order of first appearance); returns
 * the number of groups. */
int pics_get_tuning(const pics_ctx* ctx, int32_t* coil_groups, int32_t max_groups);
/* Chosen column-tile width per size group (0 for groups with 2D masks);
 * returns the number of groups. */
int pics_get_tuning_tiles(const pics_ctx* ctx, int32_t* tiles, int32_t max_groups);

const char* pics_status_string(int status);
const char* pics_last_error(const pics_ctx* ctx);

/* ---------------------------------------------------------------------------
 * 3D extension (the paper's Discussion names it as the next step): one volume
 * [p][m][n] (axis 0 = z), coil maps [nc][p][m][n], a binary mask [p][m][n],
 *   A = mu sum_c S_c^H F^H R F S_c + lambda (D_z^H D_z + D_y^H D_y + D_x^H D_x)
 *       + gamma I
 * with the unitary 3D DFT F and periodic backward differences, and the 3D
 * circulant preconditioner k = mu k_c + lambda k_d + gamma, k_c(j) = (1/N^2)
 * sum_l r(l) P(l - j), P = sum_c |DFT(s_c)|^2, k_d = 6 - 2 cos(2 pi w/p)
 * - 2 cos(2 pi u/m) - 2 cos(2 pi v/n) (Eqs. K, Kdiag, d, diagonalelements one
 * dimension up).  p, m, n must each have an FFT plan.  Buffers are device
 * c64 volumes owned by the caller; the context borrows sens and mask and owns
 * a workspace of 2 nc + 5 complex volumes.  Return codes as above. */
typedef struct {
  int32_t p, m, n, ncoils;
  double mu, lambda, gamma;
} pics3d_desc;
typedef struct pics3d_ctx pics3d_ctx;
int pics3d_create(pics3d_ctx** ctx, const pics3d_desc* desc, const void* sens, const uint8_t* mask, void* stream);
int pics3d_destroy(pics3d_ctx* ctx);
/* kind: PICS_PRECOND_NONE or PICS_PRECOND_CIRCULANT; khat_out (optional,
 * device float [p][m][n]) receives k.  Synchronises the stream. */
int pics3d_build_preconditioner(pics3d_ctx* ctx, int32_t kind, float* khat_out);
int pics3d_apply_A(pics3d_ctx* ctx, const void* x, void* y);
/* b = mu sum_c S_c^H F^H R y_c (the data part of the right-hand side, Eq.
 * system); kspace: [nc][p][m][n] c64 (samples outside the mask ignored). */
int pics3d_rhs(pics3d_ctx* ctx, const void* kspace, void* b);
int pics3d_apply_Minv(pics3d_ctx* ctx, const void* r, void* z);
/* PCG from the x given (Saad, Alg. 9.1, as pcg_solve): stop when
 * ||r|| <= tol ||b|| or after maxit products A p (PICS_WARN_MAXIT); tol = 0
 * runs exactly maxit iterations.  iters, relres: host, optional. */
int pics3d_pcg_solve(pics3d_ctx* ctx, const void* b, void* x, double tol, int32_t maxit, int32_t* iters,
                     double* relres);
const char* pics3d_last_error(const pics3d_ctx* ctx);
/* Options of a 3D context.  PICS3D_OPT_XCHUNK: for masks constant along x the
 * operator runs in chunks of X columns of the x axis, each through three
 * passes over a chunk workspace [nc][p][m][X] (kept small enough to stay in
 * the last-level cache between its passes); value: X, a multiple of the
 * column tile of the m axis (16 up to m = 320, 4 at 512, 8 at 1024) that
 * divides n, or 0 for the widest X whose workspace is at most 128 MiB
 * (PICS_ERR_INVALID otherwise).  get_option gives the X in use (0 when the
 * mask varies along x and the operator takes the full 3D transforms). */
#define PICS3D_OPT_XCHUNK 1
int pics3d_set_option(pics3d_ctx* ctx, int32_t option, int32_t value);
int pics3d_get_option(const pics3d_ctx* ctx, int32_t option, int32_t* value);

#ifdef __cplusplus
}
#endif

#endif /* PICS_H */
