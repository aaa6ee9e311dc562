/*
 * spalu.h - C ABI of the MI355X (gfx950) recursive sparse LU library.
 *
 * The library factors A x = b for a finite-difference matrix on a regular
 * 2D or 3D grid (the linear system of eq. (1.2); any invertible matrix
 * whose graph is the 5-point or 7-point stencil, symmetric or not) with the
 * recursive sparse LU "spaLU" of Zhu & Lai (arXiv 2408.14193):
 * nested dissection with segments (Section 3, Algorithm 1), leaf
 * elimination, per-level hybrid-sampled interpolative decompositions with
 * Schur sparsification, segment LU and separator elimination (Section 4,
 * Algorithm 2), and the solve x = V~ W~ b (eq. (4.13)), optionally followed
 * by FP64 iterative refinement.
 *
 * Conventions for every entry point:
 *   - Return value: SPALU_OK (0) or a negative SPALU_E* code.  On failure a
 *     thread-local message is available from spalu_last_error(), output
 *     handles are set to NULL and nothing throws across the ABI.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the current device.  All device work is enqueued on
 *     the caller's stream (a hipStream_t passed as void*, NULL = the null
 *     stream); calls return after their last host read, so results are
 *     ready once the caller synchronises that stream.
 *   - Working memory is the caller's: the caller queries a size, allocates
 *     (for example through PyTorch's caching allocator) and passes the
 *     buffer, which must stay alive until the matching free.  The library
 *     itself allocates only one device copy of an ordering's static tables
 *     per precision and device (at the first spalu_factor), from which
 *     every factorization's workspace is filled; spalu_nd_free releases
 *     it.
 *   - An ordering handle (spalu_nd_t) caches host and device state of its
 *     factorizations (tables, staging buffers, captured solve graphs): calls
 *     that use one handle must not run concurrently from several threads.
 *   - Vertex ids: interior grid node (x, y, z) has id x + nx*(y + ny*z).
 */
#ifndef SPALU_H
#define SPALU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SPALU_OK = 0,
  SPALU_EINVAL = -1,       /* bad argument (null pointer, size, dims)         */
  SPALU_ENOMEM = -2,       /* workspace smaller than the queried size         */
  SPALU_ESINGULAR = -3,    /* a zero pivot in a diagonal block                */
  SPALU_ENOCONV = -4,      /* refinement did not reach the tolerance          */
  SPALU_EDEVICE = -5,      /* a HIP runtime call failed                       */
  SPALU_EUNSUPPORTED = -6  /* matrix pattern outside the grid stencil, etc.   */
};

enum { SPALU_FP64 = 0, SPALU_FP32 = 1 };

typedef struct spalu_nd_s spalu_nd_t;
typedef struct spalu_factor_s spalu_factor_t;

/* ---------------------------------------------------------------------------
 * Nested dissection (Section 3, Algorithm 1; separator rule of eq. (3.1)).
 *
 * On a regular grid the degree-biased separator growth runs straight, so
 * every box is bisected by the grid line (2D) or plane (3D) through its
 * median vertex, perpendicular to its longest side (ties: x, then y, then
 * z); children are the two halves without the separator.  All leaves sit at
 * depth L.  Segments of level l: connected pieces of one separator whose
 * vertices border the same depth-l boxes (regular = two boxes, junction =
 * fewer), refined so that each nests in one segment of level l-1.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t levels;    /* L; 0 = smallest L with all leaf sides <= leaf_max */
  int32_t leaf_max;  /* default 7 (leaf pitch 8 on 2^m - 1 grids)        */
} spalu_nd_opts;

/* dim = 2 or 3; grid = interior sizes (nx, ny[, nz]) (host).  opts may be
 * NULL.  *out receives a caller-owned handle (spalu_nd_free). */
int spalu_nd_order(int32_t dim, const int32_t* grid, const spalu_nd_opts* opts,
                   spalu_nd_t** out);

/* Sizes: number of unknowns, L, number of etree nodes, total segments over
 * all levels.  Any output pointer may be NULL. */
int spalu_nd_info(const spalu_nd_t* nd, int64_t* n, int32_t* levels, int64_t* nnodes,
                  int64_t* nsegments);

/* perm (host, n entries): new -> old elimination order: leaves in
 * left-first depth-first order, then separators of level L..1, each level
 * left to right, vertex ids ascending inside each node. */
int spalu_nd_perm(const spalu_nd_t* nd, int64_t* perm);

/* Elimination tree in perm order (host arrays of nnodes entries): first
 * position in perm, size, level (L+1 for leaves, 1 for the root
 * separator) and parent node (-1 for the root). */
int spalu_nd_etree(const spalu_nd_t* nd, int64_t* begin, int64_t* size, int32_t* level,
                   int64_t* parent);

/* Segments of level l (1..L).  Call once with verts == NULL to get
 * *nseg and *nverts, then with host arrays: seg_ptr (nseg+1), verts
 * (nverts; each segment's vertex ids ascending, segments ordered by their
 * smallest id), flags (nseg; bit0 regular, bit1 on a level-l separator),
 * parent (nseg; segment of level l-1 that contains it, -1 if eliminated at
 * level l), npairs/pairs (2*npairs ints: coupled (c, d) pairs incl. c == d,
 * sorted).  pairs may be NULL. */
int spalu_nd_segments(const spalu_nd_t* nd, int32_t level, int64_t* nseg, int64_t* nverts,
                      int64_t* seg_ptr, int32_t* verts, int32_t* flags, int32_t* parent,
                      int64_t* npairs, int32_t* pairs);

void spalu_nd_free(spalu_nd_t* nd);

/* ---------------------------------------------------------------------------
 * Factorization (Algorithm 2).
 * ------------------------------------------------------------------------- */
typedef struct {
  double eps;          /* ID tolerance, relative |R_jj| <= eps |R_11|; 0 = off */
  int32_t precision;   /* SPALU_FP64 (plain form) or SPALU_FP32 (mixed form)  */
  uint32_t seed;       /* Philox key for the Gaussian sampling matrix         */
  double rho;          /* near field: Chebyshev distance <= max(1, rho*span)  */
  int32_t h0;          /* first number of samples of the adaptive ID          */
  int32_t probes;      /* Gaussian probes of the a-posteriori ID check        */
  double tau;          /* accept the sampled ID if the largest probe error
                          is <= tau * sqrt(n - k) * eps * |R_11| (the
                          Frobenius bound of the unsampled truncation)  */
  const int32_t* h_init; /* optional device array, per (level, segment) start
                            samples; index = seg_base[l] + c, see
                            spalu_factor_seg_base; <= 0 entries use h0     */
  const float* rank_model; /* optional device parameters of the rank predictor
                            (spalu_mlp_param_count floats, layout of
                            spalu_mlp_train_step); when set, every level's
                            features feed a BF16 inference whose predicted
                            rank fraction y gives the start samples
                            ceil(rank_margin * n * y) + rank_pad (learned
                            form); overrides h_init                       */
  float* features_out;   /* optional device array (segments x 12 floats,
                            index seg_base[l] + c) receiving every level's
                            predictor features (training data)            */
  float rank_margin;     /* default 1.0                                     */
  int32_t rank_pad;      /* default 5 (the oversampling p of Section 4.2.3) */
  float rank_skip;       /* learned form: a segment whose predicted rank n y
                            is at least n - rank_skip is kept whole, without
                            an ID (exact: only its compression is given up);
                            0 = never; default 0.5                       */
  int32_t graph;         /* 1: the level sweep is captured as a HIP graph the
                            first time these pointers (workspace, matrix,
                            h_init, rank_model, features_out) and options
                            are seen on the ordering handle, and replayed on
                            later calls with the same ones (batching form;
                            up to 4 graphs per handle, not while profiling);
                            0 (default): direct launches                  */
  int32_t symmetric;     /* 1: symmetric form for a symmetric positive
                            definite A (Section 4.4.2: A_{s,n} and A_{n,s}^T
                            share one ID, L D L^T in place of LU): the ID
                            samples the rows of A_{n,s} only (Y = [A_{N,s};
                            G A_{F,s} / sqrt(h)]), the segment blocks are
                            factored without interchanges as L D L^T and
                            stored balanced as C^{-1} = D^{-1/2} L^{-1} and
                            C^{-T} (C = L D^{1/2}), so every level's matrix
                            stays symmetric and W~ = V~^T.  A that is not
                            symmetric gives SPALU_EINVAL, a pivot that is
                            not positive SPALU_ESINGULAR (the leaves keep
                            their pivoted LU).  0 (default): the stacked ID
                            and pivoted LU of any invertible A            */
} spalu_factor_opts;

typedef struct {
  int64_t n;
  int32_t levels;
  int64_t segments;          /* segments over all levels                     */
  int64_t sparsified;        /* segments that went through the ID            */
  int64_t sample_passes;     /* ID passes (>= sparsified; more = resampling) */
  int64_t resampled;         /* segments needing more than one pass          */
  int64_t max_front;         /* largest segment size seen                    */
  double q_tilde;            /* max_l e'_l / e_l (Section 6)                 */
  int64_t workspace_bytes;
  int32_t singular_level;    /* level of a zero pivot (-1 none)              */
} spalu_factor_info;

/* Default options (eps 1e-6, FP64, seed 1234, rho 0.5, h0 8, 5 probes,
 * tau 1, no rank predictor, margin 1.0, pad 5, skip 0.5, no graph). */
void spalu_factor_opts_default(spalu_factor_opts* o);

/* Launch-shape choices of the factorization and the solve, for callers that
 * tune them (the package's autotuner): they change how the work of a level is
 * mapped onto workgroups, not what is computed (results may differ by
 * rounding where a segment moves to a tier with another summation order).
 * Process-wide; factorizations started after spalu_tuning_set use them. */
typedef struct {
  int32_t id_lds_a;        /* LDS bytes of ID tier A (one wave per segment),
                              4096..65536; default 24576                    */
  int32_t id_lds_b;        /* tier B (four waves), 16384..155648; default 73728 */
  int32_t id_lds_b2;       /* tier B2 (eight waves), 16384..155648; default 155648 */
  int32_t id_lds_c;        /* tier C (eight waves, rows of Y beyond it in
                              scratch), 32768..155648; default 155648       */
  int32_t id_c_ydiv;       /* tier C keeps far rows and row tables in LDS when
                              they leave room for max(n, R / id_c_ydiv) rows
                              of Y: 1, 2 or 4; default 2                    */
  int32_t melim_lds;       /* least LDS of a 256-thread merge group,
                              16384..155648; default 65536                  */
  int32_t melim_wave_cap;  /* merge targets of at most this many DOFs take one
                              wave each, 8..32; default 32                   */
  int32_t solve_lanes_min; /* solve sweeps: the segment-size bound P of a
                              level starts here (8, 16, 32 or 64) and doubles
                              until the level's segments and neighbour
                              counts fit; default 8                          */
  int32_t solve_lanes_max; /* levels with P up to this take the one-wave
                              matrix-core kernels (16-row tiles), larger
                              ones the block kernels; default 64             */
} spalu_tuning;

void spalu_tuning_default(spalu_tuning* t);
int spalu_tuning_get(spalu_tuning* t);
/* SPALU_EINVAL (nothing changed) when a value is out of range. */
int spalu_tuning_set(const spalu_tuning* t);

/* Bytes of device workspace that spalu_factor needs for this ND and
 * options (static layout sized by uncompressed segment sizes). */
int spalu_factor_workspace(const spalu_nd_t* nd, const spalu_factor_opts* opts, size_t* bytes);

/* Index base of level l's segments in the per-segment arrays (h_init, and
 * spalu_factor_ranks): base[l] for l = 1..L, base[L+1] = total. */
int spalu_factor_seg_base(const spalu_nd_t* nd, int64_t* base /* L+2 */);

/* Factor the CSR matrix (device arrays: rowptr n+1, colind nnz, vals nnz;
 * column indices ascending in each row, pattern inside the stencil) on
 * stream.  workspace: device buffer of at least the queried bytes, owned
 * by the caller, kept by the factor until spalu_factor_free.  The CSR
 * arrays are borrowed too: solve reads them for refinement residuals, so
 * they must outlive the factor.  info (host) may be NULL.
 * Errors: EINVAL, ENOMEM, EUNSUPPORTED, ESINGULAR (info->singular_level),
 * EDEVICE.  Synchronises the stream once at the end (status readback). */
int spalu_factor(const spalu_nd_t* nd, int64_t n, const int64_t* rowptr, const int32_t* colind,
                 const double* vals, const spalu_factor_opts* opts, void* workspace,
                 size_t workspace_bytes, void* stream, spalu_factor_t** out,
                 spalu_factor_info* info);

/* Per-segment results of the factorization (host arrays of base[L+1]
 * entries, index seg_base[l] + c): size before the ID, skeleton rank,
 * samples of the accepted pass, number of passes.  Synchronises. */
int spalu_factor_ranks(const spalu_factor_t* f, int32_t* n_before, int32_t* rank, int32_t* h,
                       int32_t* passes);

/* Algorithmic flops and HBM bytes of the factorization (host computation
 * from the actual segment sizes: leaf LUs and Schur products, ID sampling and
 * CPQR, transforms and segment LUs, coupling scaling, separator Schur GEMMs
 * and merges).  Either output may be NULL. */
int spalu_factor_work(const spalu_factor_t* f, double* flops, double* bytes);

void spalu_factor_free(spalu_factor_t* f);

/* ---------------------------------------------------------------------------
 * Solve x = V~ W~ b (eqs. (4.12)-(4.13)) and FP64 iterative refinement
 * r = b - A x, x += M r until max_j ||r_j|| / ||b_j|| <= tol.
 * ------------------------------------------------------------------------- */
typedef struct {
  double tol;        /* target relative residual; 0 = direct solve only */
  int32_t max_iter;  /* refinement iterations (default 30)              */
  int32_t graph;     /* 1: capture one application of the factor (all
                        level sweeps) as a HIP graph on first use and
                        replay it; the graph is cached on the ND handle and
                        keyed by every pointer it bakes in.  0: direct
                        launches.  NULL opts means 0.                    */
  int32_t restart;   /* 0: classical refinement x += M r.  m > 0: each
                        refinement step solves A d = r by flexible GMRES(m)
                        with the factor as right preconditioner (FP64
                        basis, Hessenberg and residual; the factor applied
                        in its own precision) and stops its Arnoldi cycle as
                        soon as every column's correction residual is below
                        tol/2; max_iter then counts factor applications.
                        1 <= m <= 32.                                     */
} spalu_solve_opts;

typedef struct {
  int32_t iterations;
  double max_rel_residual;   /* max_j ||b_j - A x_j|| / ||b_j|| at exit   */
  double first_rel_residual; /* same after the direct solve               */
} spalu_solve_info;

/* Bytes of device workspace for nrhs right-hand sides and the given options
 * (NULL: direct solve / classical refinement; the GMRES basis of
 * opts->restart > 0 takes (2 m + 1) n nrhs doubles more). */
int spalu_solve_workspace(const spalu_factor_t* f, int32_t nrhs, const spalu_solve_opts* opts,
                          size_t* bytes);

/* Refinement stops early, with ENOCONV, when three consecutive steps fail to
 * reduce the largest column residual by 10 %, or when it is not finite.
 *
 * B, X: device, column-major n x nrhs with leading dimensions ldb, ldx >= n
 * (FP64).  X may equal B.  opts, info (host) may be NULL (direct solve).
 * rel_res (host, nrhs entries, may be NULL) receives the final relative
 * residual of each column.  With refinement the call synchronises once per
 * iteration (residual norm readback); ENOCONV if tol is not reached in
 * max_iter iterations (X holds the last iterate). */
int spalu_solve(const spalu_factor_t* f, int32_t nrhs, const double* B, int64_t ldb, double* X,
                int64_t ldx, const spalu_solve_opts* opts, void* workspace,
                size_t workspace_bytes, void* stream, double* rel_res, spalu_solve_info* info);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): spalu_solve with its
 * working memory in a static device buffer of the library instead of a
 * caller workspace.  The buffer holds 64 MiB on each device the library runs
 * on and is kept until the process ends; a solve whose working memory
 * (spalu_solve_workspace) exceeds it fails with SPALU_ENOMEM.  The call
 * allocates no device memory and launches directly (opts->graph is
 * ignored); nothing in the buffer needs to start at zero, and it keeps the
 * last call's contents.  Every call on one device shares that device's
 * buffer: calls that overlap on one GPU (concurrent streams or threads)
 * race and must be serialised by the caller.  Arguments, results and
 * errors otherwise as spalu_solve. */
int spalu_solve_static(const spalu_factor_t* f, int32_t nrhs, const double* B, int64_t ldb, double* X,
                       int64_t ldx, const spalu_solve_opts* opts, void* stream, double* rel_res,
                       spalu_solve_info* info);

/* ---------------------------------------------------------------------------
 * Rank predictor training (FP32 HIP kernels).  Parameters (device floats):
 * mu[12], sd[12] (input standardisation, never trained), W1[64x12], b1[64],
 * W2[64x64], b2[64], w3[64], b3[1]; the network is relu(W1 xn + b1) ->
 * relu(W2 . + b2) -> sigmoid(w3 . + b3) predicting the rank fraction k/n of a
 * segment from its 12 features; the loss is the mean squared error.
 * ------------------------------------------------------------------------- */
int spalu_mlp_param_count(void);

/* Device workspace bytes for a batch of the given size. */
int spalu_mlp_workspace(int32_t batch, size_t* bytes);

/* y[b] = network output for feature rows X (batch x 12); all device. */
int spalu_mlp_forward(const float* params, const float* X, int32_t batch, float* y, void* workspace,
                      size_t workspace_bytes, void* stream);

/* One step on the batch (X batch x 12, targets t): loss (device float[1])
 * = mean squared error before the update; grad (device, param_count floats,
 * may be NULL) receives the gradient (zero for mu, sd); if adam_m / adam_v
 * (device, param_count floats, zero-initialised by the caller) are given,
 * one Adam update (beta 0.9, 0.999, eps 1e-8, bias-corrected with step >= 1)
 * with learning rate lr is applied to the trainable entries. */
int spalu_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* X, const float* t,
                         int32_t batch, float lr, int32_t step, float* loss, float* grad, void* workspace,
                         size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Profiling (process-wide, not thread-safe; for benchmarks).  While on, every
 * kernel launch of spalu_factor / spalu_solve is bracketed by HIP events on
 * the launch stream; at the end of each call the elapsed times are summed
 * per kernel together with the launch's algorithmic bytes and flops (what
 * the step must move and compute given the actual segment sizes, excluding
 * padding and staging).  spalu_profile(on) also clears the totals.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;       /* summed event time */
  double bytes;    /* summed algorithmic HBM bytes */
  double flops;    /* summed algorithmic flops */
} spalu_kernel_stat;

void spalu_profile(int32_t on);

/* Restricts the event timing of spalu_profile to the launches of one kernel
 * step (a name as spalu_profile_read reports it), so that a timed region
 * carries the events of that step only; NULL or "" times every step again
 * (so does spalu_profile).  Returns SPALU_EINVAL for an unknown name. */
int spalu_profile_only(const char* name);

/* Copies up to max per-kernel totals into out (host); *count = kernels with
 * at least one launch.  out may be NULL to query the count. */
int spalu_profile_read(spalu_kernel_stat* out, int32_t max, int32_t* count);

const char* spalu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPALU_H */
