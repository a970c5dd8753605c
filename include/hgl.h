/*
 * hgl -- hypergraph ranking solves on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  It computes, for a hypergraph with binary incidence
 * H (N vertices x E hyperedges) and hyperedge weights w, the normalised
 * adjacency A = Dv^-1/2 H W De^-1 H' Dv^-1/2 (paper, section 2, eq. 1),
 * Zhou's Laplacian L = I - A, and solves
 *
 *        M F = Y,   M = I + L / lambda,
 *
 * for many columns of Y.  With theta = lambda this is the paper's ranking
 * system X f = theta/(1+theta) y (eq. 6), X = I - A/(1+theta), and F equals
 * f* of eq. (3) column by column.
 *
 * Conventions (all entry points):
 *  - every array argument is a DEVICE pointer owned by the caller unless its
 *    name ends in _host (host memory, owned by the caller);
 *  - dense matrices are row-major, n_rows x k, with a leading dimension
 *    ld >= k counted in elements; row r starts at ptr + r*ld;
 *  - integer index arrays are int32;
 *  - every call is ordered on the given HIP stream; calls that fill _host
 *    outputs synchronise that stream before returning, the others return
 *    as soon as the work is enqueued;
 *  - the return value is a status: 0 = HGL_OK, positive = informational,
 *    negative = error; hgl_last_error() gives a message for the last failing
 *    call on the calling thread; no C++ exception crosses this boundary;
 *  - a handle owns its device buffers and frees them in hgl_destroy; it
 *    takes every one of them (structure, scales, workspaces and the
 *    temporaries of its own build) from the allocator given at build
 *    (hgl_allocator, e.g. the caller's framework's caching allocator), or
 *    from hipMalloc when none is given; a handle must not be used from two
 *    threads at once.  The one exception is hgl_apply_noalloc, which
 *    allocates nothing.
 */
#ifndef HGL_H
#define HGL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hgl_handle hgl_handle;

/*
 * Caller-supplied device memory for a handle.  alloc returns `bytes` of
 * device memory on the current device, usable by work on `stream` (the
 * stream of the library call that asks), or NULL on failure (the call then
 * returns HGL_ENOMEM).  free returns a pointer that alloc gave; `stream` is
 * the stream of the call that frees it (for hgl_destroy, that of the
 * handle's last call; work queued before it may still read the memory, so
 * a stream-ordered allocator must not hand it out to other streams before
 * that work ends).  ctx is passed through and must stay valid until
 * hgl_destroy returns.  A handle's calls should use one stream, or the
 * caller orders them across streams.
 */
typedef struct hgl_allocator {
  void* (*alloc)(size_t bytes, void* ctx, hipStream_t stream);
  void (*free)(void* ptr, void* ctx, hipStream_t stream);
  void* ctx;
} hgl_allocator;

enum hgl_status {
  HGL_OK = 0,
  HGL_NOT_CONVERGED = 1,  /* iteration limit hit; outputs hold the last iterate */
  HGL_EINVAL = -1,        /* invalid argument or hypergraph structure */
  HGL_ENOMEM = -2,        /* device allocation failed */
  HGL_EDEVICE = -3,       /* HIP runtime error (message carries its text) */
  HGL_EBREAKDOWN = -4,    /* CG breakdown: p'Mp <= 0 or not finite */
  HGL_ECHOLQR = -5,       /* Cholesky of a Gram matrix failed in CholQR */
  HGL_EUNSUPPORTED = -6   /* valid request this build does not handle */
};

enum hgl_dtype { HGL_F64 = 0, HGL_F32 = 1 };

enum hgl_cg_mode {
  /* every vector, product and inner product in FP64 */
  HGL_CG_PLAIN_F64 = 0,
  /* vectors and operator products in FP32; inner products accumulated in
     FP64; the residual is recomputed as Y - M F with FP64 accumulation every
     rr_period iterations and whenever a column's recursive residual claims
     convergence (residual replacement); a column stops only on that
     recomputed FP64 residual */
  HGL_CG_F32_F64DOT_RR = 1
};

typedef struct hgl_cg_opts {
  int32_t mode;       /* enum hgl_cg_mode */
  double tol;         /* per-column target ||y_j - M f_j|| / ||y_j|| */
  int32_t max_iter;   /* iteration limit (>= 1) */
  int32_t x0_given;   /* 1: F holds the starting guess on entry; 0: start from 0 */
  int32_t rr_period;  /* residual replacement period (F32 mode); 0 = only on claims */
  int32_t chunk;      /* iterations enqueued between host convergence checks; 0 = automatic:
                         each chunk is sized from the convergence rate to reach the claim level
                         and is followed at once by an FP64 residual check */
  int32_t graph;      /* 1: the first chunk of iterations runs as a HIP graph, captured on
                         first use and replayed by later solves on the handle with the same
                         arguments (pointers, sizes, options); 0: direct launches.  Ignored
                         while kernel timing (hgl_profile) is on. */
  int32_t tune;       /* 1: the column shapes of the two operator gathers (lanes per row,
                         vector width, column slabs) are picked by timing each gather on
                         first use for this k and element size and cached in the handle (a
                         one-time cost of a few milliseconds; the grouping of the FP64
                         partial sums follows the shape, so results can differ at rounding
                         level from tune = 0); 0: the widest-vector shape */
} hgl_cg_opts;

/* Library version, e.g. 100 for 0.1.0. */
int hgl_version(void);

/* Message for the last failing call on this thread ("" if none). */
const char* hgl_last_error(void);

/*
 * Build the operator for one hypergraph (paper, section 2).
 *  edge_ptr [E+1], edge_vtx [nnz]: edge-major CSR of H.  Hyperedge e is the
 *    vertex set edge_vtx[edge_ptr[e] .. edge_ptr[e+1]-1]; its ids must be
 *    strictly increasing (H is binary, so a repeated vertex is invalid), lie
 *    in [0, N), and every hyperedge must be nonempty.
 *  w [E]: hyperedge weights, finite and >= 0 (L does not change when w is
 *    scaled, so w need not sum to one).
 * Computes delta(v) = sum_e w(e) H(v,e), delta(e) = |e|, the scales
 * s_v = delta(v)^-1/2 (0 when delta(v) = 0, i.e. the pseudo-inverse) and
 * c_e = w_e / delta(e), and the vertex-major transpose of H.  The inputs are
 * copied; the caller may free them afterwards.  al (nullable): where the
 * handle takes its device memory from (copied; NULL: hipMalloc / hipFree).
 * Invalid structure or weights -> HGL_EINVAL (validation runs on the device;
 * this call synchronises); a failed allocation -> HGL_ENOMEM.
 */
int hgl_build_laplacian(int32_t N, int32_t E, int64_t nnz, const int32_t* edge_ptr,
                        const int32_t* edge_vtx, const double* w, const hgl_allocator* al,
                        hgl_handle** out, hipStream_t stream);

/*
 * Build one operator for G independent hypergraphs stored as their disjoint
 * union (vertex ids global): section 2's operator of each graph, with the
 * paper's per-query independence (section 4, one solve per test image) kept
 * per (graph, column).  vtx_offsets_host[G+1] and edge_offsets_host[G+1]
 * give each graph's vertex and hyperedge ranges; every hyperedge of graph g
 * must lie inside graph g's vertex range.  Solves on such a handle run one
 * CG recurrence per (graph, column) and may use one lambda per graph.  al:
 * as for hgl_build_laplacian.
 */
int hgl_build_laplacian_batched(int32_t G, const int32_t* vtx_offsets_host,
                                const int32_t* edge_offsets_host, int64_t nnz,
                                const int32_t* edge_ptr, const int32_t* edge_vtx,
                                const double* w, const hgl_allocator* al, hgl_handle** out,
                                hipStream_t stream);

/* Replace the weights w [E] (same rules as at build) and recompute delta(v),
 * s and c of eq. 1; the structure is reused.  This is the re-weighting step
 * of the paper's alternating scheme (section 2: w is updated with F fixed,
 * then F is solved again with the new w).  -> HGL_EINVAL on a negative or
 * non-finite weight (synchronises). */
int hgl_set_weights(hgl_handle* h, const double* w, hipStream_t stream);

/* Release the handle and its device buffers (NULL is accepted). */
void hgl_destroy(hgl_handle* h);

/* Sizes of a handle: N, E, nnz, number of graphs (any pointer may be NULL). */
int hgl_get_sizes(const hgl_handle* h, int32_t* N, int32_t* E, int64_t* nnz, int32_t* G);

/*
 * Work partition of the operator gathers (diagnostics; any pointer may be
 * NULL): row tiles of the vertex gather, hub vertex rows (split into chunks
 * and finished by a separate launch) with their chunk count, and hyperedges
 * large enough to take a whole workgroup in the edge gather.
 */
int hgl_get_partition(const hgl_handle* h, int32_t* n_tiles, int32_t* n_hub_rows, int32_t* n_hub_chunks,
                      int32_t* n_long_edges);

/*
 * Diagnostics: the column shapes under which the two operator gathers of the
 * most recent CG solve on this handle ran, written to the caller's host array
 * shape6 = {lanes per row, elements per lane, column slabs} of the edge
 * gather, then the same of the vertex gather; all zero before the first
 * solve.  With the autotuner on (hgl_cg_opts.tune) they are the tuned shapes.
 * Errors: HGL_EINVAL for a NULL argument.
 */
int hgl_get_gather_shape(const hgl_handle* h, int32_t* shape6);

/*
 * Diagnostics of the most recent CG solve on this handle (hgl_cg_solve,
 * hgl_cg_solve_batched, and the refinement of hgl_block_rsvd_invert),
 * written to the caller's host array stats4 = {iterations enqueued, chunks
 * of iterations enqueued between host synchronisations, check steps
 * (FP64-recomputed residuals deciding claimed columns), check steps after
 * which some column went on iterating}; all zero before the first solve.
 * Errors: HGL_EINVAL for a NULL argument.
 */
int hgl_get_cg_stats(const hgl_handle* h, int32_t* stats4);

/*
 * Copy the derived quantities of section 2 into caller buffers (any may be
 * NULL): dv [N] = delta(v), s [N] = delta(v)^-1/2 (0 if delta(v) = 0),
 * c [E] = w_e/delta(e), vtx_ptr [N+1] and vtx_edge [nnz] = vertex-major CSR
 * of H, each vertex's hyperedges in increasing id order.
 */
int hgl_get_operator(const hgl_handle* h, double* dv, double* s, double* c, int32_t* vtx_ptr,
                     int32_t* vtx_edge, hipStream_t stream);

/*
 * Q = (I + L/lambda) P for k columns, computed matrix-free as
 * Q = (1 + 1/lambda) P - (1/lambda) S H C H' S P with S = diag(s),
 * C = diag(c) (eq. 1 and the definition of L).  P and Q are N x k, of type
 * dt (double or float), leading dimensions ldp, ldq >= k; P and Q must not
 * overlap.  lambda > 0.  On a batched handle every graph uses this lambda.
 */
int hgl_apply(hgl_handle* h, double lambda, int32_t dt, const void* P, int64_t ldp, void* Q,
              int64_t ldq, int32_t k, hipStream_t stream);

/*
 * hgl_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, operator and kernels as hgl_apply, and the same Q.  Every
 * intermediate buffer (Z = C H' S P, E x k; the hub rows' chunk partials; the
 * per-graph factors) lives in one fixed device array of the library, 64 MiB
 * per GPU, held until the process ends; a call whose intermediates exceed it
 * (about E * k * sizeof(element) plus the hub partials) returns
 * HGL_EUNSUPPORTED and launches nothing.  The call allocates nothing: no
 * hipMalloc, no pinned staging, no timing events (kernel timing is skipped
 * for it).  The array is shared by every call on a GPU and keeps the last
 * call's contents, so calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  The current device must
 * be the handle's (HGL_EINVAL otherwise).
 */
int hgl_apply_noalloc(hgl_handle* h, double lambda, int32_t dt, const void* P, int64_t ldp, void* Q,
                      int64_t ldq, int32_t k, hipStream_t stream);

/*
 * Solve (I + L/lambda) F = Y column by column by conjugate gradient, in the
 * recurrences of the paper's section 3 (eqs. 16-20), each column with its own
 * alpha and beta (p'Mp obtained as (1 + 1/lambda) p'p - (1/lambda)
 * sum_e c_e |(H' S p)_e|^2, eq. 1, so that the update runs inside the
 * operator product).  A column whose recursive residual reaches the claim
 * level stops until an FP64 residual check: it finishes if the recomputed
 * residual meets tol, and otherwise restarts its search direction from it.
 * A column still iterating when its residual is recomputed (at a check, or
 * every rr_period iterations) goes on from the recomputed residual; it keeps
 * its search direction while that residual's norm is at most 1.1 times the
 * recursive one's, and restarts the direction from it otherwise (a direction
 * scaled to a drifted recursive residual makes the step overshoot).
 * Rows with delta(v) = 0 (no hyperedge of positive weight) are decoupled:
 * their equation is F_v = Y_v lambda/(1 + lambda), set at the start, and
 * the iteration skips them (a given start is overwritten there).
 * Y, F: N x k of type double (PLAIN_F64) or float
 * (F32_F64DOT_RR).  iters_host [G*k] (nullable) receives the iteration count
 * of each (graph, column), relres_host [G*k] (nullable) the FP64-recomputed
 * ||y - M f|| / ||y|| of the returned F (0 for a zero column, whose solution
 * is 0).  Returns HGL_OK when every column met tol, HGL_NOT_CONVERGED when
 * max_iter was reached first, HGL_EBREAKDOWN on a breakdown, HGL_EINVAL for
 * lambda <= 0, tol <= 0, k < 1 or a bad pointer/leading dimension.
 * Synchronises the stream.
 */
int hgl_cg_solve(hgl_handle* h, double lambda, const hgl_cg_opts* opts, const void* Y,
                 int64_t ldy, void* F, int64_t ldf, int32_t k, int32_t* iters_host,
                 double* relres_host, hipStream_t stream);

/* As hgl_cg_solve (section 3, eqs. 16-20) with one lambda per graph of a
 * batched handle (lambdas_host [G]): each (graph, column) pair is its own
 * recurrence, the paper's independent per-query solves (section 4) run
 * together.  All graphs share k; Y and F are the row concatenations of the
 * graphs' blocks (sum N_g x k). */
int hgl_cg_solve_batched(hgl_handle* h, const double* lambdas_host, const hgl_cg_opts* opts,
                         const void* Y, int64_t ldy, void* F, int64_t ldf, int32_t k,
                         int32_t* iters_host, double* relres_host, hipStream_t stream);

/*
 * The latency path for small hypergraphs (paper, section 4: one query vector
 * per test image on a graph of a few thousand vertices, solved by CG,
 * eqs. 16-20).  Solves (I + L/lambda) F = Y like hgl_cg_solve in the
 * HGL_CG_F32_F64DOT_RR mode, but each column is one workgroup that runs its
 * whole solve in a single launch (one launch for all k columns; columns are
 * independent, so many queries run side by side).
 *  Y, F: device, N x k FP32 row-major with leading dimensions ldy, ldf >= k.
 *    F holds the starting guess on entry when opts->x0_given, and the result
 *    on exit.
 *  opts: mode must be HGL_CG_F32_F64DOT_RR; tol, max_iter and x0_given as in
 *    hgl_cg_solve; rr_period, chunk, graph and tune are ignored.  A column's
 *    recursive residual that reaches tol/2 triggers a recomputation of
 *    Y - M F with FP64 accumulation; the column finishes when that meets tol
 *    and otherwise restarts from it.  An all-zero column gives F = 0 and
 *    relres 0 after 0 iterations.
 *  iters_host [k], relres_host [k] (nullable, host): iterations and the
 *    FP64-recomputed relative residual per column.
 * On a batched handle every (graph, column) pair is one workgroup (one
 * lambda for all graphs here; hgl_cg_solve_wg_batched takes one per graph),
 * and iters_host, relres_host are [G k], graph-major.
 * Limits per graph (the paper's query graphs are well inside them):
 * N <= 6144 and E <= 6144, at most 32,768 incidences (each of the 1024
 * threads holds at most 32 of each of the two CSRs of H), and
 * 8 (N + E + N' + 1024) + 4 N bytes of LDS at most 159 KB (N': vertices with
 * at least one hyperedge); beyond them, and for the FP64 mode,
 * HGL_EUNSUPPORTED.  The first call on a handle builds and keeps the
 * per-thread tables (about 180 KB of device memory per graph; synchronises).  Returns
 * HGL_OK, HGL_NOT_CONVERGED (a column reached max_iter), HGL_EBREAKDOWN
 * (p'Mp <= 0 or not finite, e.g. NaN input) or HGL_EINVAL (bad arguments).
 * Synchronises the stream.
 */
int hgl_cg_solve_wg(hgl_handle* h, double lambda, const hgl_cg_opts* opts, const float* Y, int64_t ldy,
                    float* F, int64_t ldf, int32_t k, int32_t* iters_host, double* relres_host,
                    hipStream_t stream);

/* As hgl_cg_solve_wg (section 3, eqs. 16-20, one solve per query as in
 * section 4) with one lambda per graph of a batched handle (lambdas_host
 * [G]); Y and F are the row concatenations of the graphs' blocks
 * (sum N_g x k), as for hgl_cg_solve_batched. */
int hgl_cg_solve_wg_batched(hgl_handle* h, const double* lambdas_host, const hgl_cg_opts* opts,
                            const float* Y, int64_t ldy, float* F, int64_t ldf, int32_t k,
                            int32_t* iters_host, double* relres_host, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Block randomized SVD (paper, section 3: Algorithm 1, the tessellation of
 * eq. 11 and the block inverse of eq. 15).
 *
 * The vertices are tessellated into n_blocks contiguous ranges given by
 * block_offsets_host[n_blocks+1] (0 = o_0 < o_1 < ... < o_n = N).  For each
 * diagonal block A_bb of the normalised adjacency A (eq. 1) the library runs
 * Algorithm 1: Y = A_bb Omega, S = orth(Y), then q times
 * { S~ = orth(A_bb' S), S = orth(A_bb S~) }, B = S' A_bb, B = U~ Sigma V',
 * U = S U~, keeping the k leading singular triplets.  orth() is CholQR
 * (Gram matrices and their Cholesky factors in FP64): two passes for the
 * basis of the last step and throughout an FP64 sketch, one pass between the
 * products of a BF16 sketch.  The small symmetric eigenproblem of B B' is
 * solved in FP32 for a BF16 sketch (Householder tridiagonalisation,
 * multisection on Sturm counts, inverse iteration with Gram-Schmidt within
 * clusters of close eigenvalues) and by FP64 parallel cyclic Jacobi for an
 * FP64 sketch.  The diagonal blocks of
 * X = I - A/(1+theta) are full rank, so the low-rank object decomposed is
 * A_bb; eq. (15) is applied as the identity-plus-low-rank inverse
 *   (I + L_bb/lambda)^-1 ~ lambda/(1+lambda) [I + U diag(s/(1+lambda-s)) U'].
 * ------------------------------------------------------------------------ */

enum hgl_sketch {
  HGL_SKETCH_BF16 = 0,  /* A_bb, Omega and S in BF16; MFMA products accumulate in FP32 */
  HGL_SKETCH_F64 = 1    /* every product in FP64 (reference precision) */
};

/* How the basis S is formed (paper, section 3, eq. 10 and Algorithm 1). */
enum hgl_rsvd_scheme {
  HGL_RSVD_SUBSPACE = 0, /* Algorithm 1: orth() after every product (default) */
  HGL_RSVD_POWER = 1     /* eq. 10: Y = (A_bb A_bb')^q A_bb Omega by 2q+1
                            products with nothing in between (the next
                            product's operand is Y itself, rounded to the
                            sketch's operand format), then one two-pass orth().
                            Fewer launches; the paper warns it is more
                            sensitive to rounding, and with a fast-decaying
                            spectrum the directions of small singular values
                            are lost as q grows.  The final CholQR then sees
                            an ill-conditioned Gram matrix and may need its
                            shifted retry, or fail with HGL_ECHOLQR. */
};

typedef struct hgl_rsvd_opts {
  int32_t k;          /* rank kept per block (>= 1) */
  int32_t p;          /* oversampling: sketch width l = k + p (l <= 96) */
  int32_t q;          /* subspace iterations (>= 0) */
  int32_t sketch;     /* enum hgl_sketch */
  uint64_t seed;      /* Philox4x32-10 key when omega is NULL */
  double refine_tol;  /* hgl_block_rsvd_invert: target relres of the refinement */
  int32_t max_refine; /* hgl_block_rsvd_invert: preconditioned CG iteration limit */
  int32_t chunk;      /* as hgl_cg_opts.chunk */
  int32_t scheme;     /* enum hgl_rsvd_scheme (0: Algorithm 1) */
} hgl_rsvd_opts;

/*
 * Algorithm 1 on every diagonal block.  omega_bf16 (nullable, device):
 * N x l row-major BF16 bit patterns, row v is the sketch row of vertex v
 * (rows of block b are its rows o_b .. o_{b+1}-1); NULL draws standard
 * normals from Philox4x32-10 keyed by opts->seed (see hgl_sketch_gaussian).
 * U_out (device, N x k FP32 row-major): rows of block b hold U_b.
 * sigma_out (nullable, device, n_blocks x k FP64): singular values of B per
 * block, decreasing.  Every block needs at least l rows.  Errors: HGL_EINVAL
 * (bad offsets, l > 96, a block smaller than l, batched handle),
 * HGL_ECHOLQR (a Gram matrix not positive definite even after the shift).
 * Synchronises the stream.
 */
int hgl_block_rsvd(hgl_handle* h, int32_t n_blocks, const int32_t* block_offsets_host,
                   const hgl_rsvd_opts* opts, const uint16_t* omega_bf16, float* U_out,
                   double* sigma_out, hipStream_t stream);

/*
 * Solve (I + L/lambda) F = Y (Y, F: N x nrhs FP32) with the block inverse
 * built from hgl_block_rsvd (eq. 15 in its identity-plus-low-rank form,
 * M_bb^-1 ~ lambda/(1+lambda) [I + U diag(sigma/(1+lambda-sigma)) U'], on the
 * tessellation of eq. 11): F0 = blockdiag(M_bb^-1) Y, refined by
 * preconditioned CG (FP32 vectors, FP64 inner products, residual
 * replacement) until the FP64-recomputed relres of every column is at most
 * opts->refine_tol.  iters_host [nrhs], relres_host [nrhs], sigma_out
 * [n_blocks*k] (device) are nullable.  Returns as hgl_cg_solve.
 */
int hgl_block_rsvd_invert(hgl_handle* h, double lambda, int32_t n_blocks,
                          const int32_t* block_offsets_host, const hgl_rsvd_opts* opts,
                          const uint16_t* omega_bf16, const float* Y, int64_t ldy, float* F,
                          int64_t ldf, int32_t nrhs, double* sigma_out, int32_t* iters_host,
                          double* relres_host, hipStream_t stream);

/*
 * rows x l standard normals, row-major, rounded to BF16 (bit patterns):
 * element i (= row*l + col) is normal number i of the stream where counter
 * c = i/2 of Philox4x32-10 (Salmon et al., SC'11; key = seed, counter =
 * (c low 32 bits, c high 32 bits, 0, 0)) gives the words (x0, x1, x2, x3)
 * and the Box-Muller pair from u1 = (x0 + 1)/2^32, u2 = x1/2^32 is
 * (sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2)).
 */
int hgl_sketch_gaussian(int64_t rows, int32_t l, uint64_t seed, uint16_t* out_bf16, hipStream_t stream);

/*
 * The generator under hgl_sketch_gaussian (Algorithm 1 step 1 draws the
 * Gaussian test matrix from it): Philox4x32-10 (Salmon et al., SC'11) on
 * caller counters, for bit-exact checks of its integer words.  ctr, out:
 * device uint32 arrays [n][4]; key = (key low 32 bits, key high 32 bits);
 * out[i] = the four output words of counter ctr[i].  Asynchronous.
 */
int hgl_philox4x32_10(int64_t n, const uint32_t* ctr, uint64_t key, uint32_t* out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Block inverse through Schur complements (paper, section 3, eqs. 12-14)
 * under nested tessellation, eq. 15 at the smallest submatrices.
 *
 * Every diagonal block M_bb = (I + L/lambda)[o_b, o_b+1) of n rows is
 * split into 2x2 blocks with floor(n/2) rows in the first, recursively
 * while both halves keep at least min_block rows.  A split block's inverse
 * is [[Z1^-1, -X11^-1 X12 Z2^-1], [-Z2^-1 X21 X11^-1, Z2^-1]] with
 * Z1 = X11 - X12 X22^-1 X21 (eq. 13), Z2 = X22 - X21 X11^-1 X12 (eq. 14),
 * and the four inverses X11^-1, X22^-1, Z1^-1, Z2^-1 are the same
 * construction one level down.  The smallest submatrices (min_block to
 * 2 min_block - 1 rows; the paper takes 50, and 500 on the second update)
 * are inverted exactly (eq. 15 with all singular values gives the same
 * matrix): those of at most 127 rows by Gauss-Jordan elimination, larger
 * ones by the same 2 x 2 construction carried on down to such pieces, in
 * FP32 like the products, which run on MFMA.  So the result is M_bb^-1 up
 * to FP32 rounding for every min_block.
 *
 * Limits: single-graph handle; 16 <= min_block <= 4096; every block 1 to
 * 4096 rows, offsets covering [0, N).  Errors: HGL_EINVAL (arguments),
 * HGL_EDEVICE.
 * ------------------------------------------------------------------------ */

/*
 * The inverse of every diagonal block by eqs. 12-14 under nested
 * tessellation (as above).  inv_out (device, nullable): the
 * blocks' inverses packed in block order, block b as n_b x n_b FP32
 * row-major at element offset sum_{c<b} n_c^2.  flops_out (host, nullable):
 * the algorithmic flops of the products (2 m n k each).  The workspace
 * (about 12 sum n_b^2 floats) and the plan stay in the handle and are
 * reused while the blocks and min_block are unchanged.  Synchronises the
 * stream.
 */
int hgl_block_schur_inverse(hgl_handle* h, double lambda, int32_t n_blocks, const int32_t* block_offsets_host,
                            int32_t min_block, float* inv_out, double* flops_out, hipStream_t stream);

/*
 * Solve (I + L/lambda) F = Y (Y, F: N x nrhs FP32, device, row-major) with
 * the block inverse of eqs. 12-14 as the preconditioner: F0 =
 * blockdiag(M_bb^-1) Y, then
 * preconditioned CG (FP32 vectors, FP64 inner products, residual
 * replacement) until every column's FP64-recomputed relres is at most
 * refine_tol or max_refine iterations ran.  chunk as hgl_cg_opts.chunk.
 * iters_host, relres_host [nrhs] nullable.  Returns as hgl_cg_solve.
 */
int hgl_block_schur_invert(hgl_handle* h, double lambda, int32_t n_blocks, const int32_t* block_offsets_host,
                           int32_t min_block, double refine_tol, int32_t max_refine, int32_t chunk,
                           const float* Y, int64_t ldy, float* F, int64_t ldf, int32_t nrhs, int32_t* iters_host,
                           double* relres_host, hipStream_t stream);

/*
 * The execution plan of hgl_block_schur_inverse (the products and leaves of
 * eqs. 12-14, phase by phase), host only (no device call),
 * for inspection.  counts7: {products, leaves, phases, workspace elements,
 * inverse elements, product tiles, flops}.  Optional outputs (host, sized
 * from counts7 by a first call with NULLs):
 *   tasks  [products x 13]: a, b, c, d (element offsets into the workspace),
 *          lda, ldb, ldc, ldd, m, n, k, alpha, beta of D = alpha A B + beta C;
 *   leaves [leaves x 5]: in, out, ldi, ldo, n (out = inverse of in);
 *   phases [phases x 5]: first tile, tiles, first leaf, leaves, largest leaf;
 *   tiles  [tiles x 2]: product, (tile row << 16) | tile column (64 x 64);
 *                       in XCD order, product -1 for an empty slot;
 *   moff   [n_blocks]: workspace offset of M_bb (n_b x n_b row-major).
 * Block b's inverse sits at offset sum_{c<b} n_c^2 (ld n_b).  Within a
 * phase the leaves and products are independent; phases run in order.
 */
int hgl_block_schur_plan(int32_t n_blocks, const int32_t* block_offsets_host, int32_t min_block, int64_t* counts7,
                         int64_t* tasks, int64_t* leaves, int32_t* phases, int64_t* tiles, int64_t* moff);

/* ------------------------------------------------------------------------
 * Weight derivatives (paper, section 2: P(w) of eq. 4 and the steepest-descent
 * update of w; the paper defers the formula, it is derived from eq. 1).
 * For N x k matrices P, Q:
 *   Gamma_e(P,Q) = <u_e(P), u_e(Q)>/delta(e)
 *                  - 1/2 sum_{v in e} s_v^2 (<P_v, (AQ)_v> + <(AP)_v, Q_v>),
 *   u_e(P) = sum_{v in e} s_v P_v   (= <P, dA/dw_e Q>, Dv's dependence on w included).
 * ------------------------------------------------------------------------ */

/*
 * The gradient of eq. 4's P(w) through the solve of eq. 3 (section 2).
 * grad_w [E] (device, FP64) = derivative with respect to w of:
 *  - G != NULL: a loss l(F) of F = (I + L/lambda)^-1 Y with upstream
 *    G = dl/dF:  grad_w[e] = Gamma_e(Z, F)/lambda, Z = M^-1 G;
 *  - G == NULL: the adaptive-weight objective
 *    J = tr(F'LF) + lambda ||F - Y||^2 + mu ||w||^2 at the given F:
 *    grad_w[e] = -Gamma_e(F,F) + Gamma_e(Z,F)/lambda + 2 mu w_e,
 *    Z = M^-1 (2 lambda (M F - Y)) (exact total derivative even when F is
 *    an approximate solve).
 * F, G, Y, Z_out: N x k, FP32 when adj->mode is F32_F64DOT_RR, FP64 when
 * PLAIN_F64; leading dimensions ldf, ldg, ldy, ldz.  The adjoint solve uses
 * hgl_cg_solve with adj; Z_out (nullable) receives Z (= dl/dY in the G case);
 * iters_host/relres_host (nullable, [k]) report the adjoint solve.  Returns
 * HGL_NOT_CONVERGED (1) when the adjoint solve reached max_iter before every
 * column met adj->tol (grad_w is then computed from that inexact Z).
 * Single-graph handles only.  Synchronises the stream.
 */
int hgl_weight_grad(hgl_handle* h, double lambda, double mu, const void* F, int64_t ldf, const void* G,
                    int64_t ldg, const void* Y, int64_t ldy, int32_t k, const hgl_cg_opts* adj,
                    double* grad_w, void* Z_out, int64_t ldz, int32_t* iters_host, double* relres_host,
                    hipStream_t stream);

/*
 * w = argmin ||w - v||_2 subject to w >= 0, sum(w) = 1 (the constraints of
 * eq. 4): w = max(v - tau, 0) with tau chosen so that w sums to one.  v, w:
 * device FP64 arrays of length E (may alias).  Asynchronous.
 */
int hgl_project_simplex(const double* v, double* w, int32_t E, hipStream_t stream);

/*
 * One projected-gradient step of the weight update (paper, section 2: w on
 * the simplex of eq. 4, descended along the gradient of P(w)):
 *   w_out = argmin ||x - (w - eta g)||_2 over {x >= 0, sum(x) = 1}.
 * w, g: device FP64 [E] (the weights and dP/dw); w_out: device FP64 [E], not
 * aliasing w or g.  eta > 0: that fixed step; eta_dev (nullable, device
 * FP64 [1]) receives it.  eta <= 0: the step is set from this gradient,
 * eta = 0.5 max|w| / max|g - mean(g)| (0 for a constant g), computed on the
 * device and written to eta_dev (then required), so a loop can reuse it as
 * its fixed step.  The difference w - eta g is formed without contraction.
 * HGL_EINVAL for E < 1, a NULL array, a non-finite eta, aliasing, or
 * eta <= 0 without eta_dev.  Asynchronous.
 */
int hgl_projected_gradient_step(const double* w, const double* g, double eta, int32_t E, double* w_out,
                                double* eta_dev, hipStream_t stream);

/*
 * One steepest-descent step on the Lagrangian of eq. 5 (the paper's active-
 * set rule): w_out = w - mu_eff grad S.  The multipliers of the active
 * constraints (1'w = 1, and w_i = 0 for the zero weights that stay at the
 * bound) make d = -grad S the projection of -g onto {sum d = 0, d_i >= 0
 * where w_i = 0}: d_i = nu - g_i where w_i > 0, max(nu - g_i, 0) where
 * w_i = 0, nu the unique root of sum d = 0 (a zero weight with g_i >= nu
 * stays active with multiplier g_i - nu; one with g_i < nu is released).
 * mu_eff = min(mu, min over d_i < 0 of w_i / -d_i): the step stops where a
 * positive weight reaches 0, which is then set to exactly 0.
 * w (on the simplex), g: device FP64 [E]; w_out (may alias w), d_out
 * (nullable): device FP64 [E].  info_dev: device FP64 [4] = {nu, mu_eff,
 * released zero weights, active zero weights}, nu = NaN when w has no
 * positive entry.  info_host (nullable): copied there after a stream
 * synchronisation; the call then returns HGL_EINVAL for such a w.  mu > 0.
 */
int hgl_active_set_step(const double* w, const double* g, double mu, int32_t E, double* w_out, double* d_out,
                        double* info_dev, double* info_host, hipStream_t stream);

/*
 * Kernel timing (diagnostics).  hgl_profile(h, enable) resets the counters;
 * with enable = 1 every later solver call on h launches its kernels with
 * start/stop events that the runtime stamps at each kernel's own start and
 * end (hipExtLaunchKernel); with enable other than 1, bits 0..15 select the
 * kinds that carry events (bit k = kind k) and bits 16..23, when nonzero,
 * stamp only every n-th launch of each such kind, so that timing one kernel
 * perturbs the launch stream little; enable = 0 stops it.  hgl_profile_read
 * returns, for one kernel kind, the number of kernel launches recorded and
 * their summed duration in milliseconds (it synchronises the device).
 * Kinds: 0 edge gather (Z = C H' S P), 1 vertex gather with inner product
 * (M P, rows up to the hub threshold and hub-row chunks), 2 CG update (F, R),
 * 3 CG direction (P), 4 reductions, 5 residual edge gather (FP64),
 * 6 residual vertex gather (FP64), 7 start-up, 8 preconditioner, 9 rSVD
 * products, 10 CholQR, 11 the small eigenproblem, 12 block extraction, 13 weight gradient,
 * 14 hub-row finish of every vertex gather.  Kinds 0..15; others ->
 * HGL_EINVAL.
 */
int hgl_profile(hgl_handle* h, int32_t enable);
int hgl_profile_read(hgl_handle* h, int32_t kind, int64_t* launches, double* ms);

/* ------------------------------------------------------------------------
 * Measurement probes (not part of the method): the device's achievable
 * peaks, the measured denominators of the roofline fractions.
 * ------------------------------------------------------------------------ */

/* Copy `bytes` (a positive multiple of 16; src, dst 16-byte aligned device
 * buffers that do not overlap) with a 16-bytes-per-lane grid-stride kernel.
 * Moves 2 * bytes through HBM when both buffers exceed the last-level cache.
 * Asynchronous. */
int hgl_peak_copy(const void* src, void* dst, int64_t bytes, hipStream_t stream);

/* `workgroups` workgroups of 4 waves; every wave runs `iters` rounds of eight
 * independent v_mfma_f32_16x16x32_bf16 on register operands (16,384 flops
 * each): 524,288 * workgroups * iters flops in all.  out (device,
 * `workgroups` floats) is written only if a sum reaches a sentinel it does
 * not reach.  Asynchronous. */
int hgl_peak_mfma_bf16(float* out, int32_t workgroups, int32_t iters, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HGL_H */
