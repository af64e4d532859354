/*
 * pslr.h -- C ABI of the PSLR (Power Schur complement Low-Rank) preconditioner
 * for one AMD MI355X (gfx950).
 *
 * Method: Q. Zheng, Y. Xi, Y. Saad, "A power Schur complement low-rank
 * correction preconditioner for general sparse linear systems",
 * arXiv 2002.00917.  Notation of the paper throughout:
 *
 *   After a reordering by subdomains (Sec. 2, eq. resystem)
 *       A = [ B  E ]   B, E block diagonal (s subdomains),
 *           [ F  C ]   F shaped like E^T,
 *   S = C - F B^{-1} E (eq. solve), C0 = blkdiag(C_i), E_s = C0 - S,
 *   C_g = C - C0 (Sec. 3.1, eq. matrixS),
 *   P_m = sum_{i=0..m} (C0^{-1} E_s)^i C0^{-1}        (eq. approx1),
 *   E_rr(m) = I - S P_m = (E_s C0^{-1})^{m+1}         (eqs. err1, err; Thm. t2),
 *   r_k-step Arnoldi on E_rr(m): E_rr ~ V H V^T       (eq. schur),
 *   G = (I - H)^{-1} - I, S_app^{-1} = P_m (I + V G V^T)  (eqs. Sinv0, Sinv).
 *
 * Local factors are exact sparse LU factorisations of every B_i and C_i by
 * default (the closed forms above then hold to rounding), or the paper's
 * threshold incomplete LU (Algorithm 4, drop tolerance 1e-2 in Sec. 4).
 *
 * Conventions shared by every entry point
 *   - Every call returns a pslr_status and never aborts; pslr_last_error()
 *     gives a thread-local message for the last failure.
 *   - Host arrays (CSR matrix, labels, options) are read during the call only;
 *     the caller keeps ownership.
 *   - Device vectors (b, z, x, lambda, grad) are caller-owned device pointers
 *     (e.g. torch tensors' data_ptr()), column-major n x nrhs with a leading
 *     dimension; they must not alias and must stay alive until the work on the
 *     given HIP stream has completed (calls are asynchronous unless stated).
 *   - Vectors cross the boundary in the ORIGINAL ordering of A and in FP64 in
 *     both precision modes; the library permutes and casts internally.
 *   - A handle owns every device buffer it allocates; it holds one workspace,
 *     so concurrent calls on one handle from different streams race.
 *   - hip_stream may be NULL (the default stream).
 *   - The triangular solves combine partial sums with atomic adds, so two
 *     applies of the same vector can differ in the last bits (the summation
 *     order varies); every result stays within the rounding of the method.
 *   - pslr_apply and pslr_apply_transpose launch kernels only (no allocation,
 *     memset or host synchronisation once the handle's workspace for that
 *     many right-hand sides exists), so they can be captured in a HIP graph.
 *     A captured apply keeps the device buffers it was captured with.  The
 *     handle never frees a buffer a captured apply may use while it lives:
 *     a call that needs a larger workspace (more right-hand sides than any
 *     earlier call, or a larger rank after pslr_set_lowrank) allocates a new
 *     one and keeps the old one until pslr_destroy, and pslr_set_lowrank
 *     keeps the replaced V and G likewise.  A graph captured before
 *     pslr_set_lowrank therefore still runs, with the OLD low-rank term:
 *     capture it again to use the new one.  pslr_destroy frees everything.
 */
#ifndef PSLR_H
#define PSLR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pslr_ctx* pslr_handle;

typedef enum {
  PSLR_OK = 0,
  PSLR_EINVAL = 1,      /* bad argument: sizes, m < 0, rank < 0, label out of range ... */
  PSLR_ESINGULAR = 2,   /* zero pivot in some B_i or C_i, or I - H singular (eq. s1 assumption) */
  PSLR_ENOCONV = 3,     /* FGMRES did not reach tol within maxit (the paper's "F");
                           best iterate, iters and relres are still written */
  PSLR_EBREAKDOWN = 4,  /* informational: Arnoldi found an invariant subspace and the
                           rank was reduced; the preconditioner is valid */
  PSLR_ENOMEM = 5,      /* host or device allocation failed */
  PSLR_EHIP = 6,        /* a HIP runtime call failed */
  PSLR_ENOTSUP = 7      /* configuration not supported (e.g. a block too large for LDS) */
} pslr_status;

typedef struct {
  int32_t m;                /* power-series upper index: sum_{i=0..m}, i.e. m+1 terms (eq. approx1) */
  int32_t rank;             /* r_k, Arnoldi steps (eq. schur); capped at min(q, 256), the widest
                               low-rank term the kernels hold (pslr_info.rank gives the rank
                               reached); 0 disables the correction */
  int32_t precision;        /* 0: FP64 apply; 1: FP32 apply (FP32 V); 2: FP32 apply with V stored in
                               BF16 where that rounding changes one apply by at most 2.5e-2
                               relative (measured at setup and by pslr_set_lowrank; else V
                               stays in FP32, see pslr_info.v_bf16).  FGMRES and Arnoldi stay
                               FP64 in every mode */
  int32_t want_transpose;   /* nonzero: also build the layouts pslr_apply_transpose needs */
  const double* v0;         /* optional host Arnoldi start vector of length q (interface order) */
  uint64_t seed;            /* used when v0 == NULL: SplitMix64 uniform in [-0.5, 0.5) */
  double pivot_threshold;   /* tau of restricted threshold partial pivoting; <= 0 means 0.1 */
  int32_t nthreads;         /* host threads for the factorisation; 0 = hardware concurrency */
  int32_t working_vectors;  /* 0: subdomain working vectors in LDS when they fit (default);
                               1: always in a global-memory workspace */
  int32_t autotune;         /* nonzero: at the end of setup, time applies over workgroup sizes
                               {512, 1024} x chunk-count scalings {1/2, 1, 2} and keep the fastest,
                               then applies of 8 right-hand sides with tiles of at most
                               {8, 4, 2, 1} right-hand sides per workgroup and keep the
                               narrowest within 5% of the fastest */
  int32_t threads;          /* workgroup size of the subdomain kernels: 0 = 1024 (the default, or
                               the autotuner's choice), else 512 or 1024 */
  int32_t factor;           /* local factors of every B_i and C_i (Algorithm 4, lines 3-4):
                               0 = exact sparse LU (nested dissection, supernodes, threshold
                               pivoting); 1 = threshold incomplete LU in the block's own row
                               order, no pivoting (ilu() of Algorithm 4; see drop_tol) */
  double drop_tol;          /* factor = 1: an entry of row i is dropped when its modulus is below
                               drop_tol times the mean modulus of the stored entries of
                               A_block[i, :] (the L entry after division by the pivot); this
                               reproduces the fill factors of Table 1; <= 0 means 1e-2, the
                               paper's setting (Sec. 4) */
  int32_t lowrank;          /* how V and H are built (Algorithm 4, lines 6-8):
                               0 = the paper's r_k-step Arnoldi on E_rr(m) (eq. schur);
                               1 = Krylov-Schur restarting of that Arnoldi process (Stewart 2001):
                                   V spans the converged invariant subspace of E_rr(m) for its
                                   r_k eigenvalues of largest modulus (a complex pair the cut
                                   would split is dropped), H = V^T E_rr V; bases of r_k + max(r_k,
                                   16) vectors, at most 60 restarts, converged when the coupling
                                   to the rest is below 1e-9 times the smallest kept modulus;
                               2 = as 1, and while every kept eigenvalue has modulus above 1 the
                                   kept count grows (to 16 more than the Ritz values above 1, up
                                   to 256), so that all eigenvalues of E_rr(m) outside the unit
                                   circle are deflated (Sec. 3.2.2); pslr_info.rank gives the
                                   count reached, which may exceed r_k */
  int32_t team;             /* B_i and C_i solves of forward applies spread over a team of
                               workgroups per subdomain (the supernodal tree of each block cut
                               into groups of whole subtrees and the top group above them;
                               exact LU only).  Block i of a family gets t_i groups: `team`
                               times its share of the family's largest block, at least one group
                               per 2048 rows (so that each group fits one workgroup's LDS), at
                               least 1 and at most 32; all groups of all blocks form one work
                               list per launch.  0 = automatic (4 when nparts <= 128, else 2 when
                               a part has more than 2048 rows, else 1), 1 = off, 2..8 */
  int32_t team_top;         /* how the team split solves its top group: 0 = automatic (2 when
                               every block's top group has at most 1024 rows and the dense
                               inverses hold at most twice the values of the family's packed
                               factors, else 1); 1 = lower and upper solve of the packed
                               top-group factors, one workgroup per subdomain; 2 = one product
                               with the dense inverse of the top group's block of L U, spread
                               over one workgroup per 64 top rows (PSLR_EINVAL when a top
                               group has more than 1024 rows) */
  int32_t team_rhs;         /* forward applies of up to team_rhs right-hand sides take the team
                               split, one right-hand side per workgroup (wider applies keep one
                               workgroup per block and tile of right-hand sides, which reads
                               the factors once per tile): 0 = automatic (1; up to 8 when the
                               tiled path would keep its working vectors in global memory, i.e.
                               blocks too large for one workgroup's LDS), 1 .. 64 */
} pslr_options;

typedef struct {
  int64_t n, p, q;          /* p interior, q interface unknowns (eq. resystem) */
  int32_t nparts;           /* s */
  int32_t m, rank, precision;
  int64_t nnz_A, nnz_E, nnz_F, nnz_Cg;
  int64_t nnz_LU_B, nnz_LU_C0;        /* stored factor entries (incl. inverted diagonal blocks) */
  int32_t supernodes_B, supernodes_C0;
  int32_t max_levels_B, max_levels_C0; /* level-schedule depth of the triangular solves */
  double fill_lu, fill_lowrank, fill_total;  /* nnz(LU)/nnz(A), nnz(V)+nnz(G) over nnz(A) (Sec. 4) */
  int64_t apply_bytes;      /* algorithmic HBM bytes of one single-rhs apply (matrix + vectors) */
  int64_t apply_bytes_rhs;  /* vector bytes added by each further right-hand side */
  int64_t series_bytes;     /* algorithmic bytes of one power-series step launch, single rhs */
  double seconds_reorder, seconds_factor, seconds_arnoldi;
  int32_t nsys;             /* systems of a batched handle (1 otherwise) */
  int32_t global_vectors;   /* 1 when the working vectors live in global memory */
  int32_t threads;          /* workgroup size of the subdomain kernels */
  int32_t lane_shift;       /* per-level chunk counts of the solves scaled by 2^lane_shift */
  int32_t max_tile;         /* widest right-hand-side tile of one workgroup (8 unless autotuned) */
  int32_t v_bf16;           /* precision 2: 1 when V is read in BF16, 0 when the setup probe kept it
                               in FP32 */
  double bf16_probe;        /* precision 2: ||z_bf16 - z_fp32|| / ||z_fp32|| of one apply to a fixed
                               vector with V in BF16 and in FP32; BF16 is kept when <= 2.5e-2 */
  int32_t lowrank;          /* pslr_options.lowrank of the setup */
  int32_t ks_restarts;      /* lowrank 1, 2: Krylov-Schur restarts (largest over systems) */
  int64_t ks_applies;       /* lowrank 1, 2: applications of E_rr(m) to a basis column */
  double ks_residual;       /* lowrank 1, 2: largest ||coupling|| / (smallest kept modulus) */
  int32_t ritz_above_one;   /* lowrank 1, 2: kept eigenvalues of E_rr(m) of modulus above 1
                               (summed over systems) */
  int32_t mfma_min_rhs;     /* applies with at least this many right-hand sides compute the
                               low-rank products V^T Y and V (G V^T Y) on the matrix cores (BF16
                               V, FP32 accumulation, Y split in three BF16 parts); 0 = never
                               (only FP32 applies with V kept in BF16) */
  int32_t team;             /* most groups of one B_i in the team split (0: no split) */
  int32_t team_top;         /* the B_i top groups' solve: 1 packed factors, 2 dense inverse (0: no
                               split) */
  int32_t team_c;           /* most groups of one C_i in the team split (0: no split) */
  int32_t team_top_c;       /* the C_i top groups' solve, as team_top */
  int32_t team_apply;       /* solves of single-right-hand-side forward applies: 0 one workgroup
                               per block, 2 team split of the B_i and the C_i.  The split runs
                               when each of its groups (rows, level scratch, the block's
                               interface values) fits one workgroup's LDS, so it also serves
                               blocks too large for the LDS of one workgroup */
} pslr_info_t;

/* Fill *opt with defaults: m = 3, rank = 16, FP64, no transpose, seed 1, tau 0.1,
 * exact LU, the paper's Arnoldi (lowrank = 0). */
void pslr_default_options(pslr_options* opt);

/* Build the preconditioner (Algorithm 4): reorder A by the labels `part`
 * (interiors of part 0..s-1 then interfaces, Sec. 2), local factors of every
 * B_i and C_i on the host (exact sparse LU, or threshold ILU: opt->factor),
 * upload, then r_k-step Arnoldi on E_rr(m) on the device in FP64 and
 * G = (I - H)^{-1} - I on the host.
 *   n, rowptr[n+1], colind[nnz], vals[nnz]: host CSR of A, original ordering.
 *   part[n]: subdomain label of each row, in [0, nparts).
 * Vertex v is an interface vertex iff a stored entry A[v,w] or A[w,v] couples
 * it to a vertex w of another part.  Returns PSLR_EBREAKDOWN (with a valid
 * handle) when Arnoldi stopped early. */
pslr_status pslr_setup(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                       const int32_t* part, int32_t nparts, const pslr_options* opt,
                       void* hip_stream, pslr_handle* out);

/* Batched setup over nsys independent systems stored as one block-diagonal
 * matrix: system s owns rows sys_ptr[s] .. sys_ptr[s+1]-1 (sys_ptr[0] = 0,
 * sys_ptr[nsys] = n), no stored entry couples two systems, every subdomain
 * label belongs to one system and the labels of system s are smaller than
 * those of system s + 1.  Every stage of an apply then runs one launch over
 * the subdomains of all systems; each system gets its own r_k-step Arnoldi
 * basis and G (the processes run together).  fgmres_solve on such a handle
 * runs one Krylov space per (system, right-hand side) pair and reports
 * iters/relres for nsys * nrhs pairs, index r * nsys + s.  v0, when given, is
 * the concatenation of the per-system start vectors (interface order). */
pslr_status pslr_setup_batched(int64_t n, const int64_t* rowptr, const int32_t* colind,
                               const double* vals, const int32_t* part, int32_t nparts,
                               int32_t nsys, const int64_t* sys_ptr, const pslr_options* opt,
                               void* hip_stream, pslr_handle* out);

/* New values for the same sparsity pattern (vals: host, nnz entries in the
 * original CSR order of the pslr_setup call): the local factors of every B_i
 * and C_i are recomputed on the host with the setup's options (the orderings
 * and supernodes depend on the pattern only), the value-dependent device
 * arrays are replaced, and the low-rank correction is rebuilt on the device
 * with the setup's construction (lowrank 1 and 2 start Krylov-Schur from the
 * previous basis).  The reordering, partition and all structural tables are
 * kept.  For repeated solves with changing values (optimisation loops).  The
 * previous factors and workspaces are freed after the device is idle, so an
 * apply captured in a HIP graph before this call must be captured again.
 * Synchronises the device.  Returns PSLR_EBREAKDOWN like pslr_setup. */
pslr_status pslr_refactor(pslr_handle h, const double* vals, void* hip_stream);

/* z = M^{-1} b, the preconditioner of Algorithm 3 (eq. application):
 *   y = g - F B^{-1} f;  y <- y + V G V^T y;  y <- P_m y;  x = B^{-1}(f - E y).
 * b, z: device, n x nrhs column-major, leading dimensions ldb, ldz >= n. */
pslr_status pslr_apply(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* z,
                       int64_t ldz, void* hip_stream);

/* pslr_apply without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and result as pslr_apply (z = M^{-1} b,
 * forward direction only, the handle's precision).  The apply's workspace
 * (y, u0, u1, the V^T y partial sums and, when a subdomain does not fit in
 * LDS, the global working vectors) is carved from one library-owned 64 MiB
 * device array per GPU instead of the handle's workspace; the call makes no
 * hipMalloc/hipFree, memset or host synchronisation and records no trace
 * events.  Its address is resolved once per device when the first handle is
 * set up there.  A call whose workspace would exceed 64 MiB returns
 * PSLR_EINVAL and launches nothing (about 3 q nrhs doubles plus the partial
 * sums: e.g. q = 67032 allows 32 right-hand sides).  All calls on one GPU share
 * that array and every apply rewrites what it uses, so calls that overlap on
 * one GPU (other streams, other threads, other handles) race: serialise them. */
pslr_status pslr_apply_noalloc(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* z,
                               int64_t ldz, void* hip_stream);

/* z = M^{-T} b, the transpose of the operator of Algorithm 3:
 *   y = g - E^T B^{-T} f;  y <- P_m^T y;  y <- y + V G^T V^T y;  x = B^{-T}(f - F^T y).
 * Needs a handle built with want_transpose != 0 (else PSLR_EINVAL). */
pslr_status pslr_apply_transpose(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb,
                                 double* z, int64_t ldz, void* hip_stream);

/* Right-preconditioned flexible GMRES(restart) in FP64 on A x = b (or A^T x = b
 * with M^{-T} when transpose != 0), independent Krylov spaces per column.
 * x: device, in = initial guess, out = solution.  Stops a column when the
 * Givens residual estimate reaches tol * ||b||, confirms with the true FP64
 * residual and restarts if needed; at most maxit inner iterations (the paper's
 * "its" and its 500-iteration failure rule, Sec. 4).  iters[nrhs], relres[nrhs]:
 * host outputs (true relative residuals); nsys * nrhs entries on a batched
 * handle.  The device runs one iteration ahead of the host's Givens updates,
 * so a cycle that stops computes one iteration it does not use.  Synchronises
 * the stream. */
pslr_status fgmres_solve(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                         int64_t ldx, int32_t restart, int32_t maxit, double tol, int32_t transpose,
                         int32_t* iters, double* relres, void* hip_stream);

/* grad[k] = - sum_r lambda[i_k, r] * z[j_k, r] for every stored entry k of A
 * (original CSR order): the gradient of a loss of z = A^{-1} b with respect to
 * A's nonzeros, given the adjoint lambda = A^{-T} dL/dz.  Device arrays. */
pslr_status pslr_sddmm_grad(pslr_handle h, int32_t nrhs, const double* lambda, int64_t ldl,
                            const double* z, int64_t ldz, double* grad, void* hip_stream);

pslr_status pslr_info(pslr_handle h, pslr_info_t* out);

/* Phase timers of the apply.  While enabled, every apply records HIP events on
 * its stream between its kernel launches, and each power-series step launch
 * stamps events at its own start and end; pslr_trace_read waits for the
 * recorded events and returns the summed elapsed times per phase (head:
 * B^{-1} f and g - F t; lowrank: V G V^T and the C0 solve it is fused with or
 * the plain C0 solve; series: the execution time of each power-series step
 * kernel, launch gaps excluded; tail: x = B^{-1}(f - E u) and the scatter).
 * reset != 0 clears the sums. */
typedef struct {
  int64_t applies;
  int64_t series_launches;
  double ms_head, ms_lowrank, ms_series, ms_tail;
} pslr_trace_t;
pslr_status pslr_trace_enable(pslr_handle h, int32_t enable);
pslr_status pslr_trace_read(pslr_handle h, pslr_trace_t* out, int32_t reset);

/* Replace V and H (host, column-major q x k and k x k) and recompute G; k = 0
 * removes the low-rank correction.  Used to apply an externally computed
 * Arnoldi basis. */
pslr_status pslr_set_lowrank(pslr_handle h, int32_t k, const double* V, int64_t ldv,
                             const double* H, int64_t ldh);

/* Delta(m, r_k) = ||X||_F ||Z^{-1}||_F with X = E_rr(m) - V H V^T and
 * Z = I - V H V^T, the upper bound of Prop. l3 on ||S^{-1} - S_app^{-1}|| /
 * ||S^{-1}|| (Sec. 3.2.3).  ||Z^{-1}||_F comes from G in closed form
 * (Z^{-1} = I + V G V^T); ||X||_F from applications of E_rr(m) on the device
 * (FP64, blocks of 32 columns) with the subtraction of V H V^T on the host:
 * exactly over the q unit vectors when nprobe = 0 (q / 32 blocks of m + 1
 * E_s C0^{-1} products: meant for small interfaces), else as the mean of
 * ||X z||^2 over nprobe Rademacher vectors drawn by SplitMix64 from seed (an
 * unbiased estimate of ||X||_F^2).  Single-system handles.  norm_x, norm_zinv
 * may be NULL.  Synchronises the stream. */
pslr_status pslr_delta(pslr_handle h, int32_t nprobe, uint64_t seed, double* delta,
                       double* norm_x, double* norm_zinv, void* hip_stream);

/* Copy the current V (q x k) and H (k x k) to host arrays (column-major). */
pslr_status pslr_get_lowrank(pslr_handle h, int32_t* k, double* V, int64_t ldv, double* H,
                             int64_t ldh);

/* Geometric split of a box grid (x fastest): label = lexicographic index,
 * x fastest, of floor(i_d * parts[d] / dims[d]).  Host only. */
pslr_status pslr_partition_geometric(int32_t ndim, const int32_t* dims, const int32_t* parts,
                                     int32_t* label);

/* Region growing: seeds are the first nparts distinct SplitMix64(seed) mod n,
 * label l belongs to the l-th seed; multi-source FIFO BFS over the
 * symmetrised pattern, neighbours in ascending index, first visitor wins;
 * vertices no seed reaches start new regions in ascending index order.
 * *nlabels receives the label count.  Host only. */
pslr_status pslr_partition_region_growing(int64_t n, const int64_t* rowptr, const int32_t* colind,
                                          int32_t nparts, uint64_t seed, int32_t* label,
                                          int32_t* nlabels);

/* The reordering of Sec. 2 as used by pslr_setup: perm[new] = old (n entries),
 * interiors of part 0..s-1 then interfaces of part 0..s-1, ascending original
 * index inside each group.  Host only. */
pslr_status pslr_reorder(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const int32_t* part, int32_t nparts, int64_t* perm, int64_t* p,
                         int64_t* q);

/* Host-only consistency check of the setup, no GPU needed: factors every B_i
 * and C_i, then reports the largest relative factorisation residual
 * ||P Q M Q^T - L U||_F / ||M||_F and the largest relative residual of the
 * packed level-scheduled solve layouts executed on the host for a fixed
 * vector (forward, and transposed when want_transpose; levels of narrow
 * supernodes once through their entry form and once through their panels).
 * Diagnostic only: no other entry point calls it. */
pslr_status pslr_host_selfcheck(int64_t n, const int64_t* rowptr, const int32_t* colind,
                                const double* vals, const int32_t* part, int32_t nparts,
                                const pslr_options* opt, double* factor_residual,
                                double* solve_residual);

/* Host-only statistics of the local factors of every B_i and C_i that
 * pslr_setup would build with these options (no GPU needed): stored factor
 * entries and level-schedule depths as pslr_info reports them, whether every
 * packed factor passes the structural level check (each position scheduled
 * once, a supernode's rows on one level, every dependency solved strictly
 * before the row that needs it), and the two residuals of
 * pslr_host_selfcheck.  For factor = 1 the factor residual is the largest
 * |(A_block - L U)_ij| / ||A_block[i, :]||_2 over the kept pattern of L + U
 * (zero up to rounding by the definition of the incomplete factorisation). */
typedef struct {
  int64_t nnz_LU_B, nnz_LU_C0;
  int32_t max_levels_B, max_levels_C0;
  int32_t levels_valid;
  double factor_residual, solve_residual;
  int32_t team;             /* the team size of the B_i and C_i solves (0: no team split) */
  int32_t team_valid;       /* 1 when every block's team split passes its structural check */
  double team_residual;     /* largest relative difference between the team-split solve of
                               every B_i and C_i (groups applied in turn on the host, the top group
                               once by its packed factors and once by its dense inverse
                               where it has one) and its plain packed solve */
  int64_t team_lds_slots_B; /* largest LDS footprint of one team workgroup over the B_i, in
                               values of the working precision: the group's own and top rows
                               (rounded up to even) plus twice its widest level.  The
                               B_i team solves also hold the block's interface values, so a
                               split runs when (slots_B + max q_i) * value size and
                               slots_C * value size fit one workgroup's LDS */
  int64_t team_lds_slots_C; /* the same over the C_i */
  int32_t team_groups_max_B; /* most subtree groups of one B_i (t_i, see pslr_options.team) */
  int32_t team_items_B;      /* subtree groups of all B_i: the work list of one B launch */
} pslr_host_stats_t;
pslr_status pslr_host_stats(int64_t n, const int64_t* rowptr, const int32_t* colind,
                            const double* vals, const int32_t* part, int32_t nparts,
                            const pslr_options* opt, pslr_host_stats_t* out);

/* Host-only step of the deflated low-rank setup (lowrank = 1, 2), exposed
 * for checking without a GPU: for a real n x n matrix Hm (column-major,
 * leading dimension ldh), an orthonormal basis W (n x *kept, column-major,
 * leading dimension ldw >= n, room for n columns) of its invariant
 * subspace for the k eigenvalues of largest modulus (k - 1 when the cut would
 * split a complex-conjugate pair; eigenvalues whose modulus ties the last kept
 * one within a relative 1e-10 are kept too, so *kept may exceed k), and
 * Hk = W^T Hm W (*kept x *kept, leading dimension ldk >= n, room for n
 * columns).  ritz_re/ritz_im
 * (n each, may be NULL) receive all eigenvalues by decreasing modulus.  This
 * is the Krylov-Schur truncation of Stewart (2001) in its real form: the
 * complex Schur form from the shifted QR algorithm, reordered, then a real
 * basis of the leading Schur vectors. */
pslr_status pslr_host_schur_select(int32_t n, const double* Hm, int64_t ldh, int32_t k, double* W,
                                   int64_t ldw, double* Hk, int64_t ldk, double* ritz_re,
                                   double* ritz_im, int32_t* kept);

pslr_status pslr_destroy(pslr_handle h);
const char* pslr_status_string(pslr_status s);
const char* pslr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PSLR_H */
