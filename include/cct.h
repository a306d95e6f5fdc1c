/*
 * cct.h - compact-triples spin-restricted CCSDT on one MI355X (gfx950).
 *
 * The library evaluates the connected-triples residual R3 of spin-restricted,
 * non-orthogonally spin-adapted CCSDT on compactly stored T3 (only occupied
 * triples i <= j <= k are kept, each with its full v^3 virtual block), the
 * T2*W driver terms, the T3 -> T1/T2 feedback, the RCCSD parts of R1/R2, the
 * R3 post-processing, the Jacobi update with orbital-energy denominators,
 * DIIS and the correlation energy.  Equations: the paper's Appendix A
 * (T1-dressed formalism, RCCSD and RCCSDT working equations, Eq. resi-rccsdt);
 * compact contractions: Sec. "Tensor contractions for compact amplitudes";
 * post-processing: Sec. "Removing redundancies in RCC amplitudes"; Jacobi
 * update: Appendix A "Coupled-cluster theory"; DIIS: Sec. "Distributed DIIS"
 * (here on one device).
 *
 * Conventions
 *   o = number of occupied, v = number of virtual spatial orbitals, n = o + v.
 *   Every host array is FP64, C-contiguous, owned by the caller and copied in
 *   or out before the call returns:
 *     f    [n][n]            bare Fock matrix f^p_q (row p, column q)
 *     B    [naux][n][n]      density-fitting factors, B[P][p][q] == B[P][q][p];
 *                            (pq|rs) = sum_P B[P][p][q] B[P][r][s]
 *     t1   [o][v]            t_i^a
 *     t2   [o][o][v][v]      t_ij^ab, must satisfy t_ij^ab == t_ji^ba
 *     t3p  [ntri][v][v][v]   packed T3, ntri = o(o+1)(o+2)/6, triples i<=j<=k in
 *                            lexicographic order (cct_packed_index), block
 *                            (i,j,k) holds t_ijk^abc for all a,b,c
 *   The library owns its device memory (allocated at cct_create) and works on
 *   the HIP stream passed at creation (NULL = the default stream).
 *
 * Errors: every int-returning function returns CCT_OK (0) or a negative code;
 * nothing aborts.  cct_last_error() gives a message for the latest failure.
 * A context is not thread-safe: one thread per context at a time.
 */
#ifndef CCT_H
#define CCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CCT_OK = 0,
  CCT_EINVAL = -1,    /* bad argument: dimension, NULL pointer, option */
  CCT_ENOMEM = -2,    /* the memory plan does not fit the device */
  CCT_EDEVICE = -3,   /* a HIP call failed (message in cct_last_error) */
  CCT_ESTATE = -4,    /* call out of order (e.g. residual before integrals) */
  CCT_ENUMERIC = -5,  /* NaN or Inf in a residual norm or the energy */
  CCT_ENOTCONV = -6   /* cct_solve reached max_iter */
};

/* Precision of the particle-particle ladder and ring contractions (the
 * dominant O(o^3 v^5) and O(o^4 v^4) terms; in a slab also the rebuild of the
 * ladder's W panels).  Everything else (T1 dressing,
 * RCCSD parts, feedback, drivers, Fock and hole-ladder terms, post-processing,
 * update, DIIS, energy) is FP64 in every mode. */
typedef enum {
  CCT_FP64 = 0,   /* FP64 MFMA */
  CCT_FP32 = 1,   /* FP32 operands, FP32 MFMA accumulation over 128 products,
                     FP64 across those */
  CCT_BF16X3 = 2  /* split BF16 (hi + lo) operands, three BF16 MFMA products
                     (lo*lo dropped), FP32 accumulation over the whole
                     contraction, FP64 output */
} cct_precision;

/* Residual term groups of Eq. resi-rccsdt (bit mask for cct_residual). */
enum {
  CCT_TERM_D1 = 1 << 0,   /* sum_d W^{ab}_{dj} t_ik^dc                 */
  CCT_TERM_D2 = 1 << 1,   /* -sum_l W^{al}_{ij} t_lk^bc                */
  CCT_TERM_F1 = 1 << 2,   /* 1/2 sum_d F^a_d t_ijk^dbc                 */
  CCT_TERM_F2 = 1 << 3,   /* -1/2 sum_l F^l_i t_ljk^abc                */
  CCT_TERM_RA = 1 << 4,   /* 1/4 sum_ld Wbar^{la}_{di} t~_{ljk}^{dbc}    */
  CCT_TERM_RB = 1 << 5,   /* -1/2 sum_ld Wbar^{la}_{id} t_jlk^dbc      */
  CCT_TERM_RC = 1 << 6,   /* -sum_ld Wbar^{lb}_{id} t_jlk^dac          */
  CCT_TERM_HH = 1 << 7,   /* 1/2 sum_lm W^{lm}_{ij} t_lmk^abc          */
  CCT_TERM_PP = 1 << 8,   /* 1/2 sum_de W^{ab}_{de} t_ijk^dec          */
  CCT_TERM_ALL = 0x1ff
};

typedef struct cct_ctx cct_ctx;

/* Device memory through the caller's allocator (for instance a framework's
 * caching allocator).  alloc returns a device pointer of at least `bytes`
 * bytes, aligned to 256 bytes, or NULL on failure; free releases it.  Both
 * receive the `user` pointer given at creation.  Pass both NULL to let the
 * library use hipMalloc / hipFree; passing exactly one is CCT_EINVAL.  The
 * library frees everything it obtained this way in the matching destroy
 * call, after synchronising its stream(s). */
typedef void* (*cct_alloc_fn)(size_t bytes, void* user);
typedef void (*cct_free_fn)(void* ptr, void* user);

/* Create a context for o occupied / v virtual orbitals and naux fitting
 * functions.  opts_json may be NULL or a JSON object with integer/string
 * fields: "diis_space" (default 8), "diis_start" (default 2), "diis_t3"
 * ("full" | "none" | "subspace:<nv>", default "full"; Sec. "Distributed
 * DIIS": with "subspace:<nv>" only the T3 components whose three virtual
 * indices are among the first nv enter the DIIS overlaps and are
 * extrapolated, the rest of T3 keeps its Jacobi step; "none" leaves T3 out),
 * "diis" (true/false, default true), "tol" (> 0: default threshold of
 * cct_solve, 1e-8),
 * "workspace_gb" (cap on the scratch buffer; default: enough for every
 * unpacked slab in one batch, limited by free device memory), "timers"
 * (true: per-phase device times for cct_get_counters), "ladder_split"
 * (true by default: the symmetric/antisymmetric ladder; false: the direct
 * form), "lp_block_k" (>= 0, default 1024: in the split-BF16 mode the
 * ladder and ring operands whose contracted length is at least this are
 * stored with hi and lo interleaved by blocks of 32; a storage layout only,
 * the results do not depend on it).  alloc/free_fn/alloc_user: the caller's device allocator (see
 * cct_alloc_fn), or both NULL.  hip_stream: a hipStream_t or NULL.  The
 * memory plan is checked against free device memory here; CCT_ENOMEM if it
 * does not fit (or if the caller's allocator returns NULL). */
int cct_create(int nocc, int nvir, int naux, cct_precision prec, const char* opts_json, cct_alloc_fn alloc,
               cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_ctx** out);
/* Free the context and all device memory it owns.  NULL is ignored. */
void cct_destroy(cct_ctx* ctx);

/* Upload the bare Fock matrix f[n][n] (host).  Need not be diagonal; the
 * orbital energies of the denominators are its diagonal. */
int cct_set_fock(cct_ctx* ctx, const double* f);
/* Upload the density-fitting factors B[naux][n][n] (host). */
int cct_set_eri_df(cct_ctx* ctx, const double* B);

/* T1 = 0, T2 = v^{ij}_{ab} / (e_i + e_j - e_a - e_b), T3 = 0; clears DIIS. */
int cct_init_mp2(cct_ctx* ctx);
/* Copy amplitudes in (host arrays; t3p == NULL means T3 = 0); clears DIIS. */
int cct_set_amplitudes(cct_ctx* ctx, const double* t1, const double* t2, const double* t3p);
/* Copy amplitudes out (host arrays; any pointer may be NULL). */
int cct_get_amplitudes(cct_ctx* ctx, double* t1, double* t2, double* t3p);

/* Evaluate the residuals at the current amplitudes.  term_mask selects R3
 * term groups (CCT_TERM_*; R1 and R2 are always complete).  R3 is
 * post-processed (symmetrize i=j<k / i<j=k blocks, zero i=j=k blocks,
 * subtract the mean over virtual permutations).  Host outputs r1 [o][v],
 * r2 [o][o][v][v], r3p [ntri][v][v][v] may be NULL.  norms (may be NULL)
 * receives the squared full-tensor Frobenius norms |R1|^2, |R2|^2, |R3|^2
 * (packed blocks weighted by the number of distinct orderings of i,j,k). */
int cct_residual(cct_ctx* ctx, unsigned term_mask, double* r1, double* r2, double* r3p, double norms[3]);
/* Copy count elements of the packed R3 of the latest cct_residual/cct_update,
 * starting at flat element offset first (element (t,a,b,c) is at
 * ((t*v + a)*v + b)*v + c), to host memory. */
int cct_copy_r3(cct_ctx* ctx, int64_t first, int64_t count, double* out);

/* One iteration: residuals, R3 post-processing, Jacobi update t += r / eps,
 * DIIS extrapolation (if enabled by options), energy of the new amplitudes.
 * e_corr and norms (squared, as in cct_residual) may be NULL.  Returns
 * CCT_ENUMERIC if a norm or the energy is not finite. */
int cct_update(cct_ctx* ctx, double* e_corr, double norms[3]);
/* Correlation energy of the current amplitudes with the bare integrals. */
int cct_energy(cct_ctx* ctx, double* e_corr);
/* Iterate until sqrt(|R1|^2 + |R2|^2 + |R3|^2) < tol or max_iter; tol <= 0
 * takes the context's option "tol" (default 1e-8).  Returns CCT_ENOTCONV
 * (with the last energy and count filled in) if not converged. */
int cct_solve(cct_ctx* ctx, int max_iter, double tol, double* e_corr, int* iters);

/* Perturbative quadruples correction E_(Q) of CCSDT(Q) (the paper's (Q)
 * appendix, Eq. ener-pt-q with the residual Eq. resi-pt-q and the Wbar
 * intermediates Eqs. q_w_vvv_voo, q_w_vvo_ooo) from the context's current T2
 * and T3 (normally converged) and the BARE integrals; T1 does not enter, and
 * the denominators use the orbital energies f_pp (canonical orbitals).  FP64
 * whatever the context's precision.  Occupied-tuple traversal: one task per
 * i <= j <= k <= l in lexicographic order (cct_q_task_count(nocc) tasks;
 * tasks with three equal indices contribute exactly 0).  e_tasks (may be
 * NULL; else cap >= cct_q_task_count entries, host memory) receives each
 * task's contribution; *e_q their fixed-order sum.  Needs, beyond the
 * context and for the duration of the call (n = o + v), about
 * 8 * (n^4 + o^2 v^4 + o^3 v^3 + 2 o^4 v^2 + 28 v^4 + 48 * 4096 ceil(v/8)^4)
 * bytes of device memory for even v and nocc <= 16 (the task blocks are also
 * kept tile-major), else 8 * (n^4 + o^2 v^4 + o^3 v^3 + 2 o^4 v^2 + 52 v^4)
 * (about 110 GB at o=10, v=90): CCT_ENOMEM if that is not free (checked
 * before allocating when the library allocates; a caller's allocator is
 * asked block by block); CCT_EINVAL for nocc > 40; CCT_ESTATE before
 * cct_set_fock / cct_set_eri_df.  Synchronous (returns after the stream has
 * drained). */
int cct_energy_q(cct_ctx* ctx, double* e_q, double* e_tasks, int64_t cap);
/* cct_energy_q without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same evaluation, arguments and results as
 * cct_energy_q, with every per-call buffer taken from a fixed 256 MiB device
 * scratch array that the library holds on each GPU it runs on until the
 * process ends (looked up once per device on the first call there).  No
 * hipMalloc, hipFree or allocating library call.  Systems whose (Q) buffers
 * exceed 256 MiB (about nocc = 4, nvir = 20; the need grows as o^2 v^4 and
 * with the v^4 task blocks) are refused with CCT_ENOMEM and a message giving
 * the need, before any device work.  Every call on a GPU shares that GPU's
 * scratch: calls that overlap on one GPU (two threads, two contexts) race and
 * must be serialised by the caller; each call initialises what it reads. */
int cct_energy_q_noalloc(cct_ctx* ctx, double* e_q, double* e_tasks, int64_t cap);
/* Number of (Q) tasks, i <= j <= k <= l < nocc: nocc(nocc+1)(nocc+2)(nocc+3)/24
 * (-1 for nocc < 0). */
int64_t cct_q_task_count(int nocc);

/* E_(Q) in the virtual-tuple order of the "ABC-based algorithm" section
 * (Eq. ener-pt-q-abc, with the alternative intermediates of Eq. q_w_alter):
 * the same correction as cct_energy_q, summed over virtual tuples
 * a <= b <= c <= d.  The virtual labels are cut into tiles of `block`
 * (1..16, <= nvir); a task is a tile quadruple tA <= tB <= tC <= tD
 * (lexicographic order, cct_q_abc_task_count(nvir, block) of them) and
 * covers every tuple of its box with a <= b <= c <= d.  The call first
 * transposes the packed T3 to the virtual-triangular layout (blocks
 * a <= b <= c of o^3 contiguous occupied elements, Fig. q_operation_counts(a)),
 * then evaluates the listed tasks: tasks (host, ntasks indices) or, with
 * tasks == NULL, all of them (ntasks ignored).  *e_q: the fixed-order sum
 * of the evaluated tasks; e_tasks (may be NULL; host, one entry per
 * evaluated task); e_tuples (may be NULL; host, block^4 entries per task:
 * the first n0 n1 n2 n3 hold the tuples of the task's box in row-major order
 * over the four tiles' labels (n_s the tile sizes), each tuple's share of
 * E_(Q), 0 for tuples outside a <= b <= c <= d or with three equal labels,
 * the rest 0); stats (may be NULL; 4 entries): device ms of the integral
 * slices and the T3 transposition, device ms of the tasks, multiply-adds of
 * the tasks' matrix-core products, multiply-adds of the tasks' Wbar builds.
 * FP64 whatever the context's precision; T1 does not enter.  Needs about
 * 8 * (v(v+1)(v+2)/6 o^3 + v^4 + (o + v)^4 + 6 o^2 v^2 + 12 block^2 v o^3
 * + 36 block^3 o^2 v + 2 block^4 o^4) bytes of device memory (about 90 GB at
 * o=20, v=180, block 4): taken from the context's workspace when it holds
 * them (the workspace is idle between iterations), else allocated for the
 * duration of the call (the caller's allocator, or hipMalloc after a check
 * of the free memory; CCT_ENOMEM with the need in the message).  CCT_EINVAL
 * for a bad block or task index; CCT_ESTATE before cct_set_fock /
 * cct_set_eri_df.  Synchronous. */
int cct_energy_q_abc(cct_ctx* ctx, int block, const int64_t* tasks, int64_t ntasks, double* e_q, double* e_tasks,
                     double* e_tuples, double stats[4]);
/* Tasks of cct_energy_q_abc: T (T + 1) (T + 2) (T + 3) / 24 with
 * T = ceil(nvir / block) (-1 for nvir < 1 or block < 1). */
int64_t cct_q_abc_task_count(int nvir, int block);
/* out[i] = element idx[i] of the packed T3 (element (t, a, b, c) at
 * ((t v + a) v + b) v + c), i < n; host arrays.  CCT_EINVAL for an index
 * outside the packed T3.  Synchronous. */
int cct_gather_t3(cct_ctx* ctx, const int64_t* idx, int64_t n, double* out);

/* Algorithmic multiply-add counts of the last residual per R3 term group
 * (indices as the CCT_TERM_* bit positions, 9 entries) and device time in ms
 * per phase (entries: 0 setup/dressing+CCSD, 1 feedback, 2 PP, 3 rings,
 * 4 HH+F2, 5 drivers, 6 F1, 7 post+update, 8 DIIS+energy).  Entry 9: the
 * multiply-adds the ladder GEMMs executed (half the PP count in the
 * symmetric/antisymmetric form) and their device time alone (timers on);
 * entry 10: the number of ladder GEMM launches (ms: 0).  Entries 11-18 (ms:
 * 0) describe the batch plan the context's workspace allows: the number of
 * batches of the T3 feedback, of rings A, B and C, of the hole ladder, of
 * the two T2 drivers (entries 11-17, fixed at cct_create), and the chunks of
 * packed blocks the last ladder evaluation took (entry 18).  The per-term
 * counts are the direct-traversal ones whichever ladder form ran.  cap =
 * length of both arrays provided; writes min(cap, 19). */
int cct_get_counters(cct_ctx* ctx, double* macs_by_term, double* ms_by_phase, int cap);

/* Tile autotuner: times every tile variant of the particle-particle ladder
 * GEMM (on a truncated M of this context's shape, scratch output) and of the
 * ring GEMM (one batch of occupied pairs) in the context's precision and uses
 * the fastest from then on (results are the same to rounding in every
 * variant).  budget_ms bounds the timing (at least one variant per class is
 * timed).  The choice is also stored in the flat JSON file named by the
 * CCT_TUNE_CACHE environment variable (if set; keys "o<o>_v<v>_<prec>_ladder"
 * and "..._rings"), which cct_create reads.  variants (may be NULL) receives
 * {ladder variant, ring variant}.  Does not touch amplitudes or residuals. */
int cct_autotune(cct_ctx* ctx, double budget_ms, int* variants);

/* Index of the packed triple (i,j,k), 0 <= i <= j <= k < nocc, in the
 * lexicographic order; -1 if the arguments are out of range or unordered. */
int64_t cct_packed_index(int nocc, int i, int j, int k);

const char* cct_strerror(int code);
const char* cct_last_error(const cct_ctx* ctx);

/* ---- batches of independent systems ------------------------------------
 * Many small closed-shell systems iterated together (the same equations as
 * a single context, one context per system).  The device part of one
 * iteration of every system (DIIS save, residual, Jacobi steps) is recorded
 * once into a HIP graph and replayed once per iteration; norm read-back,
 * DIIS extrapolation and energy follow per system on the host side. */
typedef struct cct_batch cct_batch;

/* nsys systems with sizes nocc[s], nvir[s], naux[s] (host arrays), all in
 * precision prec.  opts_json: "streams" (1..16, default 4: systems are spread
 * over that many streams, largest triples work first onto the least loaded
 * stream; the graph forks and joins them),
 * "graph" (true by default; false enqueues every iteration eagerly, the same
 * kernels in the same order), and the per-system keys of cct_create
 * ("diis", "diis_space", "diis_start", "diis_t3", "workspace_gb",
 * "ladder_split").  alloc/free_fn/alloc_user: as for cct_create, used by
 * every system.  hip_stream (may be NULL): the caller's stream becomes the
 * first of the batch's streams, on which the graph is launched and joined
 * (not destroyed by the library); the others are created by the library.
 * Errors: CCT_EINVAL (sizes, options), CCT_ENOMEM, CCT_EDEVICE. */
int cct_batch_create(int nsys, const int* nocc, const int* nvir, const int* naux, cct_precision prec,
                     const char* opts_json, cct_alloc_fn alloc, cct_free_fn free_fn, void* alloc_user,
                     void* hip_stream, cct_batch** out);
/* Upload system s's bare Fock f[n][n] and factors B[naux][n][n] (host) and
 * start it from the MP2 guess.  Does not invalidate a recorded graph (the
 * device buffers keep their addresses). */
int cct_batch_set_system(cct_batch* b, int s, const double* f, const double* B);
/* niter iterations of every system.  e_corr [nsys] and norms [nsys][3]
 * (squared norms of R1, R2, R3) after the last one; either may be NULL.
 * CCT_ESTATE if a system has no integrals; per-system errors as for
 * cct_update, with the system named in cct_batch_last_error. */
int cct_batch_iterate(cct_batch* b, int niter, double* e_corr, double* norms);
/* The context of system s (owned by the batch; valid until
 * cct_batch_destroy), for cct_get_amplitudes, cct_energy, cct_get_counters.
 * NULL if s is out of range. */
cct_ctx* cct_batch_system(cct_batch* b, int s);
/* Tunes one system of each distinct (nocc, nvir) with cct_autotune (budget
 * split evenly) and gives its choice to every system of that size; the
 * recorded graph is dropped and recorded again by the next cct_batch_iterate. */
int cct_batch_autotune(cct_batch* b, double budget_ms);
const char* cct_batch_last_error(const cct_batch* b);
void cct_batch_destroy(cct_batch* b);

/* ---- slab of packed triples ---------------------------------------------
 * The R3 terms that need only the locally stored T3 blocks, for packed
 * triples [first, first + count) of an nocc-occupied system: the
 * particle-particle ladder (paper, Sec. "RCCSDT contractions without
 * unpacking"), the F_vv part of the Fock term and the two T2*W drivers of
 * Eq. resi-rccsdt, followed by the R3 post-processing of Sec. "Removing
 * redundancies in RCC amplitudes".  This is one process's share of a run
 * sharded by packed triples; T1, T2 and the intermediates are replicated
 * inputs.  W^{ab}_{de} = sum_P B~^P_{ad} B~^P_{be} + sum_lm v~^{lm}_{de}
 * t_lm^ab is rebuilt in panels of opts "panel" rows a (default 8) and never
 * stored whole.  Ladder operands in the working precision (FP32, or hi+lo
 * BF16 when v^2 is a multiple of 4 or 8; FP64 otherwise); F_vv term and
 * drivers in FP64; R3 in FP64. */
typedef struct cct_slab cct_slab;

/* first + count <= nocc(nocc+1)(nocc+2)/6, count <= 65535.  opts_json:
 * "panel" (rows a per W panel, 1..nvir), "timers" (true: per-phase times
 * in cct_slab_get_counters).  alloc/free_fn/alloc_user: as for cct_create.
 * Errors: CCT_EINVAL, CCT_ENOMEM. */
int cct_slab_create(int nocc, int nvir, int naux, int first, int count, cct_precision prec, const char* opts_json,
                    cct_alloc_fn alloc, cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_slab** out);
/* Replicated inputs (host arrays, copied in): Bt = T1-dressed factors
 * B~[naux][n][n] (Appendix A, "T1-dressed formalism"), t2 [o][o][v][v]
 * (t_ij^ab = t_ji^ba), Fvv [a][d] = F^a_d, Wt [j][a][b][d] = W^{ab}_{dj},
 * Wvooo [a][l][i][j] = W^{al}_{ij}. */
int cct_slab_set_intermediates(cct_slab* sl, const double* Bt, const double* t2, const double* Fvv,
                               const double* Wt, const double* Wvooo);
/* The slab's stored T3 blocks, t3slab [count][v][v][v] (host). */
int cct_slab_set_t3(cct_slab* sl, const double* t3slab);
/* R3 of the slab for term_mask within CCT_TERM_PP | CCT_TERM_F1 |
 * CCT_TERM_D1 | CCT_TERM_D2 (CCT_EINVAL otherwise; F1 here is the F_vv part
 * only), post-processed.  r3slab [count][v][v][v] (host, may be NULL);
 * norm2 = sum over the slab of multiplicity x squared elements.
 * CCT_ESTATE before both setters, CCT_ENUMERIC on a non-finite norm. */
int cct_slab_residual(cct_slab* sl, unsigned term_mask, double* r3slab, double* norm2);
/* Copy count elements of the slab's R3 from element offset first (host). */
int cct_slab_copy_r3(cct_slab* sl, int64_t first, int64_t count, double* out);
/* Multiply-adds of the last residual: [0] ladder 3 count v^5, [1] W rebuild
 * (naux + o^2) v^4, [2] F_vv 3 count v^4, [3] W^{ab}_{dj} driver 6 count v^4,
 * [4] W^{al}_{ij} driver 6 count o v^3, [5] 0; milliseconds (with "timers"):
 * [0] T3 relabelling, [1] W rebuild, [2] ladder GEMMs, [3] F_vv, [4] drivers,
 * [5] post-processing.  Writes min(cap, 6) of each. */
int cct_slab_get_counters(cct_slab* sl, double* macs, double* ms, int cap);
const char* cct_slab_last_error(const cct_slab* sl);
void cct_slab_destroy(cct_slab* sl);

/* ---- quadruples ladder on compact T4 ----------------------------------------
 * The particle-particle ladder term of the RCCSDTQ quadruples residual (the
 * paper's Appendix "RCCSDTQ", Eq. resi-rccsdtq: P_(ia)(jb)(kc)(ld)
 * [1/4 sum_ef W^{ab}_{ef} t_ijkl^efcd], its O(o^4 v^6) leading term) on T4
 * stored only for occupied quadruples i <= j <= k <= l, in the compact
 * six-term form of Sec. "RCCSDTQ contractions": for every stored block
 * R[.. x at p .. y at q ..] += sum_ef W^{xy}_{ef} T[.. e at p .. f at q ..]
 * over the six pairs of virtual positions (p, q), every operand from the
 * same stored block.  Layouts (host, FP64, C-contiguous):
 *   W    [v][v][v][v]          W[a][b][e][f] = W^{ab}_{ef}; must satisfy
 *                              W^{ab}_{ef} = W^{ba}_{fe} (as the RCCSDT
 *                              intermediate does) for the compact form to
 *                              equal the permutation sum
 *   t4p  [nq][v][v][v][v]      nq = nocc(nocc+1)(nocc+2)(nocc+3)/24 blocks in
 *                              lexicographic order of i <= j <= k <= l
 *                              (cct_quad_packed_index), block (i,j,k,l) holding
 *                              t_ijkl^abcd for all a,b,c,d
 * Products in the precision of cct_precision (FP64 MFMA; FP32 or split-BF16
 * operands with FP64 output), R4 in FP64. */
typedef struct cct_quad cct_quad;

/* nocc >= 1, nvir >= 1, nq <= 65535, nvir^2 <= 46340.  opts_json: "timers"
 * (true: device times in cct_quad_get_counters).  alloc/free_fn/alloc_user,
 * hip_stream: as for cct_create.  Device memory: about 8 (v^4 + 3 nq v^4)
 * bytes (+ 4 (nq v^4 + v^4) in the mixed modes).  Errors: CCT_EINVAL,
 * CCT_ENOMEM, CCT_EDEVICE. */
int cct_quad_create(int nocc, int nvir, cct_precision prec, const char* opts_json, cct_alloc_fn alloc,
                    cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_quad** out);
/* Copy W and/or the packed T4 in (host arrays; either may be NULL, not both). */
int cct_quad_set(cct_quad* q, const double* W, const double* t4p);
/* R4 = the compact ladder term for every stored block (raw: no
 * post-processing).  r4p [nq][v^4] (host) may be NULL; norm2 (may be NULL)
 * receives sum over blocks of multiplicity x squared elements.  CCT_ESTATE
 * before both inputs are set; CCT_ENUMERIC on a non-finite norm. */
int cct_quad_ladder(cct_quad* q, double* r4p, double* norm2);
/* Copy count elements of R4 from flat element offset first (host). */
int cct_quad_copy_r4(cct_quad* q, int64_t first, int64_t count, double* out);
/* macs[0]: multiply-adds of the last evaluation (6 nq v^6); ms (with
 * "timers"): [0] relabelled copies, [1] GEMMs.  Writes min(cap, 2). */
int cct_quad_get_counters(cct_quad* q, double* macs, double* ms, int cap);
/* Number of stored blocks for nocc occupied orbitals (-1 for nocc < 0). */
int64_t cct_quad_count(int nocc);
/* Index of the stored block (i,j,k,l), i <= j <= k <= l < nocc; -1 otherwise. */
int64_t cct_quad_packed_index(int nocc, int i, int j, int k, int l);
const char* cct_quad_last_error(const cct_quad* q);
void cct_quad_destroy(cct_quad* q);

#ifdef __cplusplus
}
#endif

#endif /* CCT_H */
