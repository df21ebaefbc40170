/*
 * cc3.h - C ABI of libcc3.so, the MI355X (gfx950) implementation of the CC3
 * ground-state triples contribution to the singles and doubles residual.
 *
 * Method: Paul, Myhre & Koch, "A new and efficient implementation of CC3"
 * (arXiv 2007.01088), Sec. "Implementation", Algorithm 1.  For every
 * unordered occupied triple i >= j >= k (i == j == k skipped) the library
 * builds t3 from (bd|ck) t2 and (lj|ck) t2 contractions, the permutation
 * operator P^{abc}_{ijk} and the orbital-energy denominator, forms the
 * contravariant amplitudes, and contracts them into the contravariant
 * residual; a back-transformation gives the covariant Omega.  The full
 * nv^3 no^3 t3 tensor is never stored.
 *
 * Conventions shared by every entry point
 *   - Return value: CC3_OK (0) or a negative CC3_E_* code; cc3_last_error()
 *     then returns a thread-local message describing the failure.
 *   - Array pointers are row-major float64 arrays owned by the caller.  The
 *     one-shot residual calls (cc3_triples_residual, cc3_triples_residual_blocks,
 *     cc3_triples_residual_subset, cc3_t3_block) take device memory of the
 *     context's GPU (torch CUDA tensors, hipMalloc) or host memory, pageable or
 *     pinned, told apart with hipPointerGetAttributes: a host input is copied on
 *     `stream` into the workspace, a host output is produced there and copied
 *     back.  cc3_jacobian_prep takes device pointers only (its outputs are as
 *     large as the integral blocks).  The library keeps no pointer after the
 *     work it enqueued has completed.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without waiting for it; results are valid once the
 *     stream has reached that point.  A call with any host-memory argument
 *     waits for its stream before it returns (its host outputs are then final
 *     and its host inputs may be reused).
 *   - Index order: occupied orbitals first.  eps[no+nv]; L[nchol][nmo][nmo]
 *     (nmo = no+nv, symmetric in the last two indices); t1[no][nv] = t^a_i;
 *     t2[no][no][nv][nv] = t^{ab}_{ij} with t2[i][j][a][b] == t2[j][i][b][a];
 *     omega1[no][nv]; omega2[no][no][nv][nv].
 *   - Scratch memory comes only from the caller's workspace (size from
 *     cc3_workspace_size); the library allocates no device memory for the
 *     residual calls.
 */
#ifndef CC3_H
#define CC3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc3_ctx cc3_ctx;
typedef void* cc3_stream_t; /* hipStream_t */

/* status codes */
enum {
  CC3_OK = 0,
  CC3_E_INVAL = -1,    /* bad argument: sizes, null pointer, host pointer where only device
                          memory is accepted, unknown enum */
  CC3_E_NOMEM = -2,    /* workspace (or arena) too small for the request */
  CC3_E_DEVICE = -3,   /* a HIP runtime call failed */
  CC3_E_PRECOND = -4,  /* CC3_CHECK found a violated input symmetry or denominator */
  CC3_E_NOTFOUND = -5, /* unknown molecule or ticket */
  CC3_E_BUSY = -6,     /* serving queue full (non-blocking submit) */
  CC3_E_TIMEOUT = -7,  /* wait timed out */
  CC3_E_CANCELLED = -8 /* request was cancelled */
};

/* arithmetic of the W contractions (the t3-building GEMMs, Algorithm 1 first statement) */
enum {
  CC3_FP64 = 0,   /* FP64 MFMA everywhere */
  CC3_FP32 = 1,   /* W contractions on FP32 MFMA; each 32-k stage summed in FP32, the
                     stages accumulated in FP64 */
  CC3_BF16X3 = 2, /* W on bf16 MFMA, 2-piece split, 3 products, FP32 accumulation per term */
  CC3_BF16X6 = 3  /* W on bf16 MFMA, 3-piece split, 6 products; each 32-k stage summed in
                     FP32, the stages accumulated in FP64 */
};
/* In every precision the denominator division, the P-symmetrisation, the
 * contravariant combination and the Omega accumulation are FP64. */

/* flags */
enum {
  CC3_ACCUMULATE = 1u,    /* add the triples contribution into omega1/omega2 instead of overwriting */
  CC3_CHECK = 2u,         /* verify input symmetries (t2, L) and positive denominators first */
  CC3_ONE_STREAM = 4u,    /* run the batches of the triple loop one after another on one stream
                             instead of overlapping consecutive batches on two; the result is
                             the same, each kernel runs without a neighbour on the device
                             (standalone timing), the call is slower (one-shot calls only) */
  CC3_LOWP_CONTRACT = 8u, /* "mixed-all": with prec = CC3_FP32, the vv term and Omega1 of the
                             Omega contraction also run on FP32 MFMA, over FP32 roundings of the
                             contravariant t3 and of the (vv|ov) and (ov|ov) blocks; each K chunk
                             sums in FP32, the chunks and triples in FP64.  The oo and Fock terms
                             and the back-transformation stay FP64.  One-shot residual calls
                             only (not cc3_jacobian_prep, not serving); other precisions:
                             CC3_E_INVAL.  The workspace grows (cc3_workspace_size with it). */
  CC3_DETERMINISTIC = 16u /* accepted for callers that ask for it: every call is deterministic
                             anyway (fixed-order reductions, no floating-point atomics), so the
                             same inputs and sizes give the same bits */
};

/* ---------------------------------------------------------------------- */
/* Context                                                                  */
/* ---------------------------------------------------------------------- */

/* Create a context bound to HIP device `device`.  *out receives the handle.
 * Errors: CC3_E_INVAL (out NULL, device out of range), CC3_E_DEVICE. */
int cc3_create(cc3_ctx** out, int device);

/* Destroy a context (NULL is accepted).  Waits for nothing: the caller must
 * have synchronised the streams it used. */
int cc3_destroy(cc3_ctx* ctx);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* cc3_last_error(void);

/* ---------------------------------------------------------------------- */
/* One-shot residual                                                        */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace needed by cc3_triples_residual (nchol > 0) or
 * cc3_triples_residual_blocks (nchol == 0) for these sizes, precision and
 * flags.  Host-only computation; no context needed.
 * Supported sizes: 1 <= no <= 63, 1 <= nv <= 1024.
 * Errors: CC3_E_INVAL (sizes out of range, nchol < 0, bytes NULL, unknown prec). */
int cc3_workspace_size(int no, int nv, int nchol, int prec, unsigned flags, size_t* bytes);

/* The CC3 ground-state triples contribution (Algorithm 1) from Cholesky vectors.
 *
 * The integrals are T1-transformed (H = exp(-T1) H exp(T1), Sec. Theory):
 * Lt^J = (1 - t) L^J (1 + t) with t[no+a][i] = t1[i][a]; g_pqrs = sum_J Lt^J_pq Lt^J_rs;
 * F_kc = sum_ld t1[l][d] (2 g_kcld - g_kdlc) (T1-transformed Fock ov block of a
 * canonical reference).  The integral blocks stay resident in the workspace
 * for the whole call.
 *
 * Inputs (device or host): eps[no+nv], L[nchol][nmo][nmo], t1[no][nv], t2[no][no][nv][nv].
 * Outputs (device or host): omega1[no][nv], omega2[no][no][nv][nv]: the covariant
 * triples contribution  Omega^a_i = Ot^a_i,
 * Omega^{ab}_{ij} = 1/3 [(2 Ot^{ab}_{ij} + Ot^{ba}_{ij}) + (2 Ot^{ba}_{ji} + Ot^{ab}_{ji})],
 * written (or added, with CC3_ACCUMULATE).
 * workspace: device buffer of at least cc3_workspace_size(no, nv, nchol, prec, flags) bytes,
 * 256-byte aligned; contents on entry are ignored.
 * Errors: CC3_E_INVAL, CC3_E_NOMEM (workspace_bytes too small), CC3_E_DEVICE,
 * CC3_E_PRECOND (with CC3_CHECK). */
int cc3_triples_residual(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps,
                         const double* L, const double* t1, const double* t2, double* omega1,
                         double* omega2, int prec, unsigned flags, void* workspace,
                         size_t workspace_bytes, cc3_stream_t stream);

/* The same residual from integral blocks already in the T1-transformed basis,
 * laid out in the paper's index order (device or host, row-major; host
 * g_vvvo and g_vvov pass through the workspace in slabs of the first index):
 *   g_vvvo[b][d][c][k] = g_{bdck},  g_oovo[l][j][c][k] = g_{ljck},
 *   g_ovov[j][b][k][c] = g_{jbkc},  g_ooov[j][l][k][c] = g_{jlkc},
 *   g_vvov[d][b][k][c] = g_{dbkc},  F_ov[k][c] = F_{kc}.
 * Workspace from cc3_workspace_size(no, nv, 0, prec, flags).  Errors as above. */
int cc3_triples_residual_blocks(cc3_ctx* ctx, int no, int nv, const double* eps,
                                const double* g_vvvo, const double* g_oovo, const double* g_ovov,
                                const double* g_ooov, const double* g_vvov, const double* F_ov,
                                const double* t2, double* omega1, double* omega2, int prec,
                                unsigned flags, void* workspace, size_t workspace_bytes,
                                cc3_stream_t stream);

/* Contravariant contributions (before the back-transformation) of a listed
 * subset of unordered occupied triples only: for each distinct occupied
 * permutation (p,q,r) of a listed (i,j,k), with U = tau~_{pqr},
 *   Ot1[p][a] += sum_bc U^{abc} g_{qbrc};  Ot2[p][q][a][b] += sum_c U^{abc} F_{rc};
 *   Ot2[p][l][a][b] -= sum_c U^{abc} g_{qlrc};  Ot2[p][q][a][d] += sum_bc U^{abc} g_{dbrc}.
 * triples: HOST int32 array [ntriples][3] with i >= j >= k, not all equal, each
 * < no (copied before the call returns).  omega1_tilde[no][nv] and
 * omega2_tilde[no][no][nv][nv] (device or host) are overwritten; the call waits
 * for its stream before it returns.  Used for sampled
 * parity at large sizes and to emulate a triple-partitioned multi-GPU run.
 * Workspace as for cc3_triples_residual.  Errors: CC3_E_INVAL (bad triple),
 * CC3_E_NOMEM, CC3_E_DEVICE. */
int cc3_triples_residual_subset(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps,
                                const double* L, const double* t1, const double* t2,
                                const int32_t* triples, int ntriples, double* omega1_tilde,
                                double* omega2_tilde, int prec, unsigned flags, void* workspace,
                                size_t workspace_bytes, cc3_stream_t stream);

/* cc3_triples_residual_subset from integral blocks in the T1-transformed basis
 * (the same six blocks, layouts and host/device handling as
 * cc3_triples_residual_blocks) instead of Cholesky vectors: sampled parity and
 * a triple-partitioned run on integrals the caller holds.  Workspace from
 * cc3_workspace_size(no, nv, 0, prec, flags).  Errors as for
 * cc3_triples_residual_subset. */
int cc3_triples_residual_subset_blocks(cc3_ctx* ctx, int no, int nv, const double* eps,
                                       const double* g_vvvo, const double* g_oovo,
                                       const double* g_ovov, const double* g_ooov,
                                       const double* g_vvov, const double* F_ov, const double* t2,
                                       const int32_t* triples, int ntriples, double* omega1_tilde,
                                       double* omega2_tilde, int prec, unsigned flags,
                                       void* workspace, size_t workspace_bytes,
                                       cc3_stream_t stream);

/* cc3_triples_residual without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace is a static device array of the library (256 MiB per GPU, reserved
 * when the library's code is loaded on that GPU and held until the process ends);
 * the call runs every batch on `stream` and records no events.  Arguments, results
 * and arithmetic are those of cc3_triples_residual, except: all six arrays must be
 * device memory of the context's GPU; flags may be CC3_ACCUMULATE,
 * CC3_LOWP_CONTRACT, CC3_DETERMINISTIC (CC3_ONE_STREAM is implied); the plan takes
 * fewer triples per batch where needed to fit the array (the result is the same to
 * rounding, 1e-11 relative in FP64).  Every call on one GPU uses that GPU's one
 * array: calls whose device work overlaps (different streams, different contexts
 * on the same GPU) race and corrupt each other's results; calls ordered on one
 * stream are safe.  The array keeps the last call's contents; the call clears what
 * must start at zero itself.
 * Errors: CC3_E_INVAL (sizes, flags, host pointers), CC3_E_NOMEM (the workspace at
 * one triple per batch exceeds 256 MiB: roughly nv above 70 at no = 10),
 * CC3_E_DEVICE. */
int cc3_triples_residual_noalloc(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps,
                                 const double* L, const double* t1, const double* t2,
                                 double* omega1, double* omega2, int prec, unsigned flags,
                                 cc3_stream_t stream);

/* Debug export of the t3 amplitudes of one ordered triple (i, j, k) (any order,
 * not all equal): tau[a][b][c] = tau^{abc}_{ijk} = -(eps^{abc}_{ijk})^{-1} P^{abc}_{ijk} B^{abc}_{ijk}
 * (Algorithm 1, first statement), written to tau[nv][nv][nv] (device or host); the
 * call waits for its stream before it returns.
 * Inputs as for cc3_triples_residual.  Errors: CC3_E_INVAL, CC3_E_NOMEM, CC3_E_DEVICE. */
int cc3_t3_block(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps, const double* L,
                 const double* t1, const double* t2, int i, int j, int k, double* tau, int prec,
                 void* workspace, size_t workspace_bytes, cc3_stream_t stream);

/* cc3_t3_block from integral blocks in the T1-transformed basis (the six blocks,
 * layouts and host/device handling of cc3_triples_residual_blocks; the amplitudes
 * read g_vvvo and g_oovo, the other four are loaded as by every blocks-form call).
 * Workspace from cc3_workspace_size(no, nv, 0, prec, 0).  Errors as for cc3_t3_block. */
int cc3_t3_block_blocks(cc3_ctx* ctx, int no, int nv, const double* eps, const double* g_vvvo,
                        const double* g_oovo, const double* g_ovov, const double* g_ooov,
                        const double* g_vvov, const double* F_ov, const double* t2, int i, int j,
                        int k, double* tau, int prec, void* workspace, size_t workspace_bytes,
                        cc3_stream_t stream);

/* The t3-dependent intermediates of the preparation for the Jacobian
 * transformations (Sec. "Implementation", Algorithm 2): the same restricted loop,
 * t3 and contravariant t3 as cc3_triples_residual, then for each distinct
 * occupied permutation (p,q,r) of a triple, with U = tau~_{pqr},
 *   Z~v_{abpd} -= sum_c U^{abc} g_{qdrc},   Z~o_{aqpl} += sum_{bc} U^{abc} g_{lbrc}.
 * Outputs (device, row-major, overwritten or added with CC3_ACCUMULATE):
 *   zv[nv][nv][no][nv] = Z~v_{abid},  zo[nv][no][no][no] = Z~o_{ajil}.
 * Inputs as for cc3_triples_residual but in device memory only (a host pointer
 * gives CC3_E_INVAL); precision (of the W contractions) and workspace as for
 * cc3_triples_residual (same cc3_workspace_size).  Supported sizes additionally
 * need no^2 nv^2 < 2^31.  Errors: CC3_E_INVAL, CC3_E_NOMEM, CC3_E_DEVICE,
 * CC3_E_PRECOND (with CC3_CHECK). */
int cc3_jacobian_prep(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps, const double* L,
                      const double* t1, const double* t2, double* zv, double* zo, int prec,
                      unsigned flags, void* workspace, size_t workspace_bytes, cc3_stream_t stream);

/* How the one-shot calls batch the restricted loop for these sizes (host-only,
 * no context needed): *triples_per_batch receives the unordered triples per
 * batch, *nbatches the number of batches.  The loop's triples, in lexicographic
 * order (i >= j >= k, i == j == k excluded), are dealt round-robin: batch b holds
 * the loop positions b, b + nbatches, b + 2 nbatches, ...  Passing one batch's
 * triples, in that order, to cc3_triples_residual_subset reproduces the launch
 * configuration of that batch in the whole call (sampled parity, sharding).
 * Errors: CC3_E_INVAL (sizes as for cc3_workspace_size, NULL outputs). */
int cc3_batch_plan(int no, int nv, int nchol, int prec, unsigned flags, int* triples_per_batch,
                   int* nbatches);

/* Bytes of device workspace for cc3_transition_density at these sizes (host-only).
 * Supported sizes: 1 <= no <= 63, 1 <= nv <= 400, nchol >= 1.
 * Errors: CC3_E_INVAL. */
int cc3_transition_density_workspace_size(int no, int nv, int nchol, size_t* bytes);

/* The triples contributions to the transition density D^{m,0} of one left state
 * (Sec. "Implementation", Algorithm 3).  With tau the ground-state t3 of
 * Algorithm 1, the left-state triples
 *   L^{abc}_{ijk} = (omega - eps^{abc}_{ijk})^{-1} P^{abc}_{ijk} (L^a_i g_{jbkc} + L^{ab}_{ij} F_kc
 *                   + sum_d L^{ad}_{jk} g_{ibdc} - sum_l L^{ab}_{lk} g_{iljc}),
 * and L~, tau~ the contravariant combinations (virtual indices permuted at fixed
 * i, j, k), summed over every ordered occupied triple (p, q, r):
 *   D_cd[c][d] += 1/2 sum_ab L~_{pqr}[a,b,c] tau_{pqr}[a,b,d]
 *   D_kc[r][c] += sum_ab l2[p][q][a][b] tau~_{pqr}[a,b,c]
 *   Y^o[c][l][p][r] += sum_ab L~_{pqr}[a,b,c] t2[l][q][a][b],
 *   D_ld[l][d] -= sum_{cik} Y^o[c][l][i][k] t2[k][i][c][d],
 *   D_lk[l][k] -= 1/2 sum_{ij} sum_{abc} L~^{abc}_{ijk} tau^{abc}_{ijl}.
 * The integrals and F_kc are the T1-transformed ones of cc3_triples_residual.
 * The occupied-occupied block, which the paper evaluates in a loop over virtual
 * triples, is evaluated here as the Gram matrices <L~_{ijk}, tau_{ijl}> of the
 * cubes of each occupied pair (i, j); the loop runs over those pairs.
 * Inputs (device memory only): eps[no+nv], L[nchol][nmo][nmo], t1[no][nv],
 * t2[no][no][nv][nv] as for cc3_triples_residual; l1[no][nv] = L^a_i and
 * l2[no][no][nv][nv] = L^{ab}_{ij} (l2[i][j][a][b] == l2[j][i][b][a]) of the left
 * state; omega its excitation energy (omega - eps^{abc}_{ijk} must not vanish).
 * Outputs (device memory, row-major, overwritten or added with CC3_ACCUMULATE):
 * D_cd[nv][nv], D_kc[no][nv], D_ld[no][nv], D_lk[no][no]; Yo[nv][no][no][no] = Y^o
 * (may be NULL).  FP64 throughout.  flags: CC3_ACCUMULATE, CC3_DETERMINISTIC.
 * workspace: at least cc3_transition_density_workspace_size bytes, 256-byte aligned.
 * Errors: CC3_E_INVAL (sizes, flags, host pointers), CC3_E_NOMEM, CC3_E_DEVICE. */
int cc3_transition_density(cc3_ctx* ctx, int no, int nv, int nchol, const double* eps,
                           const double* L, const double* t1, const double* t2, const double* l1,
                           const double* l2, double omega, double* D_cd, double* D_kc,
                           double* D_ld, double* D_lk, double* Yo, unsigned flags, void* workspace,
                           size_t workspace_bytes, cc3_stream_t stream);

/* FLOP per residual call: *nominal = 4 nv^4 no^3 (the paper's asymptotic count,
 * abstract); *executed = the multiply-adds (x2) this library's triple loop
 * issues for the dominant contractions and their small companions, padding
 * excluded.  Either pointer may be NULL.  Errors: CC3_E_INVAL. */
int cc3_flops(int no, int nv, double* nominal, double* executed);

/* Core-valence separation worklist (Sec. "Results", core excitations): the
 * triple loop of the Jacobian transformations skips the occupied triples none
 * of whose indices is a core orbital of interest, which takes their cost from
 * 8 nv^4 no^3 to 8 nv^4 no^2; the ground state keeps every triple.  Writes the
 * unordered triples i >= j >= k (i == j == k excluded, as in the full loop) that
 * contain at least one of the `ncore` HOST indices `core` (each in [0, no),
 * repeats allowed), in the loop's lexicographic order, to the HOST array
 * triples[n][3] (int32), and their number to *ntriples.  With triples == NULL
 * only the count is written; otherwise `capacity` is the number of rows the
 * array holds.  The list feeds cc3_triples_residual_subset.  Host-only, no
 * context needed.  Errors: CC3_E_INVAL (bad sizes, index out of range, or
 * capacity smaller than the count). */
int cc3_cvs_triples(int no, const int32_t* core, int ncore, int32_t* triples, int capacity,
                    int* ntriples);

/* ---------------------------------------------------------------------- */
/* Kernel timing (HIP events on the launch stream)                          */
/* ---------------------------------------------------------------------- */

typedef struct cc3_kernel_stat {
  char name[32];      /* kernel family, e.g. "w_build", "omega_contract" */
  int64_t launches;   /* launches recorded since the last reset */
  double total_ms;    /* sum of event-measured durations */
  double flops;       /* algorithmic FLOP of those launches (padding excluded) */
  double bytes;       /* algorithmic HBM bytes of those launches */
} cc3_kernel_stat;

/* Turn per-launch event timing on (1) or off (0); turning it on resets the stats. */
int cc3_profile_enable(cc3_ctx* ctx, int on);
/* Copy up to `max` kernel-family stats to out; *count receives the number
 * written.  Synchronises the recorded events (blocks the host).  Errors:
 * CC3_E_INVAL, CC3_E_DEVICE. */
int cc3_profile_get(cc3_ctx* ctx, cc3_kernel_stat* out, int max, int* count);

/* ---------------------------------------------------------------------- */
/* Serving: residual requests from many molecules, as solvers issue them    */
/* ---------------------------------------------------------------------- */
/* A server owns one caller-provided device buffer (the arena) and carves
 * everything from it: the resident data of each registered molecule (eps, L,
 * t1, t2, the T1-transformed integral blocks and the result) and, per request,
 * the transient workspace of one residual evaluation.  A worker thread admits
 * queued requests in arrival order whenever a slot (an independent set of
 * streams, at most max_inflight) is free and the request's workspace fits in
 * the arena (admission by HBM footprint); admitted requests run concurrently
 * on the device, so new arrivals join work that is already in flight.  The
 * arithmetic of a request is exactly that of cc3_triples_residual (Algorithm 1);
 * the integral blocks are rebuilt only when a request brings new t1.
 *
 * Pointers passed to the serving calls may be host or device memory
 * (detected per pointer); inputs are copied before the call returns, so the
 * caller may reuse its buffers at once.  The library allocates no device
 * memory here: everything lives in the arena (the server's streams and events
 * are the only other device resources).  All calls are thread-safe.
 * Each slot uses two HIP streams and the server one more for its copies; the
 * runtime multiplexes streams onto a fixed number of hardware queues
 * (GPU_MAX_HW_QUEUES, 4 by default), and streams that share a queue wait for
 * each other, so a process serving with max_inflight slots should allow at
 * least 2 * max_inflight + 2 hardware queues.
 * Clock: the timestamps of cc3_timing are seconds on a steady host clock
 * whose zero is the server's creation. */
typedef struct cc3_server cc3_server;

typedef struct cc3_timing {
  double arrival_s; /* cc3_submit was entered (before its input copies) */
  double admit_s;   /* workspace granted from the arena and the work enqueued on a slot */
  double start_s;   /* the device began the request's first kernel (device clock mapped to host) */
  double finish_s;  /* the server observed the request's completion */
  double device_ms; /* device time from the first to the last kernel of the request */
  int slot;         /* slot the request ran on */
  int rebuilt;      /* 1 if the integral blocks were rebuilt (new t1) */
} cc3_timing;

typedef struct cc3_server_stats {
  int64_t submitted, completed, failed, cancelled;
  int queued, inflight, max_inflight_seen, molecules;
  size_t arena_bytes, arena_used, arena_peak;
  int64_t packed; /* requests that ran in packed groups */
  int64_t packs;  /* packed groups launched */
} cc3_server_stats;

/* Create a server on `device` over the arena [arena, arena + arena_bytes)
 * (device memory of that GPU, 256-byte aligned, owned by the caller and kept
 * alive until cc3_server_destroy returns).  1 <= max_inflight <= 8.
 * Errors: CC3_E_INVAL, CC3_E_DEVICE. */
int cc3_server_create(cc3_server** out, int device, void* arena, size_t arena_bytes,
                      int max_inflight);

/* Cancel queued requests, wait for the ones in flight, stop the worker and
 * free the server (NULL accepted).  Uncollected results are dropped; no other
 * call on this server may be in progress or follow. */
int cc3_server_destroy(cc3_server* srv);

/* Arena bytes of one molecule (*resident, held from register to release) and
 * of one request's transient workspace (*transient, held from admission to
 * completion) on this server.  Either pointer may be NULL.
 * Errors: CC3_E_INVAL (sizes as for cc3_workspace_size, nchol >= 1). */
int cc3_server_footprint(cc3_server* srv, int no, int nv, int nchol, int prec, size_t* resident,
                         size_t* transient);

/* Register a molecule: copies eps[no+nv] and L[nchol][nmo][nmo] (and t1[no][nv];
 * NULL means t1 = 0) into its resident arena region; *mol receives its id.
 * Blocks the caller until the copies are done.  Errors: CC3_E_INVAL,
 * CC3_E_NOMEM (no hole in the arena large enough), CC3_E_DEVICE. */
int cc3_molecule_register(cc3_server* srv, int no, int nv, int nchol, const double* eps,
                          const double* L, const double* t1, uint64_t* mol);

/* Free a molecule's arena region.  Errors: CC3_E_NOTFOUND, CC3_E_BUSY (it has
 * a request that has not been collected by cc3_wait). */
int cc3_molecule_release(cc3_server* srv, uint64_t mol);

/* Queue one residual evaluation of molecule `mol`: copies t2[no][no][nv][nv]
 * (and t1[no][nv] if not NULL; NULL keeps the molecule's current t1 and its
 * integral blocks) into the molecule's region, then queues the request and
 * returns its ticket.  prec as for cc3_triples_residual; flags: CC3_CHECK
 * (checked here, blocking, before queueing) and CC3_ACCUMULATE (applied at
 * cc3_wait).  A molecule has at most one unfinished request: submit again
 * after cc3_wait.  Errors: CC3_E_INVAL, CC3_E_NOTFOUND, CC3_E_BUSY (the
 * molecule has an unfinished request), CC3_E_NOMEM (the request's workspace
 * exceeds the whole arena), CC3_E_PRECOND, CC3_E_DEVICE. */
int cc3_submit(cc3_server* srv, uint64_t mol, const double* t1, const double* t2, int prec,
               unsigned flags, uint64_t* ticket);

/* *done = 1 once the request has finished (or failed or was cancelled), else 0.
 * Errors: CC3_E_NOTFOUND (unknown or already collected ticket). */
int cc3_poll(cc3_server* srv, uint64_t ticket, int* done);

/* Block until the request has finished, then copy (or add, with
 * CC3_ACCUMULATE; device outputs only) its covariant result into
 * omega1[no][nv] and omega2[no][no][nv][nv] (either may be NULL to skip it)
 * and fill *timing (may be NULL).  Collects the ticket.  Returns the request's
 * own status: CC3_OK, CC3_E_CANCELLED, CC3_E_NOMEM (it could not be admitted
 * with nothing in flight), CC3_E_DEVICE; CC3_E_NOTFOUND for an unknown ticket. */
int cc3_wait(cc3_server* srv, uint64_t ticket, double* omega1, double* omega2,
             cc3_timing* timing);

/* Cancel a request that has not been admitted yet (cc3_wait then returns
 * CC3_E_CANCELLED).  Errors: CC3_E_NOTFOUND; CC3_E_BUSY if it already runs. */
int cc3_cancel(cc3_server* srv, uint64_t ticket);

/* Packing of small requests into shared launches.  When a slot admits a request
 * of at most max_request_flops nominal FLOP (4 nv^4 no^3), the requests queued
 * right behind it that are as small and have the same precision (up to max_pack
 * in all) join it: the group runs on the slot's stream, batch s of every request
 * in the same launches (one persistent kernel per step of the triple loop, whose
 * workgroups loop over the union of the requests' work items), and completes
 * together.  Each request keeps its own plan, batches and reduction order, so its
 * result is bit for bit the result it has alone.  Defaults: max_pack 8,
 * max_request_flops 2e12; max_pack 1 turns packing off.
 * Errors: CC3_E_INVAL (max_pack outside [1, 64], max_request_flops < 0). */
int cc3_server_set_packing(cc3_server* srv, int max_pack, double max_request_flops);

/* Counters of the server since creation.  Errors: CC3_E_INVAL. */
int cc3_server_get_stats(cc3_server* srv, cc3_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* CC3_H */
