/*
 * esmf.h -- C ABI of libesmf, the MI355X (gfx950) library for the grouped
 * multi-density Fock build of excited-state mean-field (ESMF) theory
 * (Zhao & Neuscamman, arXiv:2002.00322).
 *
 * The operation (Sec. "Notation", Eq. J_and_K): for m generalised, not
 * necessarily symmetric, densities D_i and the two-electron integrals (pq|rs)
 * in chemists' (1122) notation,
 *
 *     J[D_i]_pq = sum_rs D_i[r][s] (rs|pq),   K[D_i]_pq = sum_rs D_i[r][s] (pr|qs),
 *
 * all m densities being served by one pass over the stored integrals
 * (Sec. "Shell-Pair Screening": several Fock matrices are built in a single
 * loop over the retained pairs, so the integrals are read once).  F = 2J - K
 * is left to the caller.
 *
 * Basis: N normalised s-type Gaussian primitives phi_p = n_p exp(-a_p |r-A_p|^2),
 * n_p = (2 a_p / pi)^(3/4); atomic units, coordinates in bohr.
 *
 * Screening (Sec. "Shell-Pair Screening", read as a Schwarz screen): with
 * Q_pq = sqrt((pq|pq)), the quartet (pq|rs) takes part iff Q_pq * Q_rs > tau,
 * the product taken in FP64.  tau = 0 keeps every quartet with a non-zero bound.
 * Pairs with Q_pq * max Q <= tau can never take part and are dropped.
 *
 * Conventions for every entry point:
 *   - Every function returns esmf_status.  ESMF_OK from a function that takes
 *     a stream means the work is enqueued on that stream; the results are
 *     valid once the stream has completed it.
 *   - Invalid arguments return ESMF_ERR_INVALID_ARG before anything is
 *     enqueued; outputs are untouched.  esmf_last_error() then holds a
 *     thread-local message.
 *   - Allocation failure returns ESMF_ERR_OUT_OF_MEMORY and leaves no partial
 *     object behind.
 *   - A HIP runtime failure returns ESMF_ERR_DEVICE.  A kernel fault surfaces
 *     as ESMF_ERR_DEVICE on a later call or when the caller synchronises.
 *   - "device" pointers are HIP device memory (e.g. torch.Tensor.data_ptr() of
 *     a contiguous float64 CUDA tensor); "host" pointers are ordinary memory.
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream).
 */
#ifndef ESMF_H
#define ESMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ESMF_OK = 0,
    ESMF_ERR_INVALID_ARG = -1,
    ESMF_ERR_OUT_OF_MEMORY = -2,
    ESMF_ERR_DEVICE = -3,
    ESMF_ERR_NOT_SUPPORTED = -4
} esmf_status;

/* Arithmetic of a build.
 * ESMF_PREC_FP64:    FP64 integrals, FP64 products and sums.
 * ESMF_PREC_MIXED:   FP32 integrals; each density is split D = D_hi + D_lo with
 *                    D_hi = fp32(D), D_lo = fp32(D - D_hi); the hi products run
 *                    on FP32 matrix cores with FP32 accumulation over chains of
 *                    2 steps (8 products), whose sums are accumulated in FP64;
 *                    the lo products (a correction of relative size 2^-24) on
 *                    BF16 matrix cores.  On an FP32 store the integrals are read
 *                    as stored; on an FP64 store each is rounded to FP32 as it is
 *                    loaded (the value an FP32 store holds, so the two give the
 *                    same bits).  Target: 1e-8 absolute on every J/K element for
 *                    the library's synthetic transition-density workloads.
 * ESMF_PREC_STORE32: FP32 integrals (half the integral stream), converted
 *                    exactly to FP64 where they enter the FP64 matrix cores:
 *                    products and sums in FP64, so the only error beyond FP64
 *                    rounding is the FP32 rounding of the stored values.  Same
 *                    matrix-core cost as the split (one FP64 product against
 *                    two FP32 ones) with fewer registers and half the LDS. */
typedef enum { ESMF_PREC_FP64 = 0, ESMF_PREC_MIXED = 1, ESMF_PREC_STORE32 = 2 } esmf_precision;

/* Storage of the screened integrals in HBM. FP64 builds need ESMF_STORE_FP64
 * or ESMF_STORE_DIRECT; STORE32 builds need ESMF_STORE_FP32; MIXED builds
 * read ESMF_STORE_FP32 or ESMF_STORE_FP64 (a mismatch is
 * ESMF_ERR_INVALID_ARG).
 * ESMF_STORE_DIRECT: integral-direct.  No integral store: the handle keeps
 *   the pair quantities (exponent sum, centre, prefactor, Schwarz factor) of
 *   all slot pairs and the block weights, O(N^2) bytes, and every build
 *   recomputes each kept integral inside the contraction, in FP64, with the
 *   same formula and screen as the stored paths.  This trades FP64 ALU work
 *   for the HBM that the integrals, the memory bottleneck of Sec. "Shell-Pair
 *   Screening", would take: molecules whose screened store does not fit can
 *   still be built.  Results equal those of an FP64 store up to rounding. */
typedef enum { ESMF_STORE_FP64 = 0, ESMF_STORE_FP32 = 1, ESMF_STORE_DIRECT = 2 } esmf_storage;

/* Opaque handle: owns the device-resident screened integral store and the
 * launch plan of one molecule.  Read-only during builds, so builds on
 * different streams may share it. */
typedef struct esmf_eri_s* esmf_eri_t;

typedef struct {
    int32_t nbf;                /* N */
    int32_t tile;               /* functions per tile of the block store */
    int64_t npairs;             /* N(N+1)/2 */
    int64_t npairs_kept;        /* pairs p >= q with Q_pq * max Q > tau */
    int64_t nquartets_kept;     /* unique (8-fold) quartets with Q_pq Q_rs > tau */
    int64_t nblocks;            /* stored tile-quartet blocks */
    int64_t nelements_stored;   /* integral slots held in HBM (zeros and row padding included) */
    int64_t device_bytes;       /* HBM held by the handle */
    int64_t workspace_bytes;    /* build workspace of a group of up to 8 densities (kept with the handle) */
    double q_max;               /* max Q_pq */
    double tau;                 /* screening threshold */
    int32_t storage;            /* esmf_storage */
    int32_t reserved;
    int64_t fp64_store_bytes;   /* bytes an ESMF_STORE_FP64 store of this block list holds (also
                                   reported by integral-direct handles, which hold none of it) */
    int64_t workspace_bytes_plan[2];  /* workspace_bytes under the two-visit [0] and the fused [1]
                                         work plan (workspace_bytes is that of the default plan) */
} esmf_eri_info;

/* Prepare the screened integral store of one molecule (Sec. "Shell-Pair
 * Screening": done once, at the start of an optimisation).
 *   nbf        N >= 1.
 *   centers    host [N][3] float64, bohr, finite.
 *   exponents  host [N] float64, finite and > 0.
 *   schwarz_tau  >= 0 and finite.
 *   storage    ESMF_STORE_FP64, ESMF_STORE_FP32 or ESMF_STORE_DIRECT.
 *   hip_stream stream on which the preparation kernels run; the call returns
 *              after the store is complete (it synchronises that stream).
 *   out        receives the handle; *out is NULL on failure.
 * Errors: INVALID_ARG (bad sizes/values/NULL), OUT_OF_MEMORY (the store does
 * not fit), DEVICE. */
esmf_status esmf_eri_prepare(int32_t nbf, const double* centers, const double* exponents,
                             double schwarz_tau, esmf_storage storage, void* hip_stream,
                             esmf_eri_t* out);

/* Prepare the store of a basis of Cartesian Gaussian functions with angular
 * momentum (the paper's basis sets have s, p and d shells, Sec.
 * "Computational Details"):
 *   phi_i(r) = N_i x^l y^m z^n exp(-a_i |r - A_i|^2), x = r_x - A_ix, ...,
 *   N_i = (2a/pi)^(3/4) (4a)^((l+m+n)/2) / sqrt((2l-1)!! (2m-1)!! (2n-1)!!),
 * i.e. each function normalised on its own (a shell's components are
 * separate functions with the same centre and exponent).
 *   lmn   host [N][3] int32: (l, m, n) of each function, each >= 0 and
 *         l + m + n <= 2 (s, p and d functions); read during the call.
 * Other arguments as esmf_eri_prepare.  The integrals over such functions are
 * computed at prepare time by the McMurchie-Davidson scheme (Hermite
 * expansion of the pair products, Hermite Coulomb integrals from the Boys
 * functions F_0..F_8); the screen is the same Schwarz test with
 * Q_ij = sqrt((ij|ij)).  Builds, batched builds and the tuner then work on
 * the store as for s functions.  Errors as esmf_eri_prepare, and
 * ESMF_ERR_NOT_SUPPORTED for ESMF_STORE_DIRECT with a function that is not
 * an s function (integral-direct builds recompute s-type integrals only). */
esmf_status esmf_eri_prepare_cart(int32_t nbf, const double* centers, const double* exponents,
                                  const int32_t* lmn, double schwarz_tau, esmf_storage storage,
                                  void* hip_stream, esmf_eri_t* out);

/* Prepare the store of a basis of contracted Cartesian functions (the
 * paper's cc-pVDZ and 6-31G* shells are fixed combinations of primitives):
 *   phi_i = N_i sum_{k in [prim_offset[i], prim_offset[i+1])} prim_coef[k] g_k,
 * g_k the normalised Cartesian primitive of esmf_eri_prepare_cart with
 * exponent prim_exp[k], the centre and powers of function i; N_i makes
 * <phi_i|phi_i> = 1 (computed here from the primitives' overlaps).
 *   lmn          host [N][3] int32, as for esmf_eri_prepare_cart.
 *   prim_offset  host [N+1] int32, prim_offset[0] = 0, 1..16 primitives each.
 *   prim_exp     host [prim_offset[N]] float64, finite and > 0.
 *   prim_coef    host [prim_offset[N]] float64, finite (coefficients of the
 *                normalised primitives).
 * Every integral is the coefficient-weighted sum over primitive quartets,
 * computed at prepare time; the screen is the Schwarz test on the contracted
 * functions.  Functions are grouped into tiles by their most diffuse
 * exponent.  Errors as esmf_eri_prepare_cart; ESMF_STORE_DIRECT takes only
 * s functions of one primitive of positive coefficient (those equal the
 * plain s functions of esmf_eri_prepare). */
esmf_status esmf_eri_prepare_contracted(int32_t nbf, const double* centers, const int32_t* lmn,
                                        const int32_t* prim_offset, const double* prim_exp,
                                        const double* prim_coef, double schwarz_tau, esmf_storage storage,
                                        void* hip_stream, esmf_eri_t* out);

/* Sizes and statistics of a handle (host struct). */
esmf_status esmf_eri_info_get(esmf_eri_t eri, esmf_eri_info* out);

/* Free a handle and its HBM.  NULL is accepted.  The caller must have
 * synchronised every stream that still uses the handle. */
esmf_status esmf_eri_release(esmf_eri_t eri);

/* Stored value of selected integrals, for verification (host arrays):
 * out[t] = (p q | r s) as held by the store for (p,q,r,s) = (p[t],q[t],r[t],s[t]),
 * 0 for a quartet the screen dropped.  Synchronous.  ESMF_ERR_NOT_SUPPORTED
 * for an integral-direct handle (it stores no integrals). */
esmf_status esmf_eri_lookup(esmf_eri_t eri, int64_t count, const int32_t* p, const int32_t* q,
                            const int32_t* r, const int32_t* s, double* out);

/* Grouped build (Eq. J_and_K for m densities in one pass over the store).
 *   m      >= 1 densities.
 *   d      device [m][N][N] float64 row-major, any (non-symmetric) D_i.
 *   j, k   device [m][N][N] float64 row-major, overwritten with J[D_i], K[D_i].
 *          They must not overlap d or each other.
 *   prec   ESMF_PREC_FP64 (needs FP64 or integral-direct storage),
 *          ESMF_PREC_MIXED (FP32 or FP64 storage) or ESMF_PREC_STORE32
 *          (FP32 storage).
 * Asynchronous on hip_stream.  The build's workspace (operand tiles and
 * partial sums, esmf_eri_info.workspace_bytes) is allocated with the first
 * build and kept with the handle until esmf_eri_release (grown when a wider
 * density group needs more; the growth waits for the handle's previous
 * builds).  Builds on one stream reuse it in stream order; a build on another
 * stream waits for the handle's previous build first, so builds of one handle
 * never overlap.  Results are bitwise reproducible: partial sums are reduced
 * in a fixed order, without atomics.  The contraction runs the handle's
 * variant (esmf_fock_tune); by default the two-visit work plan for stored
 * integrals and the fused plan (each integral evaluated once per build) for
 * integral-direct handles. */
esmf_status esmf_fock_build(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                            esmf_precision prec, void* hip_stream);

/* Grouped build with densities marked symmetric (Eq. J_and_K; the paper's
 * nine ESMF densities include two symmetric ones, Theta^T Theta and A, and
 * are all built in one loop over the retained pairs, Sec. "Shell-Pair
 * Screening").  Arguments as esmf_fock_build, plus
 *   symmetric  host [m] flags (nonzero: D_i is symmetric, D_i[p][q] ==
 *              D_i[q][p] for all p, q), or NULL (none), read during the call.
 * A non-symmetric density takes two of the contraction's 16 matrix-core
 * columns (D and D^T), a symmetric one takes one: the densities are packed in
 * order into groups of at most 16 columns and 16 densities, one pass over the
 * integrals per group, where esmf_fock_build makes groups of 8.  (Nine ESMF
 * densities with two symmetric ones: one pass instead of two.)  For exactly
 * symmetric flagged densities the results are bitwise those of
 * esmf_fock_build run on the same work plan (esmf_fock_tune); a group of
 * more than 8 densities always runs the two-visit plan, so against the
 * default fused plan they agree to rounding.  J is exact for any flagged
 * density; K of a flagged density that is not symmetric is unspecified.  A
 * group of more than 8 densities needs twice the J part of the workspace
 * (partial J tiles of 16 columns) and runs a contraction variant with a
 * 16-column J operand.  Errors as esmf_fock_build. */
esmf_status esmf_fock_build_sym(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                                esmf_precision prec, const uint8_t* symmetric, void* hip_stream);

/* The same build as esmf_fock_build without any device allocation, for
 * callers that cannot allocate (code under HIP stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The build workspace (unit table,
 * operand tiles, partial tiles) is a static array of 256 MiB of device memory
 * inside the library, one per device, held from the library's load until the
 * process ends; the handle's own workspace is not used.  Arguments, results
 * (bitwise those of esmf_fock_build with the handle's variant) and stream
 * semantics as esmf_fock_build; the handle must belong to the current device.
 * A build whose workspace exceeds the array (esmf_eri_info.workspace_bytes
 * plus a small unit table; e.g. the N = 200 chain fits, the N = 600 chain
 * does not) is refused with ESMF_ERR_INVALID_ARG before anything is
 * enqueued.  Every call
 * on a device uses the same array, and the array keeps the last call's
 * contents: calls that overlap on one device (different streams, or threads,
 * without ordering between them) race and give wrong results.  Nothing in the
 * array needs clearing between calls (each build writes all it reads). */
esmf_status esmf_fock_build_noalloc(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                                    esmf_precision prec, void* hip_stream);

/* Many independent molecules in one launch (device pointers per molecule;
 * the pointer arrays themselves are host arrays of length nmol).  Results
 * equal, bitwise, those of nmol calls of esmf_fock_build with the same
 * precision and variant (work plan, occupancy, skip).  Every argument of every molecule is validated before anything
 * is enqueued; an error names the molecule and leaves all outputs untouched.
 * FP64 batches are either all integral-direct or all stored (a mix is
 * ESMF_ERR_INVALID_ARG naming the first molecule that differs).
 *
 * The library keeps a plan per (handles, m values, precision, stream): a
 * device table of (molecule, density-group) units, their work items and
 * owned workspace, and, on a non-NULL stream, a HIP graph of the whole build
 * (table copy, operand prep, contraction with one workgroup per work item of
 * every molecule, reduction) that later calls replay.  The plan tunes itself
 * on its first call: the contraction variant (occupancy, skip) within the
 * default work plan, then, while none of the molecules has a tuned cut yet,
 * the work-item length, by cutting every molecule's plan again at half and
 * twice its length and timing the whole batch; the molecules' handles keep
 * the fastest cut (their single builds and later plans use it too; a cut set
 * by esmf_fock_tune or an earlier plan is kept).  The work-item stage waits
 * for the molecules' previous builds and drops other batched plans that use
 * them.  A call first waits on the host until the plan's previous
 * replay has finished (its pointer table is rewritten), then enqueues
 * asynchronously.  Up to four plans are cached (least recently used dropped);
 * esmf_eri_release drops every plan that uses the handle.  The workspace of
 * a plan is allocated with hipMalloc on its first call only. */
esmf_status esmf_fock_build_batched(int32_t nmol, const esmf_eri_t* eri, const int32_t* m,
                                    const double* const* d, double* const* j,
                                    double* const* k, esmf_precision prec, void* hip_stream);

/* Autotuner.  The contraction exists in variants:
 *   - the work plan: two visits of every block from its bra tile pair (runs
 *     of equal K, then of equal L; each block is read twice), or fused (one
 *     read of every block, all products on it; the bra's L values in bands of
 *     four whose accumulators stay in registers), both cut into work items
 *     of a number of blocks fixed when the store is prepared;
 *   - workgroups per CU the kernel is compiled for (register budget);
 *   - whether matrix-core fragments that read only absent granules (all-zero
 *     integrals) are skipped by a scalar test of the block's granule mask.
 * esmf_fock_tune times every variant on this handle's store (m densities,
 * scratch buffers from the library, one warm-up and the best of two timed
 * runs each), then cuts the fastest variant's plan again at half and twice
 * its work-item length and times those too (environment variable
 * ESMF_TUNE_ITEMS=0 skips this stage); the fastest becomes the handle's
 * variant for builds of that precision and its cut the handle's plan (the
 * cut is the handle's: the last tune of any precision sets it).  Variants of
 * one plan and cut give bitwise identical results; other plans and cuts sum
 * the same products in other orders (FP64 rounding apart).  Synchronous;
 * must not run while builds on the same handle are being enqueued (it waits
 * for the handle's builds and drops the batched plans that use it).  *out (optional) receives the table.  Batched plans tune
 * themselves the same way on their first call (environment variable
 * ESMF_TUNE=0 turns that off; esmf_fock_batched_report shows the result). */
typedef struct {
    int32_t candidates;            /* variants timed (<= 16) */
    int32_t chosen;                /* index of the fastest */
    int32_t plan[16];              /* 0: two visits per block, 1: fused */
    int32_t occupancy[16];         /* workgroups per CU of each variant */
    int32_t skip_zero[16];         /* 1 if the variant skips all-zero fragments */
    int32_t item_blocks[16];       /* blocks per work item of the variant's plan */
    double ms[16];                 /* best contraction time of each variant */
} esmf_tune_report;

esmf_status esmf_fock_tune(esmf_eri_t eri, int32_t m, esmf_precision prec, void* hip_stream,
                           esmf_tune_report* out);

/* What the calling thread's last successful esmf_fock_build_batched ran:
 * whether it replayed a captured HIP graph (graph = 1) or launched the
 * kernels directly (graph = 0: the NULL stream, or a stream that could not
 * be captured), the plan's units (molecule density groups) and work items,
 * the variant chosen by its tuner and the tuner's table.  Host struct;
 * ESMF_ERR_INVALID_ARG for NULL, ESMF_ERR_NOT_SUPPORTED before any batched
 * build on this thread. */
typedef struct {
    int32_t graph;
    int32_t units;
    int32_t items;
    int32_t plan;                  /* chosen variant: work plan, occupancy, skip */
    int32_t occupancy;
    int32_t skip_zero;
    int32_t candidates;            /* tuner table (0 when the tuner was off) */
    int32_t cand_plan[16];
    int32_t cand_occupancy[16];
    int32_t cand_skip_zero[16];
    double cand_ms[16];
    double item_factor;            /* chosen work-item length, as a factor of the cut at prepare time */
    int32_t item_candidates;       /* factors timed (1, 1/2, 2; 0 when that stage was off) */
    int32_t reserved;
    double item_factors[4];
    double item_ms[4];             /* contraction time of the whole batch at each factor */
} esmf_batch_report;

esmf_status esmf_fock_batched_report(esmf_batch_report* out);

/* ---- ESMF terms around the build ----------------------------------------
 * The nine generalised densities whose Fock matrices the analytic ESMF
 * derivatives need, in one call, so that all nine go through one grouped
 * build (Sec. "Shell-Pair Screening", the list of nine Fock builds; the
 * matrices are those of Table tab:notations):
 *   d[0] = Theta^T Theta              d[5] = Theta^T mu Gamma
 *   d[1] = Theta^T sigma Gamma        d[6] = Theta^T sigma Phi
 *   d[2] = A                          d[7] = Theta^T mu sigma^T Theta
 *   d[3] = R^T Theta                  d[8] = B
 *   d[4] = R^T sigma Gamma
 * with A = Gamma^T sigma^T sigma Gamma - Theta^T sigma sigma^T Theta and
 * B = Phi^T sigma^T sigma Gamma - R^T sigma sigma^T Theta.  (Table
 * tab:notations prints B's first term with Theta^T in place of Phi^T, which
 * does not conform; with Phi^T, B + B^T is the first-order change of A when
 * Theta and Gamma move along R and Phi, which is how B enters L_3 in the
 * Appendix, as R^T Theta and R^T sigma Gamma are the changes of the first two
 * densities.)
 *   nbf     N >= 1;  n_occ No >= 1;  n_virt Nv >= 1 (the paper has No + Nv = N;
 *           any sizes are accepted).
 *   theta   device [No][N], gamma [Nv][N], sigma and mu [No][Nv], r [No][N],
 *           phi [Nv][N]: float64, row-major (Theta, Gamma: first No and last Nv
 *           rows of V = U^T C; R, Phi: the same rows of W = M^T C).
 *   d       device [9][N][N] float64, overwritten; must not overlap the inputs.
 * Asynchronous on hip_stream; scratch (5 No N + 2 No^2 doubles) comes from a
 * stream-ordered pool of the library's own (kept apart from build
 * workspaces).  FP64 throughout, fixed summation order.  Errors:
 * INVALID_ARG (sizes, NULL), OUT_OF_MEMORY, DEVICE. */
esmf_status esmf_nine_densities(int32_t nbf, int32_t n_occ, int32_t n_virt, const double* theta,
                                const double* gamma, const double* sigma, const double* mu,
                                const double* r, const double* phi, double* d, void* hip_stream);

/* Two-body ESMF energy (Eq. esmf_energy_2b):
 *   E_2 = N2 F[D1].D1 + 4 c0 F[D1].D2 + 2 F[D1].A + 2 F[D2].D2,
 * F[D] = 2 J[D] - K[D], X.Y = sum_pq X_pq Y_pq, with D1 = Theta^T Theta,
 * D2 = Theta^T sigma Gamma and A as above.  The last term pairs F[D2] with D2:
 * the printed F[D2].D1 is linear in sigma, while the term comes from the block
 * of the energy quadratic in sigma (the Appendix's sigma-derivative of E has
 * the 4 Theta F[D2] Gamma^T that F[D2].D2 gives).
 *   d      device [>= 3][N][N]: D1, D2, A (the first three of esmf_nine_densities).
 *   j, k   device [>= 2][N][N]: J and K of D1 and D2 (e.g. of a build of d).
 *   n2, c0 N2 = c0^2 + 2 sum sigma^2 and c0, finite.
 *   e2     device pointer to one float64, written on hip_stream; it must
 *          not overlap d, j or k.
 * Asynchronous; deterministic (fixed reduction order).  Errors: INVALID_ARG,
 * OUT_OF_MEMORY, DEVICE. */
esmf_status esmf_energy_two_body(int32_t nbf, double n2, double c0, const double* d, const double* j,
                                 const double* k, double* e2, void* hip_stream);

/* The ESMF energy and its first derivatives (Eq. esmf_eng with E_1 of
 * Eq. esmf_energy_1b and E_2 of Eq. esmf_energy_2b as in
 * esmf_energy_two_body; the energy derivatives of the Appendix):
 *   E = (E_1 + E_2) / N2,  E_1 = G.(2 N2 D1 + 4 c0 D2 + 2 A),
 * and dE/dc0, dE/dsigma, dE/dTheta, dE/dGamma.  They are what the GVP
 * objective puts in place of the Lagrange multipliers (Sec. "Derivatives of
 * GVP-based Objective Function"): with mu = dE/dsigma, R = dE/dTheta and
 * Phi = dE/dGamma, esmf_nine_densities gives the six densities of the second
 * loop over the integrals.  (For an orbital-rotation multiplier M = dE/dX,
 * W = M^T C equals dE/dV when the rows of V are orthonormal and V is square.)
 * The Appendix prints the Theta-derivative with F[A] - F[A]^T and the
 * F[Theta^T sigma Gamma] terms garbled; these derivatives are derived from
 * E_1 and E_2 directly: 4 N2 Theta H + 4 c0 sigma Gamma H
 * - 4 sigma sigma^T Theta H + 4 c0 Theta (F2 + F2^T) + 2 Theta (FA + FA^T)
 * + 4 sigma Gamma F2^T over N2, with H = G + F1.
 *   nbf, n_occ, n_virt  N, No, Nv >= 1.
 *   c0, n2      c0 and N2 = c0^2 + 2 |sigma|^2 (finite, N2 > 0).
 *   theta [No][N], gamma [Nv][N], sigma [No][Nv]   device, as for
 *               esmf_nine_densities.
 *   g           device [N][N]: the one-electron matrix G (symmetric).
 *   d           device [>= 3][N][N]: D1, D2, A.
 *   j, k        device [>= 3][N][N]: J and K of D1, D2 and A.
 *   energy      device [4], written: E_1, E_2, E, dE/dc0.
 *   d_sigma [No][Nv], d_theta [No][N], d_gamma [Nv][N]   device, written.
 * Outputs must not overlap each other or the inputs.  Asynchronous on
 * hip_stream; scratch (4 N^2 + 5 No N + 2 No^2 + ~7200 doubles) comes from
 * the library's own stream-ordered pool.  FP64, fixed summation order
 * (deterministic).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
esmf_status esmf_energy_gradient(int32_t nbf, int32_t n_occ, int32_t n_virt, double c0, double n2,
                                 const double* theta, const double* gamma, const double* sigma, const double* g,
                                 const double* d, const double* j, const double* k, double* energy,
                                 double* d_sigma, double* d_theta, double* d_gamma, void* hip_stream);

/* Kernel timing (instrumentation).  While enabled on the calling thread, each
 * build records a pair of HIP events around its main contraction kernel(s) on
 * the build's own stream.  esmf_timing_collect waits for the recorded events,
 * returns the summed duration (ms) and the number of timed builds since the
 * previous collect, and releases the events.  Disabled by default. */
esmf_status esmf_timing_enable(int32_t enable);
esmf_status esmf_timing_collect(double* total_ms, int64_t* launches);

/* Measured peaks of the current device (instrumentation): the rates the
 * rooflines of the contraction divide by, next to the published ones. */
typedef struct {
    double fp64_mfma_tflops;    /* chains of v_mfma_f64_16x16x4f64 in registers, 8 waves per SIMD */
    double fp64_fma_tflops;     /* chains of FP64 vector FMAs, 8 waves per SIMD */
    double copy_tbps;           /* (bytes read + bytes written) / time of a streaming device copy */
    int32_t compute_units;      /* hipDeviceProp_t.multiProcessorCount */
    int32_t clock_mhz;          /* hipDeviceProp_t.clockRate (peak engine clock) */
} esmf_peaks;

/* Runs the three probe kernels on hip_stream (best of 3, 3 and 10 timed
 * launches after one warm-up each) and fills *out.  The copy moves
 * copy_bytes (1 MiB .. 64 GiB) from one device buffer to another; the
 * probe allocates and frees its own buffers (2 copy_bytes plus 2 MB per 256
 * compute units) and synchronises hip_stream.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
esmf_status esmf_probe_peaks(int64_t copy_bytes, void* hip_stream, esmf_peaks* out);

/* ---- Serving loop ---------------------------------------------------------
 * An ESMF optimisation asks for one grouped build per iteration over the same
 * integrals (Sec. "Shell-Pair Screening": the store is built once, then every
 * iteration's Fock builds loop over it).  A server keeps many such sessions'
 * stores resident in HBM, admits new sessions against an HBM budget by the
 * exact footprint of their store (unused cached workspace of the device's
 * stream-ordered pool is trimmed first), and serves build requests by continuous
 * grouping: a dispatcher thread takes pending requests in arrival order
 * (FIFO, so also FIFO within a session), forms a group of at most max_group
 * requests whose workspace fits in the largest free block of the server's
 * workspace arena (workspace_limit_bytes, allocated once at creation, so the
 * server's device memory is the stores plus the arena), and enqueues it as one grouped
 * launch (one operand prep, one contraction over the concatenated work lists,
 * one reduction) on the least loaded of nstreams streams, at most
 * max_inflight groups per stream, so that groups overlap on the device.  A
 * completion thread polls the groups' events.  Results equal, bitwise, those
 * of esmf_fock_build with the server's precision.  All calls are thread-safe.
 */
typedef struct esmf_server_s* esmf_server_t;

typedef struct {
    int32_t nstreams;              /* device streams, 1..16 */
    int32_t max_group;             /* requests per grouped launch, >= 1 */
    int32_t max_inflight;          /* grouped launches in flight per stream, >= 1 */
    esmf_precision prec;           /* precision of every build */
    esmf_storage storage;          /* FP64 or DIRECT with ESMF_PREC_FP64, FP32 with the others */
    int32_t reserved;
    int64_t hbm_budget_bytes;      /* cap on the summed footprint of resident stores */
    int64_t workspace_limit_bytes; /* workspace arena shared by the groups in flight */
} esmf_server_config;

typedef struct {
    int64_t budget_bytes;          /* hbm_budget_bytes of the config */
    int64_t resident_bytes;        /* summed footprint of open sessions */
    int32_t sessions_open;
    int32_t sessions_rejected;     /* admissions refused with ESMF_ERR_OUT_OF_MEMORY */
    int64_t requests_submitted;
    int64_t requests_completed;
    int64_t groups_launched;
    int64_t max_group_size;
} esmf_server_stats;

/* Create a server on the current device (its streams are non-blocking, at
 * the default priority).  ESMF_ERR_INVALID_ARG for a bad config. */
esmf_status esmf_server_create(const esmf_server_config* cfg, esmf_server_t* out);

/* Wait for every submitted request, stop the threads, release every open
 * session's store and the streams.  NULL is accepted. */
esmf_status esmf_server_destroy(esmf_server_t srv);

/* Admit a session: prepare its screened store (as esmf_eri_prepare, with the
 * server's storage) if its footprint fits in the budget left.  Returns
 * ESMF_ERR_OUT_OF_MEMORY, with nothing allocated, if it does not; in every
 * case *footprint_bytes (if not NULL) receives the footprint once known, so a
 * caller can tell "not now" (footprint <= budget) from "never".  Synchronous. */
esmf_status esmf_server_open_session(esmf_server_t srv, int32_t nbf, const double* centers,
                                     const double* exponents, double schwarz_tau,
                                     int32_t* session, int64_t* footprint_bytes);

/* Admit a session over a basis of contracted Cartesian functions (arguments
 * as esmf_eri_prepare_contracted; primitive functions are contractions of
 * length one): the screened store is prepared as esmf_eri_prepare_contracted
 * does, then admission and errors as esmf_server_open_session. */
esmf_status esmf_server_open_session_contracted(esmf_server_t srv, int32_t nbf, const double* centers,
                                                const int32_t* lmn, const int32_t* prim_offset,
                                                const double* prim_exp, const double* prim_coef,
                                                double schwarz_tau, int32_t* session, int64_t* footprint_bytes);

/* Wait for the session's outstanding requests, then release its store and
 * return its footprint to the budget. */
esmf_status esmf_server_close_session(esmf_server_t srv, int32_t session);

/* Queue one build (m densities, device pointers as in esmf_fock_build; the
 * caller keeps them alive and unmodified until esmf_server_wait returns).
 *   hip_stream  the producer stream (NULL = the legacy default stream): the
 *               call records an event on it, and the build waits for that
 *               event on the device, so it sees every write to d and every
 *               use of j and k enqueued on hip_stream before the call (e.g.
 *               the kernels that formed the densities).  Work on other
 *               streams must be ordered before the call by the caller.
 * Arguments are checked before anything is queued; a build whose workspace
 * exceeds the arena is refused with ESMF_ERR_OUT_OF_MEMORY.  Non-blocking
 * (no host synchronisation). */
esmf_status esmf_server_submit(esmf_server_t srv, int32_t session, int32_t m, const double* d,
                               double* j, double* k, void* hip_stream, int64_t* request);

/* Block until the request has completed on the device; *latency_ms (if not
 * NULL) receives submit-to-completion time on the host clock.  Returns the
 * request's own status.  Each request is waited for once. */
esmf_status esmf_server_wait(esmf_server_t srv, int64_t request, double* latency_ms);

esmf_status esmf_server_stats_get(esmf_server_t srv, esmf_server_stats* out);

const char* esmf_status_string(esmf_status s);

/* Thread-local detail of the last failure on the calling thread ("" if none). */
const char* esmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ESMF_H */
