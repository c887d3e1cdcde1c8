/*
 * nze.h -- C-ABI of the MI355X (gfx950) library for non-zero noise
 * extrapolation with vectorised matrix-product operators.
 *
 * Reference: A. P. Thompson, A. Soeteman, C. Cade, I. Niesen, "Non-zero noise
 * extrapolation: accurately simulating noisy quantum circuits with tensor
 * networks" (arXiv 2501.13237).
 *
 * Problem statement the calls follow (Sec. 2.1.2 "Setup", Sec. 2.2.1,
 * Sec. 2.2.2): a circuit is a sequence of noisy two-qubit gates (subcircuits)
 * acting on a product initial state; every gate U is followed by a channel C
 * of a one-parameter noise family (U -> C o U); the state is emulated as a
 * vectorised MPO of bond dimension at most D ("chi_max" here) at several noise
 * strengths lambda; Pauli-string expectation values are read out together
 * with the emulation fidelity, then extrapolated in lambda to a target.
 *
 * Conventions shared by every call
 *  - Status: every call returns 0 on success or a negative NZE_E* code; no
 *    C++ exception crosses the ABI.  nze_last_error() gives a message for the
 *    most recent failure on the calling thread.
 *  - Ownership: the caller owns every host array and the device workspace.
 *    The library never keeps a caller host pointer past the return of a call.
 *  - Threads: a handle is not thread-safe; use one handle per host thread.
 *  - Pauli codes: 0 = I, 1 = X, 2 = Y, 3 = Z.  Two-qubit Pauli index
 *    P = 4 * p_left + p_right (left = lower site index).
 *  - Pauli-transfer matrix (PTM) of a two-qubit map E: R[P][Q] =
 *    Tr(P E(Q)) / 4, row-major 16 x 16, float64.  It acts on Pauli
 *    coordinates v_P = Tr(P rho).
 */
#ifndef NZE_H
#define NZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define NZE_OK 0
#define NZE_EINVAL (-1)   /* bad argument, shape, or unsorted/overlapping sites */
#define NZE_ENOMEM (-2)   /* workspace too small (also the admission refusal)   */
#define NZE_EHIP (-3)     /* HIP runtime error                                  */
#define NZE_ENOCONV (-4)  /* Jacobi SVD reached its sweep cap without converging */
#define NZE_EFIT (-5)     /* too few admissible points for any extrapolation    */
#define NZE_ENUM (-6)     /* NaN/Inf met in the state                           */

/* ------------------------------------------------------------- precision */
#define NZE_FP64 0   /* every contraction and rotation in float64            */
#define NZE_MIXED 1  /* float32 sites, blocks and MFMA contractions/rotations;
                        Jacobi rotation parameters, truncation decisions,
                        the refinement of every update (orthonormal factor,
                        projection, fidelities), norms and readout in
                        float64                                              */

/* ------------------------------------------------------------ fit methods */
#define NZE_POLY 0      /* least-squares polynomial in lambda                 */
#define NZE_EXP3 1      /* a exp(-b lambda) + c, unweighted MSE (Sec. 2.2.2 B) */
#define NZE_LOGLIN_W 2  /* weighted log-linear fit with criteria 2-3, falling
                           back to NZE_EXP3, then NZE_EFIT (Sec. 2.2.2 B,
                           App. B.2)                                           */

/* ----------------------------------------------------------------- noise */
/* One noise family attached after every two-qubit gate (Sec. 2.2.1).  All
 * parameters are multiplied by the level's scale factor.  Channels are
 * applied in the order: two-qubit depolarizing (App. C.2.1,
 * rho -> (1 - dep) rho + dep I/4), amplitude damping with gamma = ad on each
 * qubit, Pauli channel (px, py, pz) on each qubit. */
typedef struct nze_noise {
  double dep;
  double ad;
  double px, py, pz;
} nze_noise;

/* Builds the 16 x 16 PTM of the noisy gate C o U (Sec. 2.2.1: the unitary
 * acts first, then the channel): R = R_C * R_U with
 * R_U[P][Q] = Tr(P U Q U^dagger) / 4.
 *   u_re, u_im : 4 x 4 row-major real and imaginary parts of U (host).  The
 *                computational-basis index of U is 2 * bit_left + bit_right.
 *   noise      : channel parameters (host; NULL = noiseless).
 *   scale      : level factor multiplying every noise parameter.
 *   ptm_out    : 256 float64, row-major (host, caller-allocated).
 * Host-only, float64.  Returns NZE_EINVAL on NULL u_re/u_im/ptm_out or on
 * scaled parameters outside [0, 1]. */
int nze_build_ptm(const double* u_re, const double* u_im,
                  const nze_noise* noise, double scale, double* ptm_out);

/* PTM of a two-qubit gate followed by a general two-qubit Pauli channel
 * rho -> sum_s p_s s rho s (Sec. 2.2.1 noise families; e.g. the cat-qubit CX
 * of App. C.2 with error Z on the control 3 lambda, Z on the target
 * lambda / 2, ZZ lambda / 2).
 *   rates  : 16 float64, index 4 a + b for the error s_a (x) s_b on (left,
 *            right); p_s = lambda * rates[s] for s != 0 and the identity
 *            keeps the rest.  rates[0] is ignored.
 * Returns NZE_EINVAL on NULL arguments, negative rates or lambda, or
 * probabilities outside [0, 1]. */
int nze_build_ptm_pauli(const double* u_re, const double* u_im,
                        const double* rates, double lambda, double* ptm_out);

/* Folds a noisy single-qubit gate into a two-qubit PTM: the 2x2 unitary u
 * (row-major real / imaginary parts) followed by the single-qubit Pauli
 * channel with p_s = lambda * rates[s], s = X, Y, Z at rates[1..3]
 * (rates[0] ignored; e.g. the cat-qubit Z(theta): Z lambda; H: Z 3 lambda,
 * X 2 lambda), acting on qubit 0 (left) or 1 (right) of the pair, applied
 * after (after != 0) or before the gate of ptm_in.  ptm_out may equal ptm_in.
 * Exact composition: valid when nothing else acts on that qubit in between.
 * Returns NZE_EINVAL as nze_build_ptm_pauli, or for qubit not 0/1. */
int nze_ptm_compose_1q(const double* ptm_in, const double* u_re,
                       const double* u_im, const double* rates, double lambda,
                       int32_t qubit, int32_t after, double* ptm_out);

/* ptm_out = second * first: the channel `first` followed by `second` on the
 * same pair, as one subcircuit (Sec. 2.1.2 allows any partition into
 * subcircuits).  ptm_out may alias either input.  Host-only. */
int nze_ptm_compose(const double* first, const double* second, double* ptm_out);

/* The same channel with its two qubits exchanged:
 * out[4a + b][4c + d] = in[4b + a][4d + c] (the gate acting on (right, left)
 * of a pair).  ptm_out may equal ptm_in.  Host-only. */
int nze_ptm_swap_qubits(const double* ptm_in, double* ptm_out);

/* Routing of two-qubit gates on arbitrary qubit pairs onto the open chain by
 * noiseless nearest-neighbour exchanges (SWAP gates), for circuits on 2D
 * lattices laid out along the chain (Sec. 3 orders the lattice qubits
 * column- or row-major).  Logical qubit q starts on chain site q; for each
 * input gate g, in order, the qubit qb[g] is moved towards qa[g] by SWAPs
 * until the two are neighbours, then the gate is applied, then (restore != 0)
 * the same SWAPs in reverse order move it back.
 *   n        : chain length (>= 2); n_gates: input gates (>= 0).
 *   qa, qb   : n_gates logical qubit pairs, 0 <= qa, qb < n, qa != qb
 *              (qa is the first qubit of the gate's 4x4 matrix).
 *   restore  : nonzero to restore the layout after every gate (the final
 *              permutation is then the identity).
 *   max_ops  : capacity of the three output arrays.
 *   op_site  : left chain site s of each op, acting on sites (s, s+1).
 *   op_gate  : input gate index of the op, or -1 for a SWAP.
 *   op_flip  : 1 when qa of the gate sits on site s+1 (apply its PTM with
 *              the qubits exchanged, nze_ptm_swap_qubits), else 0.
 *   n_ops    : number of ops of the routed sequence (also on NZE_ENOMEM).
 *   perm_out : NULL or n entries: chain site of each logical qubit after the
 *              last op (Pauli strings are read out through it).
 * The three op arrays may be NULL together to query n_ops (NZE_OK).
 * Host-only.  Errors: NZE_EINVAL (bad sizes or qubits), NZE_ENOMEM (op
 * arrays given and max_ops < n_ops). */
int nze_route_chain(int32_t n, int32_t n_gates, const int32_t* qa, const int32_t* qb,
                    int32_t restore, int32_t max_ops, int32_t* op_site, int32_t* op_gate,
                    uint8_t* op_flip, int32_t* n_ops, int32_t* perm_out);

/* ------------------------------------------------------------ MPO handle */
typedef struct mpo_handle mpo_t;

typedef struct mpo_config {
  int32_t n;           /* qubits on the open chain, 2 <= n <= 4096            */
  int32_t chi_max;     /* maximum bond dimension D (Sec. 2.1.1), 1..512        */
  int32_t n_levels;    /* L independent MPOs (one per noise level), >= 1      */
  int32_t precision;   /* NZE_FP64 or NZE_MIXED                               */
  double trunc_tol;    /* tau: drop s_i <= tau * s_1 (numerical zeros);
                          0 -> 1e-14 (FP64) / 1e-7 (mixed)                   */
  double tie_tol;      /* relative tie tolerance at a chi cut (a tied cluster
                          is dropped whole); 0 -> 1e-10 (FP64) / 1e-5 (mixed)*/
  double jacobi_tol;   /* relative off-diagonal threshold of the one-sided
                          Jacobi SVD: rows u, v count as orthogonal when
                          |<x_u,x_v>| <= tol |x_u||x_v| + jacobi_abs |X| |x_max|
                          (|X| Frobenius norm of the block, x_max the longer
                          of the two rows); tol is raised to at least
                          8 sqrt(C) eps (FP64, C = row length) or eps (mixed);
                          0 -> 1e-13 (FP64) / 3e-7 (mixed)                    */
  double jacobi_abs;   /* absolute part of that threshold;
                          0 -> 1e-15 (FP64) / 1e-9 (mixed)                    */
  int32_t max_sweeps;  /* Jacobi sweep cap (<= 40); 0 -> 40                   */
  int32_t block;       /* Jacobi row-block width b (pairs are 2b rows); the
                          kernels are built for b = 16.  16: the default
                          launch rules and schedule; 0: b = 16 with the
                          group size, kernel build and schedule of the tuning
                          record for (precision, chi_max, n_levels) when
                          nze_tune (or nze_tuning_set) made one, else the
                          defaults.  Other values: NZE_EINVAL                */
} mpo_config;

/* Device bytes the workspace of mpo_init must hold for cfg (0 if cfg is
 * invalid).  Also the footprint used for admission by HBM budget. */
size_t mpo_footprint(const mpo_config* cfg);

/* Creates L = cfg->n_levels MPOs in the same product state.
 *   out        : receives the handle (host).
 *   init_sites : n x 4 float64 Pauli coordinates (Tr(rho_k), Tr(X rho_k),
 *                Tr(Y rho_k), Tr(Z rho_k)) of the product state's sites
 *                (host), or NULL for |0...0> (each site (1, 0, 0, 1)).  The
 *                initial state is a product state (Sec. 2.1.2).
 *   workspace  : device memory of at least mpo_footprint(cfg) bytes, 256-byte
 *                aligned, owned by the caller and kept alive until mpo_free.
 *   stream     : hipStream_t on which all work of this handle is enqueued
 *                (NULL = the default stream).
 * Errors: NZE_EINVAL (bad cfg), NZE_ENOMEM (ws_bytes too small), NZE_EHIP. */
int mpo_init(mpo_t** out, const mpo_config* cfg, const double* init_sites,
             void* workspace, size_t ws_bytes, void* stream);

/* Releases the handle's host-side resources (not the caller's workspace).
 * Synchronises the handle's stream first.  NULL is a no-op. */
void mpo_free(mpo_t* h);

/* Applies one layer of noisy two-qubit gates to every level
 * (Sec. 2.1.2 "Approximate emulation"): for each gate the orthogonality
 * centre is moved next to it, the two site tensors are contracted, the PTM is
 * applied, the block is split by a truncated SVD to at most chi_max (the
 * closest fixed-bond-dimension state, renormalised to Frobenius norm 1), and
 * the partial fidelity (sum of kept s^2 / sum of all s^2) multiplies the
 * level's emulation fidelity (eq. emulation_fidelity).
 *   n_gates   : gates in the layer (>= 0).
 *   left_site : n_gates strictly increasing left sites; gate i acts on
 *               (left_site[i], left_site[i] + 1); pairs must be disjoint.
 *               Gates run in increasing order when left_site[0] is even and
 *               in decreasing order when it is odd (zig-zag sweep).
 *   ptm       : [n_levels][n_gates][16][16] float64 PTMs (host).
 * Asynchronous: returns once the inputs are staged; the work runs on the
 * handle's stream.  A Jacobi non-convergence or NaN is reported by the next
 * mpo_expect / mpo_stats / mpo_sync.  Errors: NZE_EINVAL, NZE_EHIP. */
int mpo_apply_layer(mpo_t* h, int32_t n_gates, const int32_t* left_site,
                    const double* ptm);

/* Several handles advanced by one layer each in the same device launches
 * (continuous batching of independent jobs).  All handles must share the
 * precision and the stream of hs[0]; arrays are indexed by handle.
 * Errors as mpo_apply_layer. */
int mpo_apply_layer_batch(mpo_t* const* hs, int32_t k, const int32_t* n_gates,
                          const int32_t* const* left_site,
                          const double* const* ptm);

/* Reads Pauli-string expectation values at every level.
 *   n_obs    : number of strings.
 *   paulis   : [n_obs][n] uint8 Pauli codes (host).
 *   values   : [n_levels][n_obs] float64 out: <P> = Tr(P rho) / Tr(rho)
 *              (trace-normalised, Sec. 2.1.2 footnote on normalisation).
 *   fidelity : [n_levels] float64 out, emulation fidelity (may be NULL).
 *   trace    : [n_levels] float64 out, Tr(rho) of the emulated (truncated,
 *              un-renormalised) state; 1 while nothing is truncated (NULL ok).
 * Synchronises the stream.  Errors: NZE_EINVAL, NZE_EHIP, NZE_ENOCONV,
 * NZE_ENUM (earlier asynchronous failures are reported here).  NZE_ENUM also
 * when a level's trace c_I is zero or a value is not finite, which happens
 * when the truncations removed the identity string (degenerate spectra of
 * Clifford states): values, fidelity and trace are still written. */
int mpo_expect(mpo_t* h, int32_t n_obs, const uint8_t* paulis, double* values,
               double* fidelity, double* trace);

typedef struct nze_stats {
  double fidelity;       /* emulation fidelity                               */
  double log_scale;      /* log of the factor removed by renormalisation      */
  double max_discarded;  /* max over gates of 1 - f                           */
  double min_cut_gap;    /* min over chi cuts of (s_r - s_{r+1}) / s_1        */
  int32_t max_bond;      /* largest current bond dimension                    */
  int32_t max_sweeps;    /* most Jacobi sweeps any SVD needed                 */
  int64_t updates;       /* two-site updates applied so far                   */
  int64_t sweeps_total;  /* Jacobi sweeps over all updates and centre moves   */
  double flops;          /* algorithmic flops executed so far: contraction
                            32 cl cm cr + superoperator 512 cl cr per update;
                            per Jacobi sweep on R rows of length C,
                            8 R^2 C (block Grams plus rotation of the data
                            rows; no accumulator); centre-move absorption
                            8 r cr c2.  The float64 refinement (Newton-Schulz,
                            projection, band polish) is not counted          */
  int64_t cap_hits;      /* SVDs that reached max_sweeps while every pair was
                            within 1000x the tolerance (the rounding floor);
                            beyond that mpo_expect/mpo_sync report
                            NZE_ENOCONV                                       */
  double cap_offdiag;    /* largest scaled off-diagonal, in units of the
                            tolerance, in the last sweep of any SVD that
                            reached max_sweeps (0 if none did)               */
  int64_t ns_scaled;     /* orthonormalisations of the float64
                            refinement whose start was too far from
                            orthonormal for the plain iteration (the scaled,
                            longer one was used)                              */
} nze_stats;

/* Per-level statistics (synchronises the stream).
 *   stats : [n_levels] out.   bonds : [n_levels][n-1] int32 out or NULL. */
int mpo_stats(mpo_t* h, nze_stats* stats, int32_t* bonds);

/* Diagnostics: time spent by workgroup 0 of each level in the phases of the
 * layer kernel, in milliseconds, [n_levels][16]: contraction, block Gram,
 * convergence test, LDS eigen-solve, rotation of the data, rotation of the
 * accumulator, barrier wait inside Jacobi, row norms, selection, absorption,
 * centre-move preparation, centre-move absorption, per-sweep overhead of the
 * Jacobi (row norms, re-sort, and the barriers that open and close a sweep),
 * then (not a time) the pair solves counted, then the mean barrier wait over
 * all workgroups, then whole-Jacobi time.
 * Synchronises the stream. */
int mpo_profile(mpo_t* h, double* ms_out);

/* Schmidt values across bond (l, l+1) of level lv (App. A.1: canonical form
 * at that bond; used for the MPO entanglement entropy), in decreasing order,
 * of the state normalised to unit Frobenius norm.  Values at or below
 * trunc_tol * s_1 are numerical zeros and are not reported.
 *   s_out : capacity cap float64 (host); the first min(count, cap) values
 *           are written and *count receives the number of values.
 * One launch of centre moves (no truncation beyond numerical zeros): the
 * orthogonality centre of every level of the handle ends at site l + 1.
 * Synchronises.  NZE_EINVAL for a bad level or bond. */
int mpo_bond_spectrum(mpo_t* h, int32_t lv, int32_t l, double* s_out,
                      int32_t cap, int32_t* count);

/* MPO entanglement entropy at bond (l, l+1) of level lv (App. A.1):
 * S_l = -sum_i p_i ln p_i with p_i = s_i^2 / sum_j s_j^2, over the Schmidt
 * values s_i that mpo_bond_spectrum reports (natural logarithm; 0 for a
 * product across the bond, ln k for k equal values).  The spectrum launch
 * moves the orthogonality centre as mpo_bond_spectrum does.  Synchronises.
 * Errors as mpo_bond_spectrum; NZE_ENUM for a zero or non-finite spectrum. */
int mpo_bond_entropy(mpo_t* h, int32_t lv, int32_t l, double* entropy);

/* True fidelity of eq. true_fidelity (Sec. 2.1.2) between two emulated
 * states: F = |<<a|b>>|^2 / (||a||^2 ||b||^2) for level la of handle a and
 * level lb of handle b (same n; any chi caps and precisions), e.g. a
 * truncated run against a run at a bond dimension that is exact (App. A.2
 * compares F with the emulation fidelity).  The overlaps are contracted site
 * by site in float64.  *overlap (NULL ok) receives the signed normalised
 * overlap <<a|b>> / (||a|| ||b||).  Synchronises both handles' streams and
 * uses the two-site scratch blocks of the handle with the larger chi cap, so
 * neither handle may have work queued on another stream meanwhile.
 * Errors: NZE_EINVAL, NZE_EHIP, NZE_ENUM (zero norm); deferred errors of
 * either handle. */
int mpo_overlap(mpo_t* a, int32_t la, mpo_t* b, int32_t lb, double* fidelity,
                double* overlap);

/* Waits for the handle's queued work and reports deferred errors
 * (NZE_ENOCONV, NZE_ENUM, NZE_EHIP). */
int mpo_sync(mpo_t* h);

/* -------------------------------------------------------- extrapolation */
typedef struct nze_fit_opts {
  int32_t degree;        /* NZE_POLY degree (default 2)                        */
  double delta_f;        /* weight exponent on fidelity (App. B.2, default 2)  */
  double delta_d;        /* weight exponent on distance (App. B.2, default 20) */
  double small;          /* criterion 2 threshold (default 1e-10)              */
  double dip_threshold;  /* fidelity defining the dip size (default 0.99)      */
  int32_t ref_sign;      /* criterion 3 reference sign: +1/-1, or 0 = sign of
                            the value at the smallest lambda                  */
  double b_max;          /* NZE_EXP3 upper bound on b; 0 -> 50 / lambda span  */
} nze_fit_opts;

/* Fills *opts with the defaults above. */
void nze_fit_opts_default(nze_fit_opts* opts);

/* Extrapolates <O>_lambda to lambda_target (Sec. 2.2.2 (B)).
 *   n_pts          : number of (lambda, value, fidelity) points.
 *   lambda, value  : n_pts float64 (host).
 *   fidelity       : n_pts float64 emulation fidelities (used by
 *                    NZE_LOGLIN_W weights; may be NULL otherwise).
 *   method         : NZE_POLY, NZE_EXP3 or NZE_LOGLIN_W.
 *   opts           : NULL for the defaults.
 *   out_value      : extrapolated value at lambda_target.
 *   out_coef       : 3 float64: POLY -> first min(3, degree+1) coefficients
 *                    c_0, c_1, c_2 (constant first); EXP3 -> (a, b, c);
 *                    LOGLIN_W -> (a, b, 0).  May be NULL.
 *   used_mask      : n_pts bytes, 1 for the points the final fit used (NULL
 *                    ok).
 *   method_used    : the method that produced out_value after fallbacks
 *                    (NULL ok).
 * Host-only, float64, stateless.  NZE_EFIT when no method has enough points:
 * the caller then falls back to the direct emulation at lambda_target. */
int nze_extrapolate(int32_t n_pts, const double* lambda, const double* value,
                    const double* fidelity, double lambda_target,
                    int32_t method, const nze_fit_opts* opts,
                    double* out_value, double* out_coef, uint8_t* used_mask,
                    int32_t* method_used);

/* Fidelity extrapolation, step (A) of Sec. 2.2.2: straight-line least squares
 * of value against fidelity over runs at increasing bond dimension, evaluated
 * at fidelity 1; *converged gets App. B.1's criterion 1 on the two last
 * points (NULL ok).  n_pts >= 2.  Host-only. */
int nze_fidelity_extrapolate(int32_t n_pts, const double* value,
                             const double* fidelity, double* out_value,
                             int32_t* converged);

/* --------------------------------------------------------------- serving */
/* A request loop over many extrapolation jobs (continuous batching).  Jobs
 * are admitted in arrival order when their mpo_footprint fits into free
 * space of a caller-owned device arena and a slot is free; admitted jobs stay
 * resident, and every nze_server_step advances all resident jobs by one layer
 * in shared persistent launches (at most 256 MPOs per launch).  A job that has
 * run all its layers is read out (mpo_expect) and its memory is released.
 * Because every MPO is computed by its own workgroups with the same
 * arithmetic, a job's results do not depend on which jobs share its launches.
 * The server is single-threaded; all work runs on `stream`. */
typedef struct nze_server nze_server_t;

typedef struct nze_job_spec {
  int32_t n, chi_max, n_levels, precision;  /* as in mpo_config               */
  int32_t n_layers;
  const int32_t* layer_gates;   /* [n_layers] gates in each layer              */
  const int32_t* left_sites;    /* the layers' left sites, concatenated (each
                                   layer as in mpo_apply_layer)               */
  const double* ptm;            /* the layers' PTMs, concatenated, each layer
                                   [n_levels][gates][16][16] float64         */
  int32_t n_obs;
  const uint8_t* paulis;        /* [n_obs][n] Pauli codes                     */
} nze_job_spec;

/* arena: 256-byte aligned device memory of arena_bytes, caller-owned.
 * max_active: most jobs resident at once. */
int nze_server_create(nze_server_t** out, void* arena, size_t arena_bytes,
                      int32_t max_active, void* stream);
void nze_server_free(nze_server_t* s);
/* Copies the job (host arrays); *job_id identifies it.  NZE_ENOMEM when the
 * job could never fit the arena. */
int nze_server_submit(nze_server_t* s, const nze_job_spec* spec, int64_t* job_id);
/* Admission, one batched layer for every resident job, read-out of finished
 * jobs.  Admission takes queued jobs in arrival order, first fit in the
 * arena; a job that does not fit yet may be passed by later jobs that do, in
 * at most 16 steps, after which nothing is admitted behind it until it fits.
 * Outputs (may be NULL): resident jobs, queued jobs, finished jobs. */
int nze_server_step(nze_server_t* s, int32_t* n_active, int32_t* n_queued,
                    int32_t* n_done);
/* state: 0 queued, 1 resident, 2 done, < 0 error code.  When done, values
 * [n_levels][n_obs] and fidelity [n_levels] are filled (NULL ok).  times[3]
 * (NULL ok): submit, admission and completion, seconds on the server clock. */
int nze_server_poll(nze_server_t* s, int64_t job_id, int32_t* state,
                    double* values, double* fidelity, double* times);
/* Highest arena offset in use so far (bytes) and launches issued. */
int nze_server_stats(nze_server_t* s, size_t* arena_high_water, int64_t* launches);

/* ------------------------------------------------------- kernel-level hooks */
/* Single kernels of the update on caller buffers, for kernel-level parity
 * tests.  All matrices are row-major device arrays in the path precision
 * (float64 for NZE_FP64, float32 for NZE_MIXED); the call synchronises
 * `stream` before returning.
 *
 * nze_kernel_theta: Theta' = (R x 1)(A B), the two-site contraction with the
 * gate's superoperator applied on the physical pair (Sec. 2.1.2 "Approximate
 * emulation"): A is (4 cl) x cm (site (cl, 4, cm)), B is cm x (4 cr) (site
 * (cm, 4, cr)), ptm is 256 float64 on the host.  X receives the
 * (4 cl) x (4 cr) block with rows (a, p') and columns (q', b) when ltr != 0,
 * or its transpose when ltr == 0.  1 <= cl, cm, cr <= 512.
 *
 * nze_kernel_rowortho: block one-sided Jacobi on the rows of X (R x C, C a
 * multiple of 4, row-major, in place) with the rotations accumulated into W
 * (R x R, overwritten; it starts as the identity): on return X holds
 * W X_in, whose rows are mutually orthogonal (their norms are the singular
 * values of X_in, in no particular order), and W is orthogonal.  norms
 * receives the R squared row norms of the result (host, float64).  *sweeps
 * gets the sweeps used (NULL ok).  Returns NZE_ENOCONV if max_sweeps were not
 * enough.  1 <= R <= 2048. */
int nze_kernel_theta(int32_t precision, int32_t cl, int32_t cm, int32_t cr,
                     const void* A, const void* B, const double* ptm,
                     int32_t ltr, void* X, void* stream);
int nze_kernel_rowortho(int32_t precision, int32_t R, int32_t C, void* X,
                        void* W, double tol_rel, double tol_abs,
                        int32_t max_sweeps, double* norms, int32_t* sweeps,
                        void* stream);

/* ------------------------------------------------------------------ tuner */
/* Launch and schedule parameters of the layer kernel for one batch shape
 * (precision, chi cap, MPOs per launch).  None changes the arithmetic of a
 * pair visit except the cross-block-only schedule, which changes the order of
 * the Jacobi rotations (results then agree within the path's tolerance, not
 * bitwise). */
typedef struct nze_tuning {
  int32_t block;             /* Jacobi row-block width b (16)                  */
  int32_t group_scale;       /* workgroups per MPO: 1 = the pairs of one Jacobi
                                round, 2 = twice that (rounds alternate between
                                two workgroup sets), when the CUs allow       */
  int32_t kernel;            /* 1 = one workgroup per CU, 2 = two per CU
                                (float kernel with scalar rotations)          */
  int32_t cross_sweeps;      /* early Jacobi sweeps whose pair solves take only
                                the cross-block rotations ...                 */
  int32_t cross_min_blocks;  /* ... in problems of at least this many blocks  */
  double ms_per_svd;         /* measured time per SVD of the tuning trial     */
} nze_tuning;

/* Device bytes nze_tune needs for (chi, precision, n_mpos). */
size_t nze_tune_footprint(int32_t chi, int32_t precision, int32_t n_mpos);

/* Measures the layer kernel on n_mpos synthetic saturated blocks of size
 * 4 chi x 4 chi (standard normal entries with row scales over four decades,
 * all blocks in one launch) for every candidate group size, kernel build and
 * cross-block schedule, twice each, and keeps the fastest (a candidate must
 * beat the previous best by 2 %).  The record is cached in the process for
 * (chi, precision, n_mpos) and written to *best.  MPOs created afterwards
 * with mpo_config.block = 0 and that shape take it (group size and kernel
 * build per launch; the schedule at mpo_init).  workspace: device memory of
 * nze_tune_footprint bytes, 256-byte aligned, caller-owned; stream as in
 * mpo_init.  Synchronises.  Errors: NZE_EINVAL, NZE_ENOMEM, NZE_EHIP,
 * NZE_ENOCONV. */
int nze_tune(int32_t chi, int32_t precision, int32_t n_mpos, void* workspace,
             size_t ws_bytes, void* stream, nze_tuning* best);

/* Reads (NZE_EINVAL when absent) or installs a cached tuning record, e.g.
 * one saved from an earlier process.  nze_tuning_set checks the fields. */
int nze_tuning_get(int32_t chi, int32_t precision, int32_t n_mpos, nze_tuning* out);
int nze_tuning_set(int32_t chi, int32_t precision, int32_t n_mpos, const nze_tuning* t);

/* nze_kernel_rowortho for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernel and results, but the Jacobi's
 * counters, barrier words, row norms and row order live in a static 64 KiB
 * array in each GPU's memory (held until the process ends) instead of the
 * scratch the library allocates on first use.  The call allocates nothing:
 * no hipMalloc, no pinned host memory; the host-side norms copy goes to the
 * caller's array.  The limit is the hook's: 1 <= R <= 2048 (NZE_EINVAL
 * beyond).  Every call on one GPU shares that GPU's array, whose first 8 KiB
 * are cleared by a fill kernel at the start of each call: calls that overlap
 * on one GPU (other streams or host threads) race and must be serialised by
 * the caller. */
int nze_kernel_rowortho_static(int32_t precision, int32_t R, int32_t C, void* X,
                               void* W, double tol_rel, double tol_abs,
                               int32_t max_sweeps, double* norms, int32_t* sweeps,
                               void* stream);

/* ------------------------------------------------------------------ misc */
/* Releases the library's internal device and pinned host buffers (launch
 * metadata staging, kernel-hook scratch) after waiting for the device.  For
 * an orderly process exit before the HIP runtime tears down; later calls
 * allocate them again.  Handles stay valid.  Not thread-safe against
 * concurrent calls of the library. */
void nze_shutdown(void);

const char* nze_strerror(int code);
const char* nze_last_error(void);
const char* nze_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NZE_H */
