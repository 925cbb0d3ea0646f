/*
 * mpsim.h -- C-ABI of the MI355X (gfx950) block-MPS Trotter evolution library.
 *
 * Method: arXiv:2511.23438. Trotterised time evolution of the periodic 2D
 * transverse-field Ising model (model section, eq. "hamiltonian", Trotter
 * step eq. "trotter_step") stored as a matrix product state whose sites are
 * half-row blocks of qubits (results section and the figure showing the
 * grouping of a 7x8 grid), with SVD truncation after every gate, the MPS
 * fidelity F_MPS tracked as the product of truncation fidelities, and the
 * fidelity-rescaled estimators of <Z_tot> (eq. "Z_tot_via_F") and <Z_tot^2>
 * (eq. "z2_tot_rescaled").
 *
 * Conventions shared by every call
 *   - grid R x C (rows x row length); qubit (r, c) has index q = r*C + c;
 *     Z|0> = +|0>;
 *   - block L_r = columns [0, ceil(C/2)) of row r, block R_r = the rest;
 *     block id = 2*r + side (0 = L, 1 = R); the fused index of a block has
 *     its first column as most significant bit; local dimension d = 2^width;
 *   - sites follow a row snake (even rows L,R; odd rows R,L);
 *   - site tensors live in device memory as row-major (b_p*d_p) x b_{p+1}
 *     matrices of interleaved complex numbers (re, im); on the host every
 *     complex array is interleaved double (re, im).
 *
 * Errors: every call returns an mps_status. Argument errors return
 * MPS_E_INVAL and change no state. MPS_E_NUMERIC (NaN/Inf or a failed
 * factorisation found on the device) and MPS_E_DEVICE (a HIP runtime error)
 * leave the handle failed: every later call on it returns MPS_E_STATE.
 * mps_last_error() returns a message for the last failing call.
 *
 * Threading: a handle is not thread-safe; distinct handles may be driven
 * from distinct threads on distinct streams.
 */
#ifndef MPSIM_H
#define MPSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_sim* mps_handle; /* opaque; owns all device memory of one instance */

typedef enum {
  MPS_OK = 0,
  MPS_E_INVAL = -1,       /* bad argument; nothing changed */
  MPS_E_NOMEM = -2,       /* device allocation failed; no handle created */
  MPS_E_DEVICE = -3,      /* HIP runtime error; handle failed */
  MPS_E_NUMERIC = -4,     /* NaN/Inf or factorisation failure on device; handle failed */
  MPS_E_STATE = -5,       /* handle already failed */
  MPS_E_UNSUPPORTED = -6  /* valid but unsupported configuration */
} mps_status;

typedef enum {
  MPS_FP64 = 0,            /* all contractions and the truncation in float64 */
  MPS_C64_FP32ACC = 1,     /* complex64 contractions, FP32 accumulation, FP64 truncation */
  MPS_BF16X3_FP32ACC = 2   /* three-term bf16 split (hi+mid+lo, 6 products), FP32 accumulation, FP64 truncation */
} mps_precision;

/* Optional device allocator (e.g. a framework's caching allocator). All
 * buffers of a handle are requested through alloc() on the handle's stream
 * and returned through free(). A NULL allocator makes the library use
 * hipMalloc/hipFree. alloc() returning NULL makes the call fail with
 * MPS_E_NOMEM. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} mps_allocator;

/* Gram side from which eig_path 0 takes the two-stage eigensolver (measured
 * crossover: the one-stage reduction is faster at 4096, the two-stage one
 * at 8192). */
#define MPS_EIG2_MIN 6144

typedef struct {
  int32_t rows, cols;      /* R x C; rows >= 1, 2 <= cols <= 8 (block width <= 4, d <= 16);
                              with layers >= 2 the cube's first two extents (>= 1) */
  int32_t chi_max;         /* maximum bond dimension, >= 1 */
  int32_t precision;       /* mps_precision */
  int32_t trotter_order;   /* 1: exp(-i dt H_X) exp(-i dt H_ZZ); 2: eq. "trotter_step" */
  int32_t schedule;        /* 1: wrap pairs routed by SWAPs and back (11R-12 updates/step);
                              2: rotating rows (7R-8 / 7R-7 updates/step, even / odd R);
                              3: route and return, any lattice: each coupled block pair in
                                 chain order, the far block swapped next to its partner,
                                 gated, swapped back;
                              4: gate by gate (the results section's own path): every ZZ
                                 bond between two blocks is a rank-2 matrix product
                                 operator that doubles the bonds between the blocks, then
                                 the doubled bonds are truncated one by one with the
                                 orthogonality centre on the bond; blocks never move.
                                 Site buffers are sized for the doubled bonds */
  int32_t periodic;        /* 1: periodic in both directions (the paper's TFIM); 0: open */
  int32_t eig_path;        /* truncation eigensolver: 0 automatic (two-stage from a Gram
                              side of MPS_EIG2_MIN on), 1 one-stage Householder
                              tridiagonalisation, 2 two-stage (dense -> band -> tridiagonal) */
  double J, h, dt;         /* couplings and time step of eq. "hamiltonian" */
  double theta0;           /* absolute angle of eq. "initial_state" */
  uint64_t seed;           /* seeds the start vectors of the eigensolver (deterministic) */
  int32_t layers;          /* 0 or 1: the rows x cols grid above, half-row blocks. >= 2: the
                              rows x cols x layers cubic lattice with one qubit per site
                              (d = 2, snake through the cube; schedule must be 3 or 4) */
  int32_t model;           /* 0: the transverse-field Ising model above. 1: the XY model of the
                              supplement's section "XY Model": H = (J/2) sum (XX + YY) on the
                              rows x cols grid with open boundaries (periodic must be 0,
                              layers 0), one qubit per site on a row snake, trotter_order 2
                              (the depth-7 split A/2 B/2 C/2 D C/2 B/2 A/2 of eq.
                              "xy_trotter_step"), schedule 3 (each bond routed and returned),
                              h ignored; the start state is eq. "xy_init" with tau = theta0:
                              the Neel state, round(J tau / 0.02 pi) (at least one when
                              tau > 0) Trotter steps of size tau / count, then
                              exp(-i pi/8 H_Z); their truncations count in F_MPS */
  int32_t eig_batch;       /* eigenvectors per band inverse-iteration launch of the two-stage
                              eigensolver: 0 means 1024, else 1..1024. That path keeps, per
                              vector in a launch, its band LU factors (99 complex per Gram
                              row: 26.6 GB for 1024 vectors at a Gram side of 16384, the
                              largest workspace of an instance); a smaller batch bounds
                              them at eig_batch * n * 99 * 16 bytes for more, narrower
                              launches. Results do not depend on it */
} mps_config;

typedef struct {
  int32_t step;            /* Trotter steps applied since init */
  int32_t eig_suspect;     /* truncations since init (or mps_set_state) whose kept weight |C|^2
                              and the sum of the kept Gram eigenvalues (bisection) differ by more
                              than 1e-9 |M|^2 (1e-5 with reduced-precision contractions): the
                              two agree whenever the eigenvectors span the top-q eigenspace, so
                              a nonzero count flags eigenvectors that did not converge */
  double z;                /* <Z_tot>_MPS, eq. "Z_tot" on the normalised MPS (XY model: the
                              conserved charge density <sum_j Z_j> / n) */
  double z2;               /* <Z_tot^2>_MPS, eq. "z2_tot" (XY model: the signal X2_tot of
                              eq. "xy_signal", staggered by the checkerboard sign) */
  double norm;             /* <psi|psi> of the stored MPS (1 up to rounding) */
  double fidelity;         /* F_MPS = product of all truncation fidelities */
  double log_fidelity;     /* log F_MPS (accumulated on the device in float64) */
  double z_rescaled;       /* F_MPS * <Z_tot>_MPS, eq. "Z_tot_via_F" */
  double z2_rescaled;      /* F_MPS^gamma * z2, eq. "z2_tot_rescaled" (XY: the rescaled
                              signal); NaN if gamma < 0 */
  double gamma;            /* the gamma used */
  double min_gap;          /* smallest relative gap (s_{q-1}-s_q)/s_0 at any truncation so far */
} mps_obs;

/* Create an instance in the product state of eq. "initial_state" (every qubit
 * cos(theta0/2)|0> + sin(theta0/2)|1>), all bonds 1, F_MPS = 1. Gate tables
 * (block-pair ZZ phases, intra-block phases, exp(-i h dt X) per block) are
 * built once here. Device memory for every site at its bond cap and for the
 * two-site workspaces is allocated here through `alloc` on `hip_stream`
 * (a hipStream_t; NULL = the null stream). On error *out is left NULL. */
mps_status mps_init_product(const mps_config* cfg, const mps_allocator* alloc,
                            void* hip_stream, mps_handle* out);

/* Apply `nsteps` >= 0 Trotter steps (Trotter step eq. "trotter_step", or its
 * first-order form) to the MPS. Every gate between two blocks is a diagonal
 * d_a x d_b phase on two neighbouring sites followed by an SVD truncation to
 * at most chi_max (results section: canonical form, truncation, unit norm
 * after each truncation, fidelity tracked separately); single-block gates
 * are applied site-locally. Asynchronous on the handle's stream. */
mps_status mps_apply_trotter_step(mps_handle h, int32_t nsteps);

/* Measure <Z_tot> and <Z_tot^2> of the current MPS with a transfer-matrix
 * sweep, and fill the fidelity-rescaled estimators (eqs. "Z_tot_via_F",
 * "z2_tot_rescaled") with the given gamma (gamma < 0: z2_rescaled = NaN).
 * Synchronises the handle's stream. */
mps_status mps_measure(mps_handle h, double gamma, mps_obs* out);

/* F_MPS(s) = product of the truncation fidelities of every gate application
 * so far (results section), and its logarithm. Synchronises. */
mps_status mps_fidelity(mps_handle h, double* fidelity, double* log_fidelity);

/* Release every device buffer of the handle. NULL-safe. */
void mps_free(mps_handle h);

/* ---------------- support: admission, diagnostics, tests ---------------- */

/* Device bytes that mps_init_product would allocate for cfg (admission). */
mps_status mps_footprint_bytes(const mps_config* cfg, size_t* bytes);

/* Schedule of `nsteps` steps from the initial snake order, as records of 6
 * int32: {kind, site, a, b, c, d}. kind 1 = two-site update:
 * {1, site, swap, gate, block at site, block at site+1}; kind 2 = single-site
 * gate: {2, site, variant, block, 0, 0} with variant 0 = U_X(h dt) D_intra,
 * 1 = D_intra U_X(h dt/2), 2 = U_X(h dt/2); kind 3 = ZZ gate as a rank-2
 * operator (schedule 4): {3, site_a, site_b, bit_a, bit_b, 0} with site_a <
 * site_b and bit j of each block's fused index (j = 0 the most significant).
 * *len receives the number of
 * int32 written (or needed, if cap is too small: then MPS_E_INVAL). Host only. */
mps_status mps_schedule_dump(const mps_config* cfg, int32_t nsteps, int32_t* ops,
                             int32_t cap, int32_t* len);

/* Current bond dimensions b_0..b_N (N+1 values, b_0 = b_N = 1). Host only. */
mps_status mps_bond_dims(mps_handle h, int32_t* dims, int32_t cap, int32_t* len);

/* Block id held by each site (N values). Host only. */
mps_status mps_site_blocks(mps_handle h, int32_t* blocks, int32_t cap, int32_t* len);

/* Singular values across bond `bond` (1..N-1), descending, computed on the
 * device with the same truncation machinery (no truncation). Moves the
 * orthogonality centre; the state is unchanged. Synchronises. */
mps_status mps_bond_spectrum(mps_handle h, int32_t bond, double* sv, int32_t cap,
                             int32_t* len);

/* Copy site p to the host: `re_im` gets b_p*d_p*b_{p+1} interleaved complex
 * values (row-major (b_p*d_p) x b_{p+1}); dims receives {b_p, d_p, b_{p+1}}.
 * Synchronises. */
mps_status mps_get_site(mps_handle h, int32_t p, double* re_im, int64_t cap,
                        int32_t* dims);

/* Replace the whole state: `bonds` = b_0..b_N (b_0 = b_N = 1, each within its
 * cap), `sites[p]` = host arrays laid out as in mps_get_site, `centre` = the
 * site carrying the norm (sites left of it left-orthonormal, right of it
 * right-orthonormal; the caller guarantees this). F_MPS is reset to 1 and
 * the step counter to 0. Block order stays the initial snake. */
mps_status mps_set_state(mps_handle h, const int32_t* bonds, const double* const* sites,
                         int32_t centre);

/* Apply one two-site update on sites (site, site+1): optional SWAP and
 * optional block-pair phase gate, then the truncation (diagnostic / test).
 * MPS_E_UNSUPPORTED on a schedule-4 handle (its buffers are sized for bond
 * truncations, not two-site contractions). */
mps_status mps_apply_two_site(mps_handle h, int32_t site, int32_t swap, int32_t gate);

/* As mps_apply_two_site, with the site of the next update as the hint the
 * step loop uses when both sides of theta have the same size: next_site >= 0
 * and < site keeps the orthogonality centre on `site` (the Gram matrix of
 * the columns is used), anything else moves it to site+1 (the rows). For
 * tests of both truncation sides. */
mps_status mps_apply_two_site_toward(mps_handle h, int32_t site, int32_t swap, int32_t gate,
                                     int32_t next_site);

/* Apply the single-site gate of the step schedule to site `site`: variant 0
 * = U_X(h dt) D_intra, 1 = D_intra U_X(h dt / 2), 2 = U_X(h dt / 2) (the
 * records of kind 2 in mps_schedule_dump; the gates inside one block, results
 * section) on the physical leg of the block the site holds. Unitary, so the
 * canonical form is kept and nothing is truncated. For driving a step op by
 * op (tests). MPS_E_INVAL for a bad site or variant, MPS_E_UNSUPPORTED for
 * the XY model (its single-site layers are part of its preparation only).
 * Asynchronous on the handle's stream. */
mps_status mps_apply_single_site(mps_handle h, int32_t site, int32_t variant);

/* Per-update truncation fidelities f and relative gaps since init (or
 * mps_set_state), in order; *len receives the count. Synchronises. */
mps_status mps_truncation_log(mps_handle h, double* f, double* gap, int32_t cap,
                              int32_t* len);

/* Dense state vector for n <= 20 qubits: 2^n interleaved complex values,
 * qubit q = r*C + c at bit n-1-q of the index. Synchronises. */
mps_status mps_to_statevector(mps_handle h, double* re_im, int64_t len);

/* Apply nsteps to each of `count` distinct handles: one host thread per
 * handle enqueues its steps on the handle's own stream, so the device runs
 * independent instances concurrently. Results equal applying the steps to
 * each handle alone. Returns when every step is enqueued (not completed);
 * MPS_E_INVAL for a NULL or repeated handle, otherwise the first failing
 * handle's status (each handle records its own error). */
mps_status mps_apply_trotter_step_batched(mps_handle* hs, int32_t count, int32_t nsteps);

/* Optional progress callback: called on the host after each two-site update
 * of mps_apply_trotter_step has been enqueued, with the index of the update
 * within the step and the number of updates per step. NULL removes it. */
typedef void (*mps_progress_fn)(void* ctx, int32_t step, int32_t update, int32_t updates_per_step);
mps_status mps_set_progress(mps_handle h, mps_progress_fn fn, void* ctx);

/* Synchronise the handle's stream and report any pending device error. */
mps_status mps_sync(mps_handle h);

/* Launch classes that mps_profile can time. */
typedef enum {
  MPS_PROF_OFF = 0,
  MPS_PROF_TRD_HEMV = 1,  /* Hermitian mat-vec of the tridiagonalisation; work = bytes of the
                             lower triangle read (16 B per complex element) */
  MPS_PROF_GRAM = 2,      /* Gram GEMM of the truncation; work = 8 flops per complex MAC of the
                             lower half */
  MPS_PROF_GEMM = 3,      /* every complex GEMM; work = 8 M N K flops (half when lower-only) */
  MPS_PROF_THETA = 4      /* two-site contraction with the gate epilogue; work = 8 M N K flops */
} mps_prof_kind;

/* Start timing every later launch of one class with HIP events recorded on
 * the handle's stream (kind 0 stops); resets the accumulated totals.
 * Diagnostic: adds two event records per timed launch. */
mps_status mps_profile(mps_handle h, int32_t kind);

/* Time only launches whose algorithmic work is at least min_work (>= 0;
 * default 0, every launch of the class); takes effect with the next
 * mps_profile call. */
mps_status mps_profile_min_work(mps_handle h, double min_work);

/* Accumulated device time (ms), number of timed launches and their
 * algorithmic work (bytes or flops, per the class). Synchronises. */
mps_status mps_profile_read(mps_handle h, double* total_ms, int64_t* launches, double* work);

/* The truncation's eigensolver on its own (results section: the kept
 * subspace of a bond is the top-q eigenspace of the Gram matrix of the
 * two-site block), for tests of the solver on chosen spectra. gram: host,
 * n x n Hermitian complex128, column-major (only the lower triangle is
 * read). eig_path: 1 one-stage (Householder tridiagonalisation), 2
 * two-stage (dense -> band -> tridiagonal); seed: start vectors of the
 * inverse iteration. Outputs (host): lam[0..q-1] the q largest eigenvalues,
 * descending; vecs the n x q row-major complex128 eigenvectors (column j
 * for lam[j], orthonormal columns). 1 <= q <= n. Allocates and frees its
 * own device workspace; synchronous on hip_stream (NULL: the default
 * stream). MPS_E_INVAL for bad arguments, MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_eigh_top(int32_t n, int32_t q, int32_t eig_path, uint64_t seed, const double* gram,
                        double* lam, double* vecs, void* hip_stream);

/* Operand extent checks (diagnostic, process-wide, off by default). While
 * enabled (enable != 0), every complex GEMM, reflector extraction, QR and
 * eigensolver launch is preceded by a host-side check that each operand's
 * first and last accessed element lie inside the one device buffer of the
 * library that holds its base address (the caller's site buffers count
 * during mps_measure_static). A failing check launches nothing and the call
 * returns MPS_E_DEVICE with a message naming the operand; the handle is then
 * failed. Host only; always MPS_OK. */
mps_status mps_debug_check_bounds(int32_t enable);

/* Last error message of the handle (thread-local message if h == NULL). */
const char* mps_last_error(mps_handle h);

#ifdef __cplusplus
}
#endif
#endif /* MPSIM_H */
