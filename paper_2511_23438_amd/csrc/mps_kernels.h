// Element-wise and reduction kernels of the block-MPS update and measurement.
#pragma once
#include "common.h"

namespace mpsim {

// A[a, s, b] <- sum_t U[s, t] A[a, t, b] for a site of shape (b0, d, b1).
void launch_apply_u1(cplx* site, int b0, int d, int b1, const cplx* U, hipStream_t s);
// dst = one site of the rank-2 operator of exp(-i phi Z Z') on a span of
// sites (mode 0 first, 1 inside, 2 last); c = cos(phi), sn = sin(phi); the
// doubled bonds take index 2 * old + k
void launch_mpo_site(const cplx* src, cplx* dst, int b0, int d, int b1, int mode, int w, int bit,
                     double c, double sn, hipStream_t s);
// dense two-qubit gate G (4 x 4) on theta of two d = 2 sites, in place,
// SWAP of the physical indices folded into the store when swap is set
void launch_theta_gate4(cplx* theta, int b0, int b2, const cplx* G, int swap, hipStream_t s);
// measurement with sign * X on a d = 2 site (see launch_meas_combine)
void launch_meas_combine_x(cplx* X, int b, int b2, double sign, hipStream_t s);
// factored Gram weights and the oriented d x d phase table (see the kernel)
void launch_pair_weights(const cplx* table, int trans, int d, int side, cplx* W, cplx* Dfull,
                         hipStream_t s);
// rows ordered (s, a) -> (a, s): U[(a d + s) q + j] = Up[(s b0 + a) q + j]
void launch_unpermute_rows(const cplx* Up, cplx* U, int b0, int d, int q, hipStream_t s);
// *dst = sum_i Re G[i, i]
void launch_trace_real(const cplx* G, long n, long ldg, double* dst, hipStream_t s);
// dst[slot] = sum |x|^2 over len entries (deterministic two-pass reduction).
void launch_norm2(const cplx* x, long len, double* partial, double* dst, hipStream_t s);
// Truncation bookkeeping: f = sc[3]/sc[2], sc[0] += log f, sc[4] = 1/sqrt(sc[3]),
// log entry count[0] gets (f, gap) and count[0] is incremented; gap from the
// ascending eigenvalues lam (lam[extra .. extra+q-1]: the kept ones);
// count[1] is incremented when sc[3] and the kept eigenvalues' sum differ by
// more than tol * sc[2].
void launch_trunc_finalize(double* sc, double* flog, int* count, const double* lam, int q, int extra,
                           int* flag, double tol, hipStream_t s);
// x *= sc[4]
void launch_scale_by(cplx* x, long len, const double* sc, hipStream_t s);
// dst (cols x rows, ld ldd) = conj(src)^T, src rows x cols (ld lds)
void launch_conj_transpose(const cplx* src, int rows, int cols, long lds, cplx* dst, long ldd,
                           hipStream_t s);
// measurement: X holds 3 stacked blocks of b x (d*b2); Y1 = X1 + z X0,
// Y2 = X2 + 2 z X1 + z^2 X0 with z = zsum[s] on the physical index.
void launch_meas_combine(cplx* X, int b, int d, int b2, const double* zsum, hipStream_t s);
void launch_env_init(cplx* E, hipStream_t s);
void launch_fill(cplx* x, long len, cplx v, hipStream_t s);

}  // namespace mpsim
