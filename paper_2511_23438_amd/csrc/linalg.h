// Dense float64 linear algebra for the truncation step: Hermitian
// eigenvectors of the top-q eigenspace (Householder tridiagonalisation,
// bisection, inverse iteration, orthonormalisation, back-transformation) and
// Householder QR for moving the orthogonality centre.
#pragma once
#include "common.h"
#include "gemm.h"

namespace mpsim {

constexpr int TRD_NB = 32, QR_NB = 32, BT_NB = 64;

// Columns whose norm is below sqrt(DBL_MIN / DBL_EPSILON) ~ 1e-146 are taken
// as zero: the squares of their entries can underflow, so |x|^2 (a sum of
// squares) would understate the column and the reflector built from it
// would not be unitary (and a norm of 0 with alpha != 0 would divide by
// zero). Every matrix reduced here has a norm of order one or larger.
constexpr double REFLECTOR_FLOOR = 1.0010415475915505e-146;

// Reflector H = I - tau v v^H with v = [1; x*scale] such that
// H^H [alpha; x] = [beta; 0], beta real. A column below REFLECTOR_FLOOR is
// left as it is (tau = 0, beta = Re alpha).
__device__ inline void reflector(cplx alpha, double xnorm2, double& beta, cplx& tau, cplx& scale) {
  const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
  if ((xnorm2 == 0.0 && alpha.y == 0.0) || nrm < REFLECTOR_FLOOR) {
    beta = alpha.x;
    tau = make_double2(0.0, 0.0);
    scale = make_double2(0.0, 0.0);
    return;
  }
  beta = (alpha.x >= 0.0) ? -nrm : nrm;
  tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
  scale = cinv(make_double2(alpha.x - beta, alpha.y));
}


struct LinalgWork {
  long nmax = 0, qmax = 0, mmax = 0;  // eig dim, wanted count, QR rows
  cplx* W = nullptr;        // nmax x TRD_NB (col-major, ld nmax)
  cplx* tpart = nullptr;    // partial sums (column step reductions)
  long tpart_elems = 0;
  cplx* P = nullptr;        // Hermitian mat-vec partials, nt*nt*64
  long P_elems = 0;
  double* d = nullptr;      // tridiagonal diagonal (nmax)
  double* e = nullptr;      // off-diagonal (nmax)
  cplx* tau = nullptr;      // tridiagonalisation reflector scalars (nmax)
  cplx* qtau = nullptr;     // QR reflector scalars (max QR columns)
  double* e2 = nullptr;     // squared off-diagonal (nmax)
  cplx* dpart = nullptr;    // partial dot products (column steps)
  cplx* tsum = nullptr;     // reduced column-step sums (2*TRD_NB + 1)
  double* npart = nullptr;  // partial norms (QR column steps)
  double* scal = nullptr;   // 16 doubles of scalars
  double* lam = nullptr;    // eigenvalues (qmax + 1), ascending
  double* iwork = nullptr;  // inverse-iteration work, 6 * nmax * qmax
  cplx* T = nullptr;        // block reflector factors, (maxk/QR_NB + 1) * 64 * 64
  long T_elems = 0;
  cplx* S = nullptr;        // 64 x 64 scratch
  cplx* W1 = nullptr;       // 64 x wmax
  cplx* W2 = nullptr;       // 64 x wmax
  long wmax = 0;
  cplx* V = nullptr;        // clean reflector block, vmax x 64 (col-major)
  long vmax = 0;
  cplx* gpart = nullptr;    // split-K partials
  long gpart_elems = 0;
  int* flag = nullptr;      // numeric failure flag (device)
  // two-stage path
  cplx* T1 = nullptr;       // stage-1 panel block factors, (nmax/TRD_NB + 1) * 4096
  cplx* X2 = nullptr;       // nmax x 64 (row-major)
  cplx* S2 = nullptr;       // 64 x 64
  cplx* acc = nullptr;      // stage-1 reflectors of a panel group, he2hb_acc_elems(nmax)
  cplx* Ab = nullptr;       // band, nmax x (2*TRD_NB + 1), bulge-chased in place
  cplx* Br = nullptr;       // row-major copy of the band before chasing
  cplx* Ubuf = nullptr;     // inverse-iteration U rows, band_invit_work_elems()
  int invit_batch = 1024;   // vectors per band inverse-iteration launch
  // bulge-chasing launch sequences captured as HIP graphs, per (n, band)
  struct HbGraph {
    int n = -1;
    const cplx* ab = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  HbGraph hbg[2];
  int hbg_next = 0;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  Prof* prof = nullptr;     // optional launch timing
};

// Elements (r, c), r0 <= r < r0 + rows, c0 <= c < c0 + cols, of a strided
// matrix (element (r, c) at A[r*rs + c*cs], rs, cs >= 0) must lie in one
// buffer of the library (while operand checks are on; throws BoundsError).
void require_strided(const void* A, long rs, long cs, long r0, long c0, long rows, long cols,
                     const char* what);

// Reduce Hermitian A (n x n, column-major, lower triangle referenced) to real
// symmetric tridiagonal form A = Q T Q^H. T goes to w.d / w.e, reflectors
// stay in the strictly lower part of A (unit entry stored explicitly), their
// scalars in w.tau.
void hetrd_lower(int n, cplx* A, long lda, LinalgWork& w, hipStream_t s);

// Eigenvalues number lo..lo+cnt-1 (ascending, 0-based) of T by bisection.
void tridiag_eigvals(int n, int lo, int cnt, LinalgWork& w, hipStream_t s);

// Eigenvectors of T for the `q` largest eigenvalues (already in w.lam[1..q]
// when w.lam[0] holds the (q+1)-th largest, or w.lam[0..q-1] if has_extra=0)
// by inverse iteration; written as real values into X (n x q row-major,
// ld ldx), column j for the j-th largest eigenvalue.
void tridiag_invit(int n, int q, int lam_off, LinalgWork& w, cplx* X, long ldx, uint64_t seed,
                   hipStream_t s);

// X (n x q row-major) <- Q X with Q from hetrd_lower (reflectors in A).
void hetrd_backtransform(int n, const cplx* A, long lda, int q, cplx* X, long ldx,
                         LinalgWork& w, hipStream_t s);

// Householder QR of the m x k matrix with element (r, c) at A[r*rs + c*cs]
// (either rs == 1 or cs == 1), in place: R in the upper triangle,
// reflectors below, scalars in w.tau, block factors in w.T.
void qr_factor(int m, int k, cplx* A, long rs, long cs, LinalgWork& w, hipStream_t s);
// Explicit Q (m x kmin row-major, ld ldq) from a factored matrix.
void qr_form_q(int m, int k, const cplx* A, long rs, long cs, LinalgWork& w, cplx* Q, long ldq,
               hipStream_t s);
// R (kmin x k row-major, ld ldr) from a factored matrix.
void qr_get_r(int m, int k, const cplx* A, long rs, long cs, cplx* R, long ldr, hipStream_t s);

// Block reflectors (compact WY): V from the reflectors stored at
// A[(row0 + r)*rs + (col0 + j)*cs] into w.V, T into `T` (64 x 64 row-major);
// C <- (I - V op(T) V^H) C with op(T) = T or T^H (tconj).
void extract_v(const cplx* A, long rs, long cs, int row0, int col0, int mrows, int ib, cplx* V,
               long ldv, hipStream_t s);
void block_reflector(const cplx* A, long rs, long cs, int row0, int col0, int mrows, int ib,
                     const cplx* tau, cplx* T, LinalgWork& w, hipStream_t s);
void apply_block_reflector(int mrows, int ncols, int ib, const cplx* T, int tconj, cplx* C, long rs,
                           long cs, LinalgWork& w, hipStream_t s);

// Two-stage path (band.hip): dense -> band (half-width TRD_NB) by panel QR
// and two-sided MFMA updates, band -> tridiagonal by bulge chasing
// (eigenvalues), inverse iteration on the band, QR, back-transformation.
// Same contract as heev_top.
void heev_top_2stage(int n, cplx* G, long ldg, int q, cplx* U, long ldu, cplx* Xtmp, LinalgWork& w,
                     uint64_t seed, hipStream_t s);
// Elements of w.Ubuf for `q` vectors of side n, `batch` vectors per launch.
long band_invit_work_elems(long n, int q, int batch);
// Destroys the captured graphs and the capture stream of `w`.
void linalg_release(LinalgWork& w);
constexpr int BAND_W = 2 * TRD_NB + 1;
// stage-1 panels whose reflectors are accumulated before the trailing update
constexpr int HB_GROUP = 4;
// accumulated V and W (nmax x HB_GROUP*TRD_NB each, column-major) and the two
// small products of a panel with them
inline long he2hb_acc_elems(long nmax) {
  return 2 * nmax * HB_GROUP * TRD_NB + 2L * HB_GROUP * TRD_NB * TRD_NB;
}

// Top-q eigenspace of Hermitian G (n x n column-major, overwritten): an
// orthonormal basis U (n x q row-major, ld ldu) ordered by descending
// eigenvalue. `Xtmp` is an n x q scratch buffer. Eigenvalues
// (q + 1 largest if q < n, ascending) are left in w.lam.
void heev_top(int n, cplx* G, long ldg, int q, cplx* U, long ldu, cplx* Xtmp, LinalgWork& w,
              uint64_t seed, hipStream_t s);

}  // namespace mpsim
