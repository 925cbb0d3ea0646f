// Dense float64 linear algebra on gfx950 for the truncation step.
//
// The truncation of a two-site block needs an orthonormal basis of the top-q
// eigenspace of the Gram matrix G = M M^H (or M^H M). Every part runs on the
// device:
//   1. blocked Householder reduction of G to real tridiagonal T: per column a
//      reflector (with the panel's earlier reflectors applied on the fly) and
//      a Hermitian matrix-vector product on the lower-triangle tiles of the
//      trailing matrix; per panel of 32 columns a rank-64 update on MFMA;
//   2. bisection with Sturm counts for the wanted eigenvalues of T;
//   3. inverse iteration (tridiagonal LU with partial pivoting) for their
//      eigenvectors, one thread per vector;
//   4. Householder QR of the vectors (repairs orthogonality inside clusters
//      of close eigenvalues; only the spanned subspace matters);
//   5. back-transformation by the tridiagonalisation reflectors in blocks of
//      64 (compact WY form, MFMA GEMMs).
// Householder QR (panel column steps + WY trailing updates) also moves the
// orthogonality centre of the MPS.
#include "linalg.h"

#include <algorithm>
#include <cfloat>

namespace mpsim {

static ZOp strided_op(const cplx* base, long rs, long cs, int conj = 0) {
  if (cs == 1) return zop(base, rs, 0, conj);
  return zop(base, cs, 1, conj);
}

// ---------------------------------------------------------------------------
// Tridiagonalisation (lower), panels of TRD_NB columns. Per column c:
//   k_trd_col  : finish the previous column of the panel (alpha from its
//                partial dot products, scale its reflector, add alpha*v to
//                its W column), apply the panel's earlier reflectors to
//                column c, and partial sums of |x|^2, W^H x, V^H x;
//   k_trd_hemv : forms the reflector from those partials (every workgroup,
//                identically), then y = A22 v on the lower-triangle tiles of
//                the trailing matrix;
//   k_trd_w    : sums the tile partials of each row, subtracts the panel
//                corrections, scales by tau into the new W column, and
//                partial sums of y^H v.
// Hand-offs between workgroups happen only at kernel boundaries (device-scope
// fences cost a write-back of the per-XCD L2 on this part).
// scal: [0] beta [1,2] tau [3,4] scale of the latest column.
#define TP (2 * TRD_NB + 1)
// workgroups of the mat-vec kernel; each loops over tiles
constexpr int HEMV_WGS = 2048;

// alpha = -(tau/2) * sum of the partial dot products y^H v of the previous
// column, reduced by the whole workgroup (every thread must call it).
__device__ inline cplx trd_alpha(const double* scal, const cplx* dpart, int ndp, double* sh) {
  cplx ds = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < ndp; b += blockDim.x) ds = cadd(ds, dpart[b]);
  ds.x = block_sum(ds.x, sh);
  ds.y = block_sum(ds.y, sh);
  return cscale(cmul(make_double2(scal[1], scal[2]), ds), -0.5);
}

// One workgroup per 64 rows of column c; wave q owns the panel columns
// jj = q, q + 4, ... (their reflector and W entries stay in registers for
// both the update and the dot products).
__global__ __launch_bounds__(256) void k_trd_col(int n, cplx* A, long lda, cplx* W, long ldw, int i0,
                                                 int j, int c, const double* scal, const cplx* dpart,
                                                 int ndp, cplx* tpart) {
  __shared__ cplx wrow[TRD_NB], vrow[TRD_NB];
  __shared__ cplx part[4][64];
  __shared__ cplx abuf[64];
  __shared__ double dsh[4];
  const int t = threadIdx.x, lane = t & 63, q = t >> 6;
  const long r = c + (long)blockIdx.x * 64 + lane;
  const bool in = r < n;
  cplx a0 = make_double2(0.0, 0.0);
  if (q == 0 && in) a0 = A[(long)c * lda + r];
  const cplx alpha = (j > 0) ? trd_alpha(scal, dpart, ndp, dsh) : make_double2(0.0, 0.0);
  const cplx scp = make_double2(scal[3], scal[4]);
  if (t < j) {
    cplx wv = W[(long)t * ldw + c];
    if (t == j - 1) wv = cadd(wv, alpha);
    wrow[t] = cconj(wv);
    vrow[t] = (t == j - 1) ? make_double2(1.0, 0.0) : cconj(A[(long)(i0 + t) * lda + c]);
  }
  cplx vv[8], ww[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int jj = q + 4 * u;
    cplx v = make_double2(0.0, 0.0), w = make_double2(0.0, 0.0);
    if (in && jj < j) {
      if (jj == j - 1) {
        // the previous column: scale its reflector, add alpha v to its W
        if (r == c) {
          v = make_double2(1.0, 0.0);
          w = cadd(W[(long)jj * ldw + r], alpha);
        } else {
          v = cmul(A[(long)(c - 1) * lda + r], scp);
          A[(long)(c - 1) * lda + r] = v;
          w = cadd(W[(long)jj * ldw + r], cmul(alpha, v));
          W[(long)jj * ldw + r] = w;
        }
      } else {
        v = A[(long)(i0 + jj) * lda + r];
        w = W[(long)jj * ldw + r];
      }
    }
    vv[u] = v;
    ww[u] = w;
  }
  __syncthreads();
  cplx s = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int jj = q + 4 * u;
    if (jj < j) s = cadd(s, cadd(cmul(vv[u], wrow[jj]), cmul(ww[u], vrow[jj])));
  }
  part[q][lane] = s;
  __syncthreads();
  if (q == 0) {
    cplx a = csub(a0, cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane])));
    if (r == c) a.y = 0.0;
    if (in) A[(long)c * lda + r] = a;
    abuf[lane] = a;
  }
  __syncthreads();
  const cplx a = abuf[lane];
  const bool act = in && r >= c + 2;
  // values u < 8: conj(W[r, jj]) x, u >= 8: conj(V[r, jj]) x for jj = q + 4 (u mod 8);
  // reduced over the wave by a butterfly that halves the number of values
  // held per lane at each exchange (16 -> 1), then two plain exchanges
  cplx vals[16];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const bool ok = act && (q + 4 * u) < j;
    vals[u] = ok ? cmulc(ww[u], a) : make_double2(0.0, 0.0);
    vals[8 + u] = ok ? cmulc(vv[u], a) : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int half = 8, m = 32; half >= 1; half >>= 1, m >>= 1) {
    const bool upper = (lane & m) != 0;
#pragma unroll
    for (int q2 = 0; q2 < half; ++q2) {
      const cplx keep = upper ? vals[q2 + half] : vals[q2];
      const cplx send = upper ? vals[q2] : vals[q2 + half];
      cplx got;
      got.x = __shfl_xor(send.x, m, 64);
      got.y = __shfl_xor(send.y, m, 64);
      vals[q2] = cadd(keep, got);
    }
  }
  cplx z = vals[0];
  z.x += __shfl_xor(z.x, 2, 64);
  z.y += __shfl_xor(z.y, 2, 64);
  z.x += __shfl_xor(z.x, 1, 64);
  z.y += __shfl_xor(z.y, 1, 64);
  if ((lane & 3) == 0) {
    const int vid = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                    ((lane >> 2) & 1);
    const int jj = q + 4 * (vid & 7);
    if (jj < j) tpart[(long)blockIdx.x * TP + (vid < 8 ? 1 + jj : 1 + j + jj)] = z;
  }
  if (q == 0) {
    const double x2 = wave_sum(act ? cabs2(a) : 0.0);
    if (lane == 0) tpart[(long)blockIdx.x * TP] = make_double2(x2, 0.0);
  }
}

__device__ inline cplx trd_v(const cplx* A, long lda, int n, int c, long r, cplx sc) {
  if (r >= n) return make_double2(0.0, 0.0);
  if (r == c + 1) return make_double2(1.0, 0.0);
  return cmul(A[(long)c * lda + r], sc);
}

// y = A22 v over the lower-triangle tiles (64 x 64) of the trailing matrix;
// tile (I, J) writes A_IJ v_J to P[I][J] and, off the diagonal, A_IJ^H v_I to
// P[J][I]. Each workgroup forms the reflector once, then loops over tiles.
__global__ __launch_bounds__(256) void k_trd_hemv(int n, const cplx* A, long lda, int c, int j,
                                                     const cplx* tpart, int nparts, cplx* tsum,
                                                     double* scal, double* d, double* e, cplx* tau,
                                                     cplx* P, int nt, long ntiles) {
  __shared__ cplx vI[64], vJ[64];
  __shared__ cplx red[4][64];
  __shared__ cplx sc_s;
  const int t = threadIdx.x;
  const int lane = t & 63, wq = t >> 6;
  if (wq == 1) {
    // wave 1 of workgroup w reduces value 1 + w (+ grid multiples) of
    // W^H x and V^H x (values 1..2j) for the finalising kernel, while wave 0
    // forms the reflector
    for (int k = 1 + blockIdx.x; k <= 2 * j; k += gridDim.x) {
      cplx acc = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int b = lane; b < nparts; b += 64) acc = cadd(acc, tpart[(long)b * TP + k]);
      acc.x = wave_sum(acc.x);
      acc.y = wave_sum(acc.y);
      if (lane == 0) tsum[k] = acc;
    }
  }
  if (wq == 0) {
    // reflector of column c from |x|^2 (partials of the column kernel)
    double xn = 0.0;
#pragma unroll 4
    for (int b = lane; b < nparts; b += 64) xn += tpart[(long)b * TP].x;
    xn = wave_sum(xn);
    if (lane == 0) {
      double beta;
      cplx tauv, scl;
      reflector(A[(long)c * lda + c + 1], xn, beta, tauv, scl);
      sc_s = scl;
      if (blockIdx.x == 0) {
        scal[0] = beta; scal[1] = tauv.x; scal[2] = tauv.y; scal[3] = scl.x; scal[4] = scl.y;
        tau[c] = tauv;
        e[c] = beta;
        d[c] = A[(long)c * lda + c].x;
      }
    }
  }
  __syncthreads();
  const int o = c + 1;
  const cplx sc = sc_s;
  const int rr = lane, cg = wq;
#pragma unroll 1
  for (long k = blockIdx.x; k < ntiles; k += gridDim.x) {
    // tile order: column block J outer (descending), row block I inner, so
    // workgroups running together read neighbouring segments of the same 64
    // columns
    long a = (long)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > k) --a;
    while ((a + 1) * (a + 2) / 2 <= k) ++a;
    const long b = k - a * (a + 1) / 2;
    const long J = nt - 1 - a, I = nt - 1 - b;
    if (t < 64) vI[t] = trd_v(A, lda, n, c, o + I * 64 + t, sc);
    else if (t < 128) vJ[t - 64] = trd_v(A, lda, n, c, o + J * 64 + (t - 64), sc);
    __syncthreads();
    const long row = o + I * 64 + rr;
    cplx y = make_double2(0.0, 0.0);
    if (I == J) {
#pragma unroll 1
      for (int cc = 0; cc < 16; ++cc) {
        const int cl = cg * 16 + cc;
        const long col = o + J * 64 + cl;
        cplx av = make_double2(0.0, 0.0);
        if (row < n && col < n) {
          if (cl < rr) av = A[col * lda + row];
          else if (cl > rr) av = cconj(A[row * lda + col]);
          else av = make_double2(A[col * lda + row].x, 0.0);
        }
        y = cadd(y, cmul(av, vJ[cl]));
      }
    } else {
      const cplx vi = vI[rr];
#pragma unroll 1
      for (int g8 = 0; g8 < 2; ++g8) {
        cplx av[8];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const long col = o + J * 64 + cg * 16 + g8 * 8 + cc;
          av[cc] = (row < n && col < n) ? A[col * lda + row] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          y = cadd(y, cmul(av[cc], vJ[cg * 16 + g8 * 8 + cc]));
          av[cc] = cmulc(av[cc], vi);
        }
        // column sums over the 64 lanes: butterfly halving the values held
        // per lane (8 -> 1), then three plain exchanges
#pragma unroll
        for (int half = 4, m = 32; half >= 1; half >>= 1, m >>= 1) {
          const bool upper = (rr & m) != 0;
#pragma unroll
          for (int q2 = 0; q2 < half; ++q2) {
            const cplx keep = upper ? av[q2 + half] : av[q2];
            const cplx send = upper ? av[q2] : av[q2 + half];
            cplx got;
            got.x = __shfl_xor(send.x, m, 64);
            got.y = __shfl_xor(send.y, m, 64);
            av[q2] = cadd(keep, got);
          }
        }
        cplx z = av[0];
#pragma unroll
        for (int m = 4; m >= 1; m >>= 1) {
          z.x += __shfl_xor(z.x, m, 64);
          z.y += __shfl_xor(z.y, m, 64);
        }
        // lane rr holds the sum for column b3 + 2 b4 + 4 b5 of this group
        if ((rr & 7) == 0) {
          const int colid = ((rr >> 5) & 1) * 4 + ((rr >> 4) & 1) * 2 + ((rr >> 3) & 1);
          P[(J * nt + I) * 64 + cg * 16 + g8 * 8 + colid] = z;
        }
      }
    }
    red[cg][rr] = y;
    __syncthreads();
    if (t < 64) P[(I * nt + J) * 64 + t] = cadd(cadd(red[0][t], red[1][t]), cadd(red[2][t], red[3][t]));
  }
}

// One workgroup per 64-row block: wave q sums the tile partials J = q, q+4, ...
// of its rows and subtracts the panel corrections of columns jj = q, q+4, ...;
// wave 0 combines, scales by tau into the new W column and reduces y^H v.
__global__ __launch_bounds__(256) void k_trd_w(int n, const cplx* A, long lda, cplx* W, long ldw, int i0,
                                               int j, int c, const cplx* tsum,
                                               const cplx* P, int nt, const double* scal,
                                               cplx* dpart) {
  __shared__ cplx t1[TRD_NB], t2[TRD_NB];
  __shared__ cplx part[4][64];
  const int t = threadIdx.x;
  const int x = t & 63, q = t >> 6;
  const int o = c + 1;
  const cplx tauv = make_double2(scal[1], scal[2]);
  const cplx sc = make_double2(scal[3], scal[4]);
  if (t < 2 * j) {
    // W^H x (t < j) and V^H x (t >= j), reduced by the mat-vec's workgroup 0
    const cplx acc = tsum[1 + t];
    if (t < j) t1[t] = cadd(cconj(W[(long)t * ldw + o]), cmul(sc, acc));
    else t2[t - j] = cadd(cconj(A[(long)(i0 + t - j) * lda + o]), cmul(sc, acc));
  }
  const long I = blockIdx.x;
  const long r = o + I * 64 + x;
  const bool in = r < n;
  const cplx* Pr = P + I * nt * 64 + x;
  cplx s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
  long Jb = q;
  for (; Jb + 12 < nt; Jb += 16) {
    s0 = cadd(s0, Pr[Jb * 64]);
    s1 = cadd(s1, Pr[(Jb + 4) * 64]);
    s2 = cadd(s2, Pr[(Jb + 8) * 64]);
    s3 = cadd(s3, Pr[(Jb + 12) * 64]);
  }
  for (; Jb < nt; Jb += 4) s0 = cadd(s0, Pr[Jb * 64]);
  cplx av[8], wv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int jj = q + 4 * u;
    av[u] = (in && jj < j) ? A[(long)(i0 + jj) * lda + r] : make_double2(0.0, 0.0);
    wv[u] = (in && jj < j) ? W[(long)jj * ldw + r] : make_double2(0.0, 0.0);
  }
  cplx v = make_double2(0.0, 0.0);
  if (q == 0 && in) v = (r == o) ? make_double2(1.0, 0.0) : cmul(A[(long)c * lda + r], sc);
  __syncthreads();
  cplx s = cadd(cadd(s0, s1), cadd(s2, s3));
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int jj = q + 4 * u;
    if (jj < j) s = csub(s, cadd(cmul(av[u], t1[jj]), cmul(wv[u], t2[jj])));
  }
  part[q][x] = s;
  __syncthreads();
  if (q == 0) {
    cplx y = make_double2(0.0, 0.0);
    if (in) {
      y = cmul(tauv, cadd(cadd(part[0][x], part[1][x]), cadd(part[2][x], part[3][x])));
      W[(long)j * ldw + r] = y;
    }
    const cplx dt = cmulc(y, v);
    const double dre = wave_sum(dt.x);
    const double dim = wave_sum(dt.y);
    if (x == 0) dpart[blockIdx.x] = make_double2(dre, dim);
  }
}

// Last column of a panel: scale its reflector, store the unit entry and add
// alpha*v to its W column (rows c+1..n-1).
__global__ __launch_bounds__(256) void k_trd_finish(int n, cplx* A, long lda, cplx* W, long ldw, int j,
                                                    int c, const double* scal, const cplx* dpart,
                                                    int ndp) {
  __shared__ double dsh[4];
  const cplx alpha = trd_alpha(scal, dpart, ndp, dsh);
  const cplx sc = make_double2(scal[3], scal[4]);
  const long r = c + 1 + (long)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  cplx v;
  if (r == c + 1) v = make_double2(1.0, 0.0);
  else v = cmul(A[(long)c * lda + r], sc);
  A[(long)c * lda + r] = v;
  W[(long)j * ldw + r] = cadd(W[(long)j * ldw + r], cmul(alpha, v));
}

__global__ void k_trd_last(int n, const cplx* A, long lda, double* d) {
  d[n - 1] = A[(long)(n - 1) * lda + (n - 1)].x;
}

void hetrd_lower(int n, cplx* A, long lda, LinalgWork& w, hipStream_t s) {
  const long ldw = w.nmax;
  int ndp = 0;
  for (int i0 = 0; i0 < n - 1; i0 += TRD_NB) {
    const int ib = std::min(TRD_NB, n - 1 - i0);
    for (int j = 0; j < ib; ++j) {
      const int c = i0 + j;
      const int nb1 = ceil_div(n - c, 64);
      hipLaunchKernelGGL(k_trd_col, dim3(nb1), dim3(256), 0, s, n, A, lda, w.W, ldw, i0, j, c,
                         (const double*)w.scal, (const cplx*)w.dpart, ndp, w.tpart);
      const int np = n - c - 1;
      const int nt = ceil_div(np, 64);
      const long ntiles = (long)nt * (nt + 1) / 2;
      // at least 2j workgroups: each reduces some of the 2j column-step sums
      const unsigned grid = (unsigned)std::max<long>(std::min<long>(ntiles, HEMV_WGS), 2 * j);
      if (w.prof) w.prof->begin(PROF_TRD_HEMV, 16.0 * np * (np + 1.0) * 0.5, s);
      hipLaunchKernelGGL(k_trd_hemv, dim3(grid), dim3(256), 0, s, n, (const cplx*)A, lda, c, j,
                         (const cplx*)w.tpart, nb1, w.tsum, w.scal, w.d, w.e, w.tau, w.P, nt, ntiles);
      if (w.prof) w.prof->end(PROF_TRD_HEMV, 16.0 * np * (np + 1.0) * 0.5, s);
      hipLaunchKernelGGL(k_trd_w, dim3(nt), dim3(256), 0, s, n, (const cplx*)A, lda, w.W, ldw, i0, j, c,
                         (const cplx*)w.tsum, (const cplx*)w.P, nt, (const double*)w.scal,
                         w.dpart);
      ndp = nt;
    }
    const int cl = i0 + ib - 1;
    hipLaunchKernelGGL(k_trd_finish, dim3(ceil_div(n - cl - 1, 256)), dim3(256), 0, s, n, A, lda, w.W,
                       ldw, ib - 1, cl, (const double*)w.scal, (const cplx*)w.dpart, ndp);
    const int o2 = i0 + ib;
    if (o2 < n) {
      const int nn = n - o2;
      cplx* C = A + (long)o2 * lda + o2;
      // C -= [V W] [W V]^H  (one GEMM over a concatenated K of 2 ib)
      ZGemm g1 = zgemm_args(nn, nn, 2 * ib, zop(A + (long)i0 * lda + o2, lda, 1),
                            zop(w.W + o2, ldw, 0, 1), C, lda, 1, make_double2(-1.0, 0.0),
                            make_double2(1.0, 0.0));
      g1.kcat = ib;
      g1.A2 = zop(w.W + o2, ldw, 1);
      g1.B2 = zop(A + (long)i0 * lda + o2, lda, 0, 1);
      g1.lower_only = 1;
      zgemm(g1, nullptr, 0, s, w.prof);
    }
  }
  hipLaunchKernelGGL(k_trd_last, dim3(1), dim3(1), 0, s, n, (const cplx*)A, lda, w.d);
}

// ---------------------------------------------------------------------------
// Tridiagonal eigenvalues (bisection) and eigenvectors (inverse iteration)

// bounds[0] = Gershgorin lower, [1] = upper, [2] = norm estimate, [3] = pivmin
__global__ __launch_bounds__(256) void k_trd_prep(int n, const double* d, const double* e, double* e2,
                                                  double* bounds) {
  __shared__ double sh[8];
  double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    double ep = (i < n - 1) ? fabs(e[i]) : 0.0;
    lo = fmin(lo, d[i] - em - ep);
    hi = fmax(hi, d[i] + em + ep);
    if (i < n - 1) {
      e2[i] = e[i] * e[i];
      emax = fmax(emax, e[i] * e[i]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, lane_xch_bit(lo, off));
    hi = fmax(hi, lane_xch_bit(hi, off));
    emax = fmax(emax, lane_xch_bit(emax, off));
  }
  __shared__ double slo[4], shi[4], sem[4];
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { slo[w] = lo; shi[w] = hi; sem[w] = emax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      slo[0] = fmin(slo[0], slo[k]);
      shi[0] = fmax(shi[0], shi[k]);
      sem[0] = fmax(sem[0], sem[k]);
    }
    double tn = fmax(fabs(slo[0]), fabs(shi[0]));
    double pad = 2.0 * DBL_EPSILON * tn + 4.0 * DBL_MIN;
    bounds[0] = slo[0] - pad;
    bounds[1] = shi[0] + pad;
    bounds[2] = tn;
    bounds[3] = DBL_MIN * fmax(1.0, sem[0]);
    (void)sh;
  }
}

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) below x. The
// entries are read in blocks of SC (the same addresses in every lane, so the
// loads of a block are issued together and only the first waits), then the
// recurrence runs through the block; the arithmetic is that of a plain loop.
constexpr int SC = 16;
__device__ inline int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) <= pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  int i = 1;
  for (; i + SC <= n; i += SC) {
    double dd[SC], ee[SC];
#pragma unroll
    for (int u = 0; u < SC; ++u) {
      dd[u] = d[i + u];
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < SC; ++u) {
      q = dd[u] - x - ee[u] / q;
      if (fabs(q) <= pivmin) q = -pivmin;
      if (q < 0.0) ++cnt;
    }
  }
  for (; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) <= pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Multisection: one wave per wanted eigenvalue. Each round the 64 lanes
// evaluate Sturm counts at 64 interior points of the current interval and a
// ballot keeps the sub-interval that contains the eigenvalue, so the interval
// shrinks 65-fold per round.
__global__ __launch_bounds__(64) void k_bisect(int n, const double* d, const double* e2, int lo, int cnt,
                                               const double* bounds, double* lam) {
  const int k = blockIdx.x;
  if (k >= cnt) return;
  const int lane = threadIdx.x;
  const int idx = lo + k;
  double a = bounds[0], b = bounds[1];
  const double atol = DBL_EPSILON * bounds[2], pivmin = bounds[3];
  for (int it = 0; it < 64; ++it) {
    if (b - a <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + atol) break;
    const double x = a + (b - a) * (double)(lane + 1) / 65.0;
    const bool above = sturm_count(n, d, e2, x, pivmin) > idx;
    const unsigned long long mask = __ballot(above);
    // counts are monotone in x: the lanes above the eigenvalue form a suffix
    const int f = (mask == 0ULL) ? 64 : __ffsll((long long)mask) - 1;
    const double na = (f == 0) ? a : a + (b - a) * (double)f / 65.0;
    const double nb = (f == 64) ? b : a + (b - a) * (double)(f + 1) / 65.0;
    if (!(na > a || nb < b)) break;
    a = na;
    b = nb;
  }
  if (lane == 0) lam[k] = 0.5 * (a + b);
}

__device__ inline double hash_uniform(uint64_t seed, uint64_t a, uint64_t b) {
  uint64_t z = seed ^ (a * 0x9E3779B97F4A7C15ULL) ^ (b * 0xC2B2AE3D27D4EB4FULL);
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

// One thread per wanted eigenvector; factor arrays interleaved [i*q + kq] so
// that neighbouring threads touch neighbouring addresses. The recurrences of
// the factorisation and of the two triangular solves carry their running
// values in registers; memory holds only the factors and the vector.
__global__ __launch_bounds__(64) void k_invit(int n, const double* d, const double* e, int q,
                                              const double* lam, int lam_off, const double* bounds,
                                              double* work, cplx* X, long ldx, uint64_t seed) {
  const int kq = blockIdx.x * blockDim.x + threadIdx.x;
  if (kq >= q) return;
  const long nq = (long)n * q;
  double* fl = work;            // multipliers
  double* fd = work + nq;       // pivots (diagonal of U)
  double* fu = work + 2 * nq;   // first superdiagonal of U
  double* fu2 = work + 3 * nq;  // second superdiagonal of U
  double* xx = work + 4 * nq;   // vector
  double* pv = work + 5 * nq;   // 1 where rows i, i+1 were interchanged
#define AT(arr, i) arr[(long)(i) * q + kq]
  const double lmb = lam[lam_off + q - 1 - kq];
  double epsp = DBL_EPSILON * bounds[2];
  if (epsp == 0.0) epsp = DBL_MIN;
  // LU with partial pivoting of T - lmb I. Running row i: (di, ui) pending,
  // the next row's sub/diag/super come from d, e.
  double di = d[0] - lmb;
  double ui = (n > 1) ? e[0] : 0.0;
#pragma unroll 8
  for (int i = 0; i < n - 1; ++i) {
    const double li = e[i];
    const double dn = d[i + 1] - lmb;
    const double un = (i < n - 2) ? e[i + 1] : 0.0;
    if (fabs(di) >= fabs(li)) {
      const double fact = (di != 0.0) ? li / di : 0.0;
      AT(fl, i) = fact;
      AT(fd, i) = di;
      AT(fu, i) = ui;
      AT(fu2, i) = 0.0;
      AT(pv, i) = 0.0;
      di = dn - fact * ui;
      ui = un;
    } else {
      const double fact = di / li;
      AT(fl, i) = fact;
      AT(fd, i) = li;
      AT(fu, i) = dn;
      AT(fu2, i) = un;
      AT(pv, i) = 1.0;
      di = ui - fact * dn;
      ui = -fact * un;
    }
  }
  AT(fd, n - 1) = di;
  // The passes below read each chunk of IC rows into registers before any of
  // the chunk's stores (AT addresses depend on q, so the compiler cannot
  // move a load above an earlier store itself); every row is read before it
  // is written, and the arithmetic is that of the plain loops.
  constexpr int IC = 16;
  for (int i0 = 0; i0 < n; i0 += IC) {
    double v[IC];
#pragma unroll
    for (int u = 0; u < IC; ++u)
      if (i0 + u < n) v[u] = AT(fd, i0 + u);
#pragma unroll
    for (int u = 0; u < IC; ++u)
      if (i0 + u < n && fabs(v[u]) < epsp) AT(fd, i0 + u) = (v[u] < 0.0) ? -epsp : epsp;
  }
  for (int i = 0; i < n; ++i) AT(xx, i) = hash_uniform(seed, (uint64_t)kq, (uint64_t)i);
  for (int it = 0; it < 3; ++it) {
    // forward: apply the row interchanges and multipliers
    double cur = AT(xx, 0);
    for (int i0 = 0; i0 < n - 1; i0 += IC) {
      double nx[IC], fv[IC], pw[IC];
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n - 1) {
          nx[u] = AT(xx, i0 + u + 1);
          fv[u] = AT(fl, i0 + u);
          pw[u] = AT(pv, i0 + u);
        }
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n - 1) {
          if (pw[u] == 0.0) {
            AT(xx, i0 + u) = cur;
            cur = nx[u] - fv[u] * cur;
          } else {
            AT(xx, i0 + u) = nx[u];
            cur = cur - fv[u] * nx[u];
          }
        }
    }
    AT(xx, n - 1) = cur;
    // backward: upper triangular with two superdiagonals
    double x1 = AT(xx, n - 1) / AT(fd, n - 1);
    AT(xx, n - 1) = x1;
    double x2 = 0.0;
    if (n > 1) {
      const double v = (AT(xx, n - 2) - AT(fu, n - 2) * x1) / AT(fd, n - 2);
      AT(xx, n - 2) = v;
      x2 = x1;
      x1 = v;
    }
    double mx = fmax(fabs(x1), fabs(x2));
    for (int i1 = n - 3; i1 >= 0; i1 -= IC) {
      double xv[IC], uv[IC], u2[IC], dv[IC];
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i1 - u >= 0) {
          xv[u] = AT(xx, i1 - u);
          uv[u] = AT(fu, i1 - u);
          u2[u] = AT(fu2, i1 - u);
          dv[u] = AT(fd, i1 - u);
        }
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i1 - u >= 0) {
          const double v = (xv[u] - uv[u] * x1 - u2[u] * x2) / dv[u];
          AT(xx, i1 - u) = v;
          x2 = x1;
          x1 = v;
          mx = fmax(mx, fabs(v));
        }
    }
    if (!(mx > 0.0) || !isfinite(mx)) mx = 1.0;
    double s2 = 0.0;
    for (int i0 = 0; i0 < n; i0 += IC) {
      double xv[IC];
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n) xv[u] = AT(xx, i0 + u);
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n) {
          const double v = xv[u] / mx;
          s2 += v * v;
        }
    }
    double nrm = sqrt(s2);
    if (!(nrm > 0.0)) nrm = 1.0;
    const double sc = 1.0 / (mx * nrm);
    for (int i0 = 0; i0 < n; i0 += IC) {
      double xv[IC];
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n) xv[u] = AT(xx, i0 + u);
#pragma unroll
      for (int u = 0; u < IC; ++u)
        if (i0 + u < n) AT(xx, i0 + u) = xv[u] * sc;
    }
  }
  for (int i0 = 0; i0 < n; i0 += IC) {
    double xv[IC];
#pragma unroll
    for (int u = 0; u < IC; ++u)
      if (i0 + u < n) xv[u] = AT(xx, i0 + u);
#pragma unroll
    for (int u = 0; u < IC; ++u)
      if (i0 + u < n) X[(long)(i0 + u) * ldx + kq] = make_double2(xv[u], 0.0);
  }
#undef AT
}

void tridiag_eigvals(int n, int lo, int cnt, LinalgWork& w, hipStream_t s) {
  hipLaunchKernelGGL(k_trd_prep, dim3(1), dim3(256), 0, s, n, (const double*)w.d, (const double*)w.e,
                     w.e2, w.scal + 8);
  hipLaunchKernelGGL(k_bisect, dim3(cnt), dim3(64), 0, s, n, (const double*)w.d,
                     (const double*)w.e2, lo, cnt, (const double*)(w.scal + 8), w.lam);
}

void tridiag_invit(int n, int q, int lam_off, LinalgWork& w, cplx* X, long ldx, uint64_t seed,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_invit, dim3(ceil_div(q, 64)), dim3(64), 0, s, n, (const double*)w.d,
                     (const double*)w.e, q, (const double*)w.lam, lam_off,
                     (const double*)(w.scal + 8), w.iwork, X, ldx, seed);
}

// ---------------------------------------------------------------------------
// Block reflectors

// V (mrows x ib, column-major ld ldv): unit lower trapezoidal from the
// reflectors stored at A[row0 + rr, col0 + jj].
__global__ void k_extract_v(const cplx* A, long rs, long cs, int row0, int col0, int mrows, int ib,
                            cplx* V, long ldv) {
  const long total = (long)mrows * ib;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long rr = idx % mrows, jj = idx / mrows;
    cplx v;
    if (rr < jj) v = make_double2(0.0, 0.0);
    else if (rr == jj) v = make_double2(1.0, 0.0);
    else v = A[(row0 + rr) * rs + (col0 + jj) * cs];
    V[jj * ldv + rr] = v;
  }
}

void require_strided(const void* A, long rs, long cs, long r0, long c0, long rows, long cols,
                     const char* what) {
  if (rows <= 0 || cols <= 0) return;
  bounds_require(A, r0 * rs + c0 * cs, (r0 + rows - 1) * rs + (c0 + cols - 1) * cs, sizeof(cplx),
                 what);
}

void extract_v(const cplx* A, long rs, long cs, int row0, int col0, int mrows, int ib, cplx* V,
               long ldv, hipStream_t s) {
  require_strided(A, rs, cs, row0, col0, mrows, ib, "reflectors: source");
  require_strided(V, 1, ldv, 0, 0, mrows, ib, "reflectors: V");
  const long tv = (long)mrows * ib;
  const int bl = (int)std::min<long>((tv + 255) / 256, 2048);
  hipLaunchKernelGGL(k_extract_v, dim3(std::max(bl, 1)), dim3(256), 0, s, A, rs, cs, row0, col0, mrows,
                     ib, V, ldv);
}

// Forward column-wise block reflector factor: T upper (ib x ib, row-major
// ld 64, zero elsewhere in its 64 x 64 block) with H_0 ... H_{ib-1} =
// I - V T V^H, from S = V^H V and tau: T[i][i] = tau_i and, for j > i,
// T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] S[l][j]. Row i depends only on its
// own earlier entries and on S, so thread i forms it alone, with no barrier
// between columns: k_larft64 (ib <= 64) keeps the rows in LDS, k_larft
// (ib <= QR_NB) in registers.
__global__ __launch_bounds__(64) void k_larft64(int ib, const cplx* S, const cplx* tau, cplx* T) {
  __shared__ cplx Ts[64][65];
  __shared__ cplx Ss[64][65];
  __shared__ cplx ts[64];
  const int i = threadIdx.x;
  ts[i] = (i < ib) ? tau[i] : make_double2(0.0, 0.0);
  // column i of S, 16 loads in flight at a time
  for (int r0 = 0; r0 < 64; r0 += 16) {
    cplx sv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      sv[u] = (r0 + u < ib && i < ib) ? S[(r0 + u) * 64 + i] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      Ts[r0 + u][i] = make_double2(0.0, 0.0);
      Ss[r0 + u][i] = sv[u];
    }
  }
  __syncthreads();
  // thread i reads and writes only row i of Ts (and reads Ss): no barrier
  // between columns
  for (int j = 0; j < ib; ++j) {
    if (i < j) {
      cplx acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int l = i; l < j; ++l) acc = cadd(acc, cmul(Ts[i][l], Ss[l][j]));
      Ts[i][j] = cmul(cscale(ts[j], -1.0), acc);
    } else if (i == j) {
      Ts[i][i] = ts[i];
    }
  }
  __syncthreads();
  for (int r = 0; r < 64; ++r) T[r * 64 + i] = Ts[r][i];
}

__global__ __launch_bounds__(64) void k_larft(int ib, const cplx* S, const cplx* tau, cplx* T) {
  __shared__ cplx Ss[QR_NB][QR_NB + 1];
  __shared__ cplx ts[QR_NB];
  const int i = threadIdx.x;
  {
    // all 16 loads of this thread in flight at once
    cplx sv[QR_NB * QR_NB / 64];
#pragma unroll
    for (int u = 0; u < QR_NB * QR_NB / 64; ++u) {
      const int e = i + 64 * u, r = e / QR_NB, c = e % QR_NB;
      sv[u] = (r < ib && c < ib) ? S[r * 64 + c] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < QR_NB * QR_NB / 64; ++u) {
      const int e = i + 64 * u;
      Ss[e / QR_NB][e % QR_NB] = sv[u];
    }
  }
  if (i < QR_NB) ts[i] = (i < ib) ? tau[i] : make_double2(0.0, 0.0);
  __syncthreads();
  // row i of T: T[i][j] = -tau_j sum_{l = i .. j-1} T[i][l] S[l][j]; the
  // entries l < i of the row are exact zeros, so the sum runs over every
  // l < j without a lane-dependent bound (no branches in the unrolled loop)
  cplx row[QR_NB];
#pragma unroll
  for (int j = 0; j < QR_NB; ++j) {
    cplx acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < j; ++l) acc = cadd(acc, cmul(row[l], Ss[l][j]));
    cplx v = make_double2(0.0, 0.0);
    if (i < ib && j < ib) {
      if (j == i) v = ts[j];
      else if (j > i) v = cmul(cscale(ts[j], -1.0), acc);
    }
    row[j] = v;
  }
  // rows through LDS, so that the stores of one row are contiguous across lanes
  __syncthreads();
  if (i < QR_NB) {
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) Ss[i][c] = row[c];
  }
  __syncthreads();
  for (int r = 0; r < 64; ++r)
    T[(long)r * 64 + i] = (r < QR_NB && i < QR_NB) ? Ss[r < QR_NB ? r : 0][i < QR_NB ? i : 0]
                                                   : make_double2(0.0, 0.0);
}

void block_reflector(const cplx* A, long rs, long cs, int row0, int col0, int mrows, int ib,
                            const cplx* tau, cplx* T, LinalgWork& w, hipStream_t s) {
  const long ldv = w.vmax;
  require_strided(A, rs, cs, row0, col0, mrows, ib, "block reflector: source");
  require_strided(w.V, 1, ldv, 0, 0, mrows, ib, "block reflector: V");
  require_strided(T, 64, 1, 0, 0, ib, ib, "block reflector: T");
  long total = (long)mrows * ib;
  int blocks = (int)std::min<long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(k_extract_v, dim3(blocks), dim3(256), 0, s, A, rs, cs, row0, col0, mrows, ib,
                     w.V, ldv);
  // S = V^H V (ib x ib, ld 64)
  ZGemm g = zgemm_args(ib, ib, mrows, zop(w.V, ldv, 0, 1), zop(w.V, ldv, 1), w.S, 64, 0,
                       make_double2(1.0, 0.0), make_double2(0.0, 0.0));
  zgemm(g, w.gpart, w.gpart_elems, s, w.prof);
  if (ib <= QR_NB) hipLaunchKernelGGL(k_larft, dim3(1), dim3(64), 0, s, ib, (const cplx*)w.S, tau, T);
  else hipLaunchKernelGGL(k_larft64, dim3(1), dim3(64), 0, s, ib, (const cplx*)w.S, tau, T);
}

// Apply (I - V op(T) V^H) to the mrows x ncols block C (element (r, c) at
// C[r*rs + c*cs]); op(T) = T or T^H. V and T as built by block_reflector.
void apply_block_reflector(int mrows, int ncols, int ib, const cplx* T, int tconj,
                                  cplx* C, long rs, long cs, LinalgWork& w, hipStream_t s) {
  if (ncols <= 0 || mrows <= 0) return;
  const long ldv = w.vmax;
  const cplx one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  // W1 = V^H C (ib x ncols, ld wmax)
  ZGemm g1 = zgemm_args(ib, ncols, mrows, zop(w.V, ldv, 0, 1), strided_op(C, rs, cs), w.W1, w.wmax,
                        0, one, zero);
  zgemm(g1, w.gpart, w.gpart_elems, s, w.prof);
  // W2 = op(T) W1
  ZGemm g2 = zgemm_args(ib, ncols, ib, tconj ? zop(T, 64, 1, 1) : zop(T, 64, 0), zop(w.W1, w.wmax, 0),
                        w.W2, w.wmax, 0, one, zero);
  zgemm(g2, nullptr, 0, s, w.prof);
  // C -= V W2
  ZOp cop = strided_op(C, rs, cs);
  ZGemm g3 = zgemm_args(mrows, ncols, ib, zop(w.V, ldv, 1), zop(w.W2, w.wmax, 0), C, cop.ld,
                        cop.trans, make_double2(-1.0, 0.0), one);
  zgemm(g3, nullptr, 0, s, w.prof);
}

// ---------------------------------------------------------------------------
// Householder QR

// Column steps of the panel factorisation, one launch per column. The
// partial sums of column c (|x|^2 below the diagonal and the unscaled
// products sum_r conj(A[r,c]) A[r,jj] for the later columns jj of the panel)
// are reduced by every workgroup of the step; the reflector's scale is
// applied to the reduced sums, so the dot products v^H A[:,jj] need no second
// pass. The step then applies the reflector to its rows and forms the
// partial sums of column c+1 from the updated values it holds.
// Partial layout: one row of QR_NB values per workgroup (its four waves'
// sums added in LDS first, so the next step has a quarter as many rows to
// read); values 0..30 are the products, 31 holds |x|^2.

// butterfly over the 64 lanes of 32 complex values (halving the values held
// per lane at each exchange), then one plain exchange; lane l with (l & 1) == 0
// returns value b5*16 + b4*8 + b3*4 + b2*2 + b1 (bits of l)
__device__ inline cplx qr_butterfly(cplx vals[QR_NB], int lane, int& vid) {
#pragma unroll
  for (int half = QR_NB / 2, mm = 32; half >= 1; half >>= 1, mm >>= 1) {
    const bool upper = (lane & mm) != 0;
#pragma unroll
    for (int q2 = 0; q2 < half; ++q2) {
      // selected by value: a conditional between two array elements takes
      // an element's address, which would put the array in scratch memory
      const cplx keep = csel(upper, vals[q2], vals[q2 + half]);
      const cplx send = csel(upper, vals[q2 + half], vals[q2]);
      cplx got;
      got.x = __shfl_xor(send.x, mm, 64);
      got.y = __shfl_xor(send.y, mm, 64);
      vals[q2] = cadd(keep, got);
    }
  }
  cplx z = vals[0];
  z.x += __shfl_xor(z.x, 1, 64);
  z.y += __shfl_xor(z.y, 1, 64);
  vid = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
        ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
  return z;
}

// Each wave's butterfly result (lanes with (lane & 1) == 0 hold value vid)
// is added over the four waves in a fixed order; the workgroup writes its row
// of partials. Every thread must call it.
__device__ inline void qr_store_partials(cplx z, int vid, cplx (*wred)[QR_NB], cplx* part) {
  const int t = threadIdx.x;
  if ((t & 1) == 0) wred[t >> 6][vid] = z;
  __syncthreads();
  if (t < QR_NB)
    part[(long)blockIdx.x * QR_NB + t] = cadd(cadd(wred[0][t], wred[1][t]), cadd(wred[2][t], wred[3][t]));
}

// partial sums of the first column c of a panel (rows c+1 .. m-1)
__global__ __launch_bounds__(256) void k_qr_first(int m, const cplx* A, long rs, long cs, int c,
                                                  int pe, cplx* piv, cplx* part) {
  __shared__ cplx wred[4][QR_NB];
  const int t = threadIdx.x, lane = t & 63;
  // copy of the pivot row c (columns c .. pe-1) for the first column step
  if (blockIdx.x == 0 && t < QR_NB)
    piv[t] = (c + t < pe) ? A[(long)c * rs + (long)(c + t) * cs] : make_double2(0.0, 0.0);
  const long r = c + 1 + (long)blockIdx.x * 256 + t;
  const bool in = r < m;
  const cplx x = in ? A[r * rs + (long)c * cs] : make_double2(0.0, 0.0);
  cplx vals[QR_NB];
#pragma unroll
  for (int u = 0; u < QR_NB - 1; ++u) {
    const int jj = c + 1 + u;
    vals[u] = (in && jj < pe) ? cmulc(x, A[r * rs + (long)jj * cs]) : make_double2(0.0, 0.0);
  }
  vals[QR_NB - 1] = make_double2(cabs2(x), 0.0);
  int vid;
  const cplx z = qr_butterfly(vals, lane, vid);
  qr_store_partials(z, vid, wred, part);
}

// The pivot row c is read from piv, a copy written by the previous launch:
// workgroup 0 rewrites row c of A during this launch, so no other workgroup
// may read it there. The thread holding row c + 1 writes its updated values
// to piv_next for the next launch.
__global__ __launch_bounds__(256) void k_qr_col(int m, cplx* A, long rs, long cs, int c, int pe,
                                                const cplx* piv, const cplx* part, int nparts,
                                                cplx* piv_next, cplx* part_next, cplx* tau_out) {
  __shared__ cplx red[8][QR_NB];
  __shared__ cplx prow[QR_NB];
  __shared__ cplx wj[QR_NB];
  __shared__ double sh[5];
  const int t = threadIdx.x, lane = t & 63;
  const int ncol = pe - c - 1;  // later columns of the panel
  // every global value the step needs is requested first, so the loads of
  // the pivot row and of this thread's row overlap the reduction
  const long r = c + (long)blockIdx.x * 256 + t;
  const bool in = r < m;
  cplx a[QR_NB];  // this thread's row, columns c .. c + QR_NB - 1
#pragma unroll
  for (int u = 0; u < QR_NB; ++u)
    a[u] = (in && c + u < pe) ? A[r * rs + (long)(c + u) * cs] : make_double2(0.0, 0.0);
  cplx pr = make_double2(0.0, 0.0);
  if (t < QR_NB) pr = piv[t];
  {
    // reduce the partials: thread (g, u) sums parts g, g + 8, ... with 16
    // loads in flight per round (the partials come from every XCD, so the
    // reduction is bound by load latency; summation order as a plain loop)
    const int u = t & (QR_NB - 1), g = t >> 5;
    cplx acc = make_double2(0.0, 0.0);
    if (u < ncol || u == QR_NB - 1) {
      for (int p0 = g; p0 < nparts; p0 += 8 * 16) {
        cplx pv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int p = p0 + 8 * i;
          pv[i] = (p < nparts) ? part[(long)p * QR_NB + u] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) acc = cadd(acc, pv[i]);
      }
    }
    red[g][u] = acc;
  }
  if (t < QR_NB) prow[t] = pr;
  __syncthreads();
  if (t < QR_NB) {
    cplx sum = red[0][t];
    for (int g = 1; g < 8; ++g) sum = cadd(sum, red[g][t]);
    red[0][t] = sum;
  }
  __syncthreads();
  if (t == 0) {
    double beta;
    cplx tau, scl;
    reflector(prow[0], red[0][QR_NB - 1].x, beta, tau, scl);
    sh[0] = beta; sh[1] = tau.x; sh[2] = tau.y; sh[3] = scl.x; sh[4] = scl.y;
    if (blockIdx.x == 0) tau_out[c] = tau;
  }
  __syncthreads();
  const cplx sc = make_double2(sh[3], sh[4]);
  const cplx tau = make_double2(sh[1], sh[2]);
  if (t < ncol)  // v^H A[:, jj] = A[c, jj] + conj(scale) * sum_r conj(A[r,c]) A[r,jj]
    wj[t] = cadd(prow[t + 1], cmulc(sc, red[0][t]));
  __syncthreads();
  const cplx ctau = cconj(tau);
  cplx v = make_double2(0.0, 0.0);
  if (in) {
    v = (r == c) ? make_double2(1.0, 0.0) : cmul(a[0], sc);
    A[r * rs + (long)c * cs] = (r == c) ? make_double2(sh[0], 0.0) : v;
  }
#pragma unroll
  for (int u = 0; u < QR_NB - 1; ++u) {
    const int jj = c + 1 + u;
    cplx val = make_double2(0.0, 0.0);
    if (in && jj < pe) {
      val = csub(a[u + 1], cmul(ctau, cmul(v, wj[u])));
      A[r * rs + (long)jj * cs] = val;
    }
    a[u] = val;
  }
  if (c + 1 >= pe) return;
  if (r == c + 1) {
#pragma unroll
    for (int u = 0; u < QR_NB; ++u) piv_next[u] = (u < QR_NB - 1) ? a[u] : make_double2(0.0, 0.0);
  }
  // partial sums of column c + 1 over rows c+2 .. m-1
  const bool act = in && r >= c + 2;
  const cplx x = act ? a[0] : make_double2(0.0, 0.0);
  cplx vals[QR_NB];
#pragma unroll
  for (int u = 0; u < QR_NB - 1; ++u)
    vals[u] = (u + 1 < QR_NB - 1) ? cmulc(x, a[u + 1 < QR_NB - 1 ? u + 1 : 0]) : make_double2(0.0, 0.0);
  vals[QR_NB - 1] = make_double2(cabs2(x), 0.0);
  int vid;
  const cplx z = qr_butterfly(vals, lane, vid);
  // red is free again: its last reader (wj) is behind a barrier
  qr_store_partials(z, vid, red, part_next);
}

void qr_factor(int m, int k, cplx* A, long rs, long cs, LinalgWork& w, hipStream_t s) {
  const int kmin = std::min(m, k);
  require_strided(A, rs, cs, 0, 0, m, k, "QR: matrix");
  if (kmin > 0) {
    // the two (pivot row, partials) halves of the column steps
    const long nparts = std::max(1, ceil_div(m, 256));
    require_strided(w.tpart, 1, 0, 0, 0, w.tpart_elems, 1, "QR: column-step partials");
    if (2 * (QR_NB + nparts * QR_NB) > w.tpart_elems)
      throw BoundsError{"QR: column-step partials need " + std::to_string(2 * (QR_NB + nparts * QR_NB)) +
                        " elements, the buffer holds " + std::to_string(w.tpart_elems)};
  }
  // two buffers of (pivot row copy, partial sums), alternating between
  // column steps
  cplx* pivA = w.tpart;
  cplx* pivB = w.tpart + w.tpart_elems / 2;
  cplx* partA = pivA + QR_NB;
  cplx* partB = pivB + QR_NB;
  for (int p0 = 0, panel = 0; p0 < kmin; p0 += QR_NB, ++panel) {
    const int pe = std::min(p0 + QR_NB, kmin);
    const int nb0 = std::max(1, ceil_div(m - p0 - 1, 256));
    hipLaunchKernelGGL(k_qr_first, dim3(nb0), dim3(256), 0, s, m, (const cplx*)A, rs, cs, p0, pe, pivA,
                       partA);
    int nparts = nb0;
    for (int c = p0; c < pe; ++c) {
      const int nbr = ceil_div(m - c, 256);
      hipLaunchKernelGGL(k_qr_col, dim3(nbr), dim3(256), 0, s, m, A, rs, cs, c, pe, (const cplx*)pivA,
                         (const cplx*)partA, nparts, pivB, partB, w.qtau);
      std::swap(pivA, pivB);
      std::swap(partA, partB);
      nparts = nbr;
    }
    const int ib = pe - p0;
    cplx* T = w.T + (long)panel * 4096;
    block_reflector(A, rs, cs, p0, p0, m - p0, ib, w.qtau + p0, T, w, s);
    if (pe < k)
      apply_block_reflector(m - p0, k - pe, ib, T, 1, A + (long)p0 * rs + (long)pe * cs, rs, cs, w, s);
  }
}

__global__ void k_set_identity(int m, int k, cplx* Q, long ldq) {
  const long total = (long)m * k;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / k, c = idx % k;
    Q[r * ldq + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
}

void qr_form_q(int m, int k, const cplx* A, long rs, long cs, LinalgWork& w, cplx* Q, long ldq,
               hipStream_t s) {
  const int kmin = std::min(m, k);
  long total = (long)m * kmin;
  int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_set_identity, dim3(blocks), dim3(256), 0, s, m, kmin, Q, ldq);
  const int npanels = ceil_div(kmin, QR_NB);
  for (int panel = npanels - 1; panel >= 0; --panel) {
    const int p0 = panel * QR_NB, pe = std::min(p0 + QR_NB, kmin), ib = pe - p0;
    const cplx* T = w.T + (long)panel * 4096;
    long tv = (long)(m - p0) * ib;
    int bl = (int)std::min<long>((tv + 255) / 256, 2048);
    hipLaunchKernelGGL(k_extract_v, dim3(bl), dim3(256), 0, s, A, rs, cs, p0, p0, m - p0, ib, w.V,
                       (long)w.vmax);
    apply_block_reflector(m - p0, kmin - p0, ib, T, 0, Q + (long)p0 * ldq + p0, ldq, 1, w, s);
  }
}

__global__ void k_get_r(int m, int k, const cplx* A, long rs, long cs, cplx* R, long ldr) {
  const int kmin = m < k ? m : k;
  const long total = (long)kmin * k;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long i = idx / k, j = idx % k;
    R[i * ldr + j] = (j >= i) ? A[i * rs + j * cs] : make_double2(0.0, 0.0);
  }
}

void qr_get_r(int m, int k, const cplx* A, long rs, long cs, cplx* R, long ldr, hipStream_t s) {
  long total = (long)std::min(m, k) * k;
  int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_get_r, dim3(std::max(blocks, 1)), dim3(256), 0, s, m, k, A, rs, cs, R, ldr);
}

// ---------------------------------------------------------------------------

void hetrd_backtransform(int n, const cplx* A, long lda, int q, cplx* X, long ldx, LinalgWork& w,
                         hipStream_t s) {
  const int nref = n - 1;
  if (nref <= 0) return;
  const int ngroups = ceil_div(nref, BT_NB);
  for (int gi = ngroups - 1; gi >= 0; --gi) {
    const int c0 = gi * BT_NB, ib = std::min(BT_NB, nref - c0);
    const int mrows = n - (c0 + 1);
    block_reflector(A, 1, lda, c0 + 1, c0, mrows, ib, w.tau + c0, w.T, w, s);
    apply_block_reflector(mrows, q, ib, w.T, 0, X + (long)(c0 + 1) * ldx, ldx, 1, w, s);
  }
}

void heev_top(int n, cplx* G, long ldg, int q, cplx* U, long ldu, cplx* Xtmp, LinalgWork& w,
              uint64_t seed, hipStream_t s) {
  require_strided(G, 1, ldg, 0, 0, n, n, "eigensolver: Gram matrix");
  require_strided(U, ldu, 1, 0, 0, n, q, "eigensolver: eigenvectors");
  require_strided(Xtmp, q, 1, 0, 0, n, q, "eigensolver: work vectors");
  require_strided(w.iwork, 1, 0, 0, 0, 6L * n * q / 2, 1, "eigensolver: inverse-iteration work");
  hetrd_lower(n, G, ldg, w, s);
  const int extra = (q < n) ? 1 : 0;
  tridiag_eigvals(n, n - q - extra, q + extra, w, s);
  tridiag_invit(n, q, extra, w, Xtmp, q, seed, s);
  qr_factor(n, q, Xtmp, q, 1, w, s);
  qr_form_q(n, q, Xtmp, q, 1, w, U, ldu, s);
  hetrd_backtransform(n, G, ldg, q, U, ldu, w, s);
}

}  // namespace mpsim
