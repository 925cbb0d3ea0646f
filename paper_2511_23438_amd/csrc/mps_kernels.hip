// Element-wise and reduction kernels of the block-MPS update and measurement.
#include "mps_kernels.h"

#include <algorithm>
#include <cfloat>

namespace mpsim {

// Single-site gate on the physical leg (intra-block gates and the transverse
// layer are site-local: the bond dimensions do not change).
__global__ __launch_bounds__(256) void k_apply_u1(cplx* site, int b0, int d, int b1, const cplx* U) {
  __shared__ cplx Us[256];
  for (int i = threadIdx.x; i < d * d; i += blockDim.x) Us[i] = U[i];
  __syncthreads();
  const long pairs = (long)b0 * b1;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < pairs;
       idx += (long)gridDim.x * blockDim.x) {
    const long a = idx / b1, c = idx % b1;
    // fully unrolled over the largest d, so v stays in registers
    cplx v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = (t < d) ? site[(a * d + t) * b1 + c] : make_double2(0.0, 0.0);
    for (int s = 0; s < d; ++s) {
      cplx acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t < d) acc = cadd(acc, cmul(Us[s * d + t], v[t]));
      site[(a * d + s) * b1 + c] = acc;
    }
  }
}

// One site of the rank-2 operator exp(-i phi Z Z') = cos(phi) I I - i sin(phi) Z Z'
// on the span of sites between the two qubits; the operator index k joins
// the doubled bonds (new index 2 * old + k). mode 0: first site, the right
// bond gains k with weights cos(phi) and -i sin(phi) z(s); mode 1: inside,
// k passes through unchanged; mode 2: last site, the left bond gains k with
// weights 1 and z(s). z(s) = +1 / -1 for bit `bit` (0 = most significant of
// w bits) of the fused index s equal to 0 / 1.
__global__ void k_mpo_site(const cplx* src, cplx* dst, int b0, int d, int b1, int mode, int w,
                           int bit, double c, double sn) {
  const long ob0 = mode == 0 ? b0 : 2L * b0, ob1 = mode == 2 ? b1 : 2L * b1;
  const long total = ob0 * d * ob1;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long oc = idx % ob1;
    const long rest = idx / ob1;
    const int sidx = (int)(rest % d);
    const long oa = rest / d;
    const double z = 1.0 - 2.0 * ((sidx >> (w - 1 - bit)) & 1);
    cplx v;
    if (mode == 0) {
      const int k = (int)(oc & 1);
      v = src[(oa * d + sidx) * b1 + (oc >> 1)];
      v = k == 0 ? cscale(v, c) : cmul(make_double2(0.0, -sn * z), v);
    } else if (mode == 1) {
      const bool same = (oa & 1) == (oc & 1);
      v = same ? src[((oa >> 1) * d + sidx) * b1 + (oc >> 1)] : make_double2(0.0, 0.0);
    } else {
      v = src[((oa >> 1) * d + sidx) * b1 + oc];
      if (oa & 1) v = cscale(v, z);
    }
    dst[idx] = v;
  }
}

void launch_mpo_site(const cplx* src, cplx* dst, int b0, int d, int b1, int mode, int w, int bit,
                     double c, double sn, hipStream_t s) {
  const long total = (mode == 0 ? b0 : 2L * b0) * (long)d * (mode == 2 ? b1 : 2L * b1);
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_mpo_site, dim3(std::max(blocks, 1)), dim3(256), 0, s, src, dst, b0, d, b1, mode,
                     w, bit, c, sn);
}

// Dense two-qubit gate on theta of two d = 2 sites, (2 b0) x (2 b2)
// row-major: for every (a, c) the four values theta[a, s1, s2, c] are mixed
// by G (row-major 4 x 4 over s1 s2, s1 the more significant) and written
// back, at [a, t2, t1, c] when swap is set. Each thread owns one (a, c), so
// the update is in place.
__global__ void k_theta_gate4(cplx* th, int b0, int b2, const cplx* G, int swap) {
  __shared__ cplx Gs[16];
  if (threadIdx.x < 16) Gs[threadIdx.x] = G[threadIdx.x];
  __syncthreads();
  const long pairs = (long)b0 * b2;
  const long ld = 2L * b2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < pairs;
       idx += (long)gridDim.x * blockDim.x) {
    const long a = idx / b2, c = idx % b2;
    cplx v[4];
#pragma unroll
    for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) v[s1 * 2 + s2] = th[(a * 2 + s1) * ld + s2 * b2 + c];
#pragma unroll
    for (int t1 = 0; t1 < 2; ++t1)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2) {
        cplx acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = cadd(acc, cmul(Gs[(t1 * 2 + t2) * 4 + u], v[u]));
        const long at = swap ? (a * 2 + t2) * ld + t1 * b2 + c : (a * 2 + t1) * ld + t2 * b2 + c;
        th[at] = acc;
      }
  }
}

void launch_theta_gate4(cplx* theta, int b0, int b2, const cplx* G, int swap, hipStream_t s) {
  const long pairs = (long)b0 * b2;
  const int blocks = (int)std::min<long>((pairs + 255) / 256, 8192);
  hipLaunchKernelGGL(k_theta_gate4, dim3(std::max(blocks, 1)), dim3(256), 0, s, theta, b0, b2, G, swap);
}

// Measurement with the operator sign * X on a d = 2 site: X holds the three
// stacked blocks X0, X1, X2 (each b x (2 b2)); Y1 = X1 + sign X X0,
// Y2 = X2 + 2 sign X X1 + X0 (X^2 = I), X flipping the physical index.
// Each thread owns one (a, c) and both physical values.
__global__ void k_meas_combine_x(cplx* X, int b, int b2, double sign) {
  const long blk = 2L * b * b2;
  const long pairs = (long)b * b2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < pairs;
       idx += (long)gridDim.x * blockDim.x) {
    const long a = idx / b2, c = idx % b2;
    const long i0 = (a * 2) * b2 + c, i1 = (a * 2 + 1) * b2 + c;
    const cplx x00 = X[i0], x01 = X[i1];
    const cplx x10 = X[blk + i0], x11 = X[blk + i1];
    const cplx x20 = X[2 * blk + i0], x21 = X[2 * blk + i1];
    X[blk + i0] = cadd(x10, cscale(x01, sign));
    X[blk + i1] = cadd(x11, cscale(x00, sign));
    X[2 * blk + i0] = cadd(cadd(x20, cscale(x11, 2.0 * sign)), x00);
    X[2 * blk + i1] = cadd(cadd(x21, cscale(x10, 2.0 * sign)), x01);
  }
}

void launch_meas_combine_x(cplx* X, int b, int b2, double sign, hipStream_t s) {
  const long pairs = (long)b * b2;
  const int blocks = (int)std::min<long>((pairs + 255) / 256, 8192);
  hipLaunchKernelGGL(k_meas_combine_x, dim3(std::max(blocks, 1)), dim3(256), 0, s, X, b, b2, sign);
}

// Weights of the factored Gram matrix of a two-site update without SWAP.
// Dfull[s1][s2] = D[s1][s2] (the block-pair phase table, stored [s_a][s_b]
// for the lower block id a; trans when the lower id sits at site i+1; all
// ones without a gate). side 0 (rows of theta): W[pidx(s1, s1')][s2] =
// D[s1][s2] conj(D[s1'][s2]); side 1 (columns): W[pidx(s2, s2')][s1] =
// conj(D[s1][s2]) D[s1][s2']; pidx(x, y) = x (x + 1) / 2 + y for y <= x.
__global__ void k_pair_weights(const cplx* table, int trans, int d, int side, cplx* W, cplx* Dfull) {
  const int t = threadIdx.x;
  for (int e = t; e < d * d; e += blockDim.x) {
    const int s1 = e / d, s2 = e % d;
    Dfull[e] = table ? (trans ? table[s2 * d + s1] : table[s1 * d + s2]) : make_double2(1.0, 0.0);
  }
  __syncthreads();
  const int np = d * (d + 1) / 2;
  for (int e = t; e < np * d; e += blockDim.x) {
    const int p = e / d, k = e % d;
    int x = 0;
    while ((x + 1) * (x + 2) / 2 <= p) ++x;
    const int y = p - x * (x + 1) / 2;
    cplx w;
    if (side == 0) w = cmulc(Dfull[y * d + k], Dfull[x * d + k]);   // D[x][k] conj(D[y][k])
    else w = cmulc(Dfull[k * d + x], Dfull[k * d + y]);             // conj(D[k][x]) D[k][y]
    W[e] = w;
  }
}

void launch_pair_weights(const cplx* table, int trans, int d, int side, cplx* W, cplx* Dfull,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_pair_weights, dim3(1), dim3(256), 0, s, table, trans, d, side, W, Dfull);
}

// U[(a d + s) q + j] = Up[(s b0 + a) q + j]: rows ordered (s, a) back to (a, s)
__global__ void k_unpermute_rows(const cplx* Up, cplx* U, int b0, int d, int q) {
  const long total = (long)b0 * d * q;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long row = idx / q, j = idx % q;
    const long a = row / d, sidx = row % d;
    U[idx] = Up[(sidx * b0 + a) * q + j];
  }
}

void launch_unpermute_rows(const cplx* Up, cplx* U, int b0, int d, int q, hipStream_t s) {
  const long total = (long)b0 * d * q;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_unpermute_rows, dim3(std::max(blocks, 1)), dim3(256), 0, s, Up, U, b0, d, q);
}

// dst = sum of the real parts of the n diagonal entries of G (ld ldg), one
// workgroup, fixed summation order
__global__ __launch_bounds__(256) void k_trace_real(const cplx* G, long n, long ldg, double* dst) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) acc += G[i * ldg + i].x;
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *dst = acc;
}

void launch_trace_real(const cplx* G, long n, long ldg, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_real, dim3(1), dim3(256), 0, s, G, n, ldg, dst);
}

void launch_apply_u1(cplx* site, int b0, int d, int b1, const cplx* U, hipStream_t s) {
  long pairs = (long)b0 * b1;
  int blocks = (int)std::min<long>((pairs + 255) / 256, 4096);
  hipLaunchKernelGGL(k_apply_u1, dim3(std::max(blocks, 1)), dim3(256), 0, s, site, b0, d, b1, U);
}

#define NORM_BLOCKS 512
__global__ __launch_bounds__(256) void k_norm2_part(const cplx* x, long len, double* partial) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
    acc += cabs2(x[i]);
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_norm2_final(const double* partial, int np, double* dst) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *dst = acc;
}

void launch_norm2(const cplx* x, long len, double* partial, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_part, dim3(NORM_BLOCKS), dim3(256), 0, s, x, len, partial);
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(256), 0, s, (const double*)partial, NORM_BLOCKS, dst);
}

// One wave. count[0]: next log position (kept on the device); count[1]:
// truncations whose kept weight |C|^2 = trace(U^H G U) differs from the sum
// of the top q eigenvalues of G (bisection) by more than tol |M|^2 -- the
// two agree whenever U spans the top-q eigenspace, so a difference means
// the eigenvectors did not converge.
__global__ __launch_bounds__(64) void k_trunc_finalize(double* sc, double* flog, int* count,
                                                       const double* lam, int q, int extra, int* flag,
                                                       double tol) {
  const int t = threadIdx.x;
  double part = 0.0;
  for (int k = extra + t; k < q + extra; k += 64) part += lam[k];
  const double lsum = wave_sum(part);
  if (t != 0) return;
  const int idx = count[0];
  count[0] = idx + 1;
  const double nM = sc[2], nC = sc[3];
  const double f = nC / nM;
  double gap = INFINITY;
  if (extra) {
    const double lmax = fmax(lam[q], 0.0), lq = fmax(lam[1], 0.0), lq1 = fmax(lam[0], 0.0);
    if (lmax > 0.0) gap = (sqrt(lq) - sqrt(lq1)) / sqrt(lmax);
  }
  if (!(f > 0.0) || !isfinite(f) || !(nC > 0.0)) *flag = 1;
  if (!(fabs(nC - lsum) <= tol * nM)) count[1] += 1;
  sc[0] += log(f);
  sc[1] = fmin(sc[1], gap);
  sc[4] = 1.0 / sqrt(nC);
  flog[2 * idx] = f;
  flog[2 * idx + 1] = gap;
}

void launch_trunc_finalize(double* sc, double* flog, int* count, const double* lam, int q, int extra,
                           int* flag, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_trunc_finalize, dim3(1), dim3(64), 0, s, sc, flog, count, lam, q, extra, flag,
                     tol);
}

__global__ void k_scale_by(cplx* x, long len, const double* sc) {
  const double f = sc[4];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
    x[i] = cscale(x[i], f);
}

void launch_scale_by(cplx* x, long len, const double* sc, hipStream_t s) {
  int blocks = (int)std::min<long>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(k_scale_by, dim3(std::max(blocks, 1)), dim3(256), 0, s, x, len, sc);
}

// 32x32 LDS tiles for coalesced reads and writes.
__global__ __launch_bounds__(256) void k_conj_transpose(const cplx* src, int rows, int cols, long lds,
                                                        cplx* dst, long ldd) {
  __shared__ cplx tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[(long)r * lds + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[(long)c * ldd + r] = cconj(tile[tx][k]);
  }
}

void launch_conj_transpose(const cplx* src, int rows, int cols, long lds, cplx* dst, long ldd,
                           hipStream_t s) {
  dim3 grid(ceil_div(cols, 32), ceil_div(rows, 32));
  hipLaunchKernelGGL(k_conj_transpose, grid, dim3(256), 0, s, src, rows, cols, lds, dst, ldd);
}

__global__ void k_meas_combine(cplx* X, int b, int d, int b2, const double* zsum) {
  const long blk = (long)b * d * b2;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < blk; i += (long)gridDim.x * blockDim.x) {
    const int sidx = (int)((i / b2) % d);
    const double z = zsum[sidx];
    const cplx x0 = X[i], x1 = X[blk + i], x2 = X[2 * blk + i];
    X[2 * blk + i] = cadd(cadd(x2, cscale(x1, 2.0 * z)), cscale(x0, z * z));
    X[blk + i] = cadd(x1, cscale(x0, z));
  }
}

void launch_meas_combine(cplx* X, int b, int d, int b2, const double* zsum, hipStream_t s) {
  long blk = (long)b * d * b2;
  int blocks = (int)std::min<long>((blk + 255) / 256, 8192);
  hipLaunchKernelGGL(k_meas_combine, dim3(std::max(blocks, 1)), dim3(256), 0, s, X, b, d, b2, zsum);
}

__global__ void k_env_init(cplx* E) {
  E[0] = make_double2(1.0, 0.0);
  E[1] = make_double2(0.0, 0.0);
  E[2] = make_double2(0.0, 0.0);
}

void launch_env_init(cplx* E, hipStream_t s) {
  hipLaunchKernelGGL(k_env_init, dim3(1), dim3(1), 0, s, E);
}

__global__ void k_fill(cplx* x, long len, cplx v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
    x[i] = v;
}

void launch_fill(cplx* x, long len, cplx v, hipStream_t s) {
  int blocks = (int)std::min<long>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill, dim3(std::max(blocks, 1)), dim3(256), 0, s, x, len, v);
}

}  // namespace mpsim
