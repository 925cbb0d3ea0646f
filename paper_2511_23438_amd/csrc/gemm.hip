// Complex float64 GEMM on gfx950 matrix cores.
//
// A complex product is four real products on v_mfma_f64_16x16x4f64:
//   Cr += Ar*Br - Ai*Bi,  Ci += Ar*Bi + Ai*Br.
// Tiles of 64x64 outputs per 256-thread workgroup (4 waves, 32x32 each as
// 2x2 MFMA blocks), K staged through LDS 16 at a time with the real and
// imaginary planes split (planar in LDS, interleaved in HBM), and the next
// K-tile prefetched into registers while the current one is multiplied.
// Operand lane layout of the f64 16x16x4 instruction: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; result register v of lane l holds
// D[4v + l/16][l%16].
#include "gemm.h"

#include <algorithm>

namespace mpsim {

typedef double d4 __attribute__((ext_vector_type(4)));

#define BM 64
#define BN 64
#define BK 16

struct ZGemmDev {
  ZGemm g;
  int ksplit;
  long kchunk;
  cplx* partial;
};

template <int TA>
__device__ inline void load_a(const ZGemm& g, const cplx* A, int m0, long k0, long kend,
                              cplx r[4]) {
  int t = threadIdx.x;
  if (TA == 0) {  // (i,k) at A[i*ld + k]: 4 consecutive k per thread
    int i = t >> 2, kk = (t & 3) * 4;
    long gi = m0 + i;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long gk = k0 + kk + u;
      r[u] = (gi < g.M && gk < kend) ? A[gi * g.A.ld + gk] : make_double2(0, 0);
    }
  } else {        // (i,k) at A[k*ld + i]: 4 consecutive i per thread
    int k = t >> 4, ii = (t & 15) * 4;
    long gk = k0 + k;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long gi = m0 + ii + u;
      r[u] = (gi < g.M && gk < kend) ? A[gk * g.A.ld + gi] : make_double2(0, 0);
    }
  }
}

template <int TB>
__device__ inline void load_b(const ZGemm& g, const cplx* B, int n0, long k0, long kend,
                              cplx r[4]) {
  int t = threadIdx.x;
  if (TB == 0) {  // (k,j) at B[k*ld + j]: 4 consecutive j
    int k = t >> 4, jj = (t & 15) * 4;
    long gk = k0 + k;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long gj = n0 + jj + u;
      r[u] = (gj < g.N && gk < kend) ? B[gk * g.B.ld + gj] : make_double2(0, 0);
    }
  } else {        // (k,j) at B[j*ld + k]: 4 consecutive k
    int j = t >> 2, kk = (t & 3) * 4;
    long gj = n0 + j;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long gk = k0 + kk + u;
      r[u] = (gj < g.N && gk < kend) ? B[gj * g.B.ld + gk] : make_double2(0, 0);
    }
  }
}

template <int TA>
__device__ inline void store_a(double (*As)[BK][BM], const cplx r[4], int conj) {
  int t = threadIdx.x;
  double sg = conj ? -1.0 : 1.0;
  if (TA == 0) {
    int i = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { As[0][kk + u][i] = r[u].x; As[1][kk + u][i] = sg * r[u].y; }
  } else {
    int k = t >> 4, ii = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { As[0][k][ii + u] = r[u].x; As[1][k][ii + u] = sg * r[u].y; }
  }
}

template <int TB>
__device__ inline void store_b(double (*Bs)[BK][BN], const cplx r[4], int conj) {
  int t = threadIdx.x;
  double sg = conj ? -1.0 : 1.0;
  if (TB == 0) {
    int k = t >> 4, jj = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { Bs[0][k][jj + u] = r[u].x; Bs[1][k][jj + u] = sg * r[u].y; }
  } else {
    int j = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { Bs[0][kk + u][j] = r[u].x; Bs[1][kk + u][j] = sg * r[u].y; }
  }
}

template <int TA, int TB>
__global__ __launch_bounds__(256) void zgemm_kernel(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  __shared__ double As[2][BK][BM];
  __shared__ double Bs[2][BK][BN];
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  if (g.lower_only && n0 >= m0 + BM) return;
  if (g.upper_only && m0 >= n0 + BN) return;
  const int bz = blockIdx.z;
  const int bat = bz / gd.ksplit, ks = bz % gd.ksplit;
  const cplx* A = g.A.p + (long)bat * g.A.stride;
  const cplx* B = g.B.p + (long)bat * g.B.stride;
  const long kbeg = (long)ks * gd.kchunk;
  long kend = kbeg + gd.kchunk;
  if (kend > g.K) kend = g.K;

  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (d4){0, 0, 0, 0};
      ci[a][b] = (d4){0, 0, 0, 0};
    }

  cplx ra[4], rb[4];
  if (kbeg < kend) {
    load_a<TA>(g, A, m0, kbeg, kend, ra);
    load_b<TB>(g, B, n0, kbeg, kend, rb);
  }
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    store_a<TA>(As, ra, g.A.conj);
    store_b<TB>(Bs, rb, g.B.conj);
    __syncthreads();
    if (k0 + BK < kend) {
      load_a<TA>(g, A, m0, k0 + BK, kend, ra);
      load_b<TB>(g, B, n0, k0 + BK, kend, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (l >> 4);
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = As[0][kr][wr + a * 16 + (l & 15)];
        ai[a] = As[1][kr][wr + a * 16 + (l & 15)];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Bs[0][kr][wc + b * 16 + (l & 15)];
        bi[b] = Bs[1][kr][wc + b * 16 + (l & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cr[a][b], 0, 0, 0);
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], bi[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], ci[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], ci[a][b], 0, 0, 0);
        }
    }
  }

  // epilogue
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long row = m0 + wr + a * 16 + 4 * v + (l >> 4);
        const long col = n0 + wc + b * 16 + (l & 15);
        if (row >= g.M || col >= g.N) continue;
        cplx val = make_double2(cr[a][b][v], ci[a][b][v]);
        if (gd.ksplit > 1) {
          gd.partial[((long)bz * g.M + row) * g.N + col] = val;
          continue;
        }
        cplx* C = g.C + (long)bat * g.strideC;
        if (g.epi == EPI_THETA) {
          const long al = row / g.d1, s1 = row % g.d1;
          const long s2 = col / g.b2, gg = col % g.b2;
          if (g.phase) {
            cplx ph = g.phase_trans ? g.phase[s2 * g.d1 + s1] : g.phase[s1 * g.d2 + s2];
            val = cmul(val, ph);
          }
          if (g.swap) C[(al * g.d2 + s2) * ((long)g.d1 * g.b2) + s1 * g.b2 + gg] = val;
          else C[row * g.ldc + col] = val;
          continue;
        }
        const long idx = g.transC ? col * g.ldc + row : row * g.ldc + col;
        cplx out = cmul(g.alpha, val);
        if (g.beta.x != 0.0 || g.beta.y != 0.0) out = cadd(out, cmul(g.beta, C[idx]));
        C[idx] = out;
      }
}

// Sum the split-K partials and apply the store epilogue.
__global__ void zgemm_reduce(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  long total = (long)g.M * g.N;
  int bat = blockIdx.y;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    long row = e / g.N, col = e % g.N;
    cplx s = make_double2(0, 0);
    for (int k = 0; k < gd.ksplit; ++k)
      s = cadd(s, gd.partial[((long)(bat * gd.ksplit + k) * g.M + row) * g.N + col]);
    cplx* C = g.C + (long)bat * g.strideC;
    const long idx = g.transC ? col * g.ldc + row : row * g.ldc + col;
    cplx out = cmul(g.alpha, s);
    if (g.beta.x != 0.0 || g.beta.y != 0.0) out = cadd(out, cmul(g.beta, C[idx]));
    C[idx] = out;
  }
}

void zgemm(const ZGemm& g0, cplx* partial, long partial_elems, hipStream_t s, Prof* prof) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return;
  ZGemm g = g0;
  if (g.transC && g.epi == EPI_STORE) {
    // A column-major result is stored as C^T = op(B)^T op(A)^T, row-major,
    // so that neighbouring lanes write neighbouring addresses.
    std::swap(g.A, g.B);
    g.A.trans ^= 1;
    g.B.trans ^= 1;
    std::swap(g.M, g.N);
    g.transC = 0;
    std::swap(g.lower_only, g.upper_only);
  }
  ZGemmDev gd;
  gd.g = g;
  gd.ksplit = 1;
  gd.kchunk = g.K;
  gd.partial = partial;
  long tiles = (long)ceil_div(g.M, BM) * ceil_div(g.N, BN) * g.batch;
  if (g.K <= 0) {
    // C = beta*C (alpha * empty product)
    ZGemmDev z = gd;
    z.ksplit = 1;
    z.kchunk = 0;
    dim3 grid(ceil_div(g.N, BN), ceil_div(g.M, BM), g.batch);
    hipLaunchKernelGGL((zgemm_kernel<0, 0>), grid, dim3(256), 0, s, z);
    return;
  }
  if (partial && g.epi == EPI_STORE && !g.lower_only && !g.upper_only && tiles < 128 &&
      g.K >= 1024) {
    int ks = (int)std::min<long>(g.K / 256, (256 + tiles - 1) / tiles);
    while (ks > 1 && (long)ks * g.batch * g.M * g.N > partial_elems) --ks;
    if (ks > 1) {
      gd.ksplit = ks;
      gd.kchunk = ((g.K + ks - 1) / ks + BK - 1) / BK * BK;
      gd.ksplit = (int)((g.K + gd.kchunk - 1) / gd.kchunk);
    }
  }
  dim3 grid(ceil_div(g.N, BN), ceil_div(g.M, BM), g.batch * gd.ksplit);
  const int ta = g.A.trans, tb = g.B.trans;
  const int pk = (prof && prof->kind == PROF_GEMM) ? PROF_GEMM : g.tag;
  double flops = 8.0 * g.M * (double)g.N * g.K * g.batch;
  if (g.lower_only || g.upper_only) flops = 8.0 * g.M * (g.M + 1.0) * 0.5 * g.K * g.batch;
  if (prof) prof->begin(pk, s);
  if (ta == 0 && tb == 0) hipLaunchKernelGGL((zgemm_kernel<0, 0>), grid, dim3(256), 0, s, gd);
  else if (ta == 0 && tb == 1) hipLaunchKernelGGL((zgemm_kernel<0, 1>), grid, dim3(256), 0, s, gd);
  else if (ta == 1 && tb == 0) hipLaunchKernelGGL((zgemm_kernel<1, 0>), grid, dim3(256), 0, s, gd);
  else hipLaunchKernelGGL((zgemm_kernel<1, 1>), grid, dim3(256), 0, s, gd);
  if (gd.ksplit > 1) {
    long total = (long)g.M * g.N;
    int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(zgemm_reduce, dim3(blocks, g.batch), dim3(256), 0, s, gd);
  }
  if (prof) prof->end(pk, flops, s);
}

}  // namespace mpsim
