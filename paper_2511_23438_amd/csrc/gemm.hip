// Complex float64 GEMM on gfx950 matrix cores.
//
// A complex product takes three real products on v_mfma_f64_16x16x4f64
// (Gauss): with T1 = Ar*Br, T2 = Ai*Bi, T3 = (Ar + Ai)*(Br + Bi),
//   Cr = T1 - T2,  Ci = T3 - T1 - T2;
// the sums Ar + Ai and Br + Bi are formed once when a tile is staged in LDS
// (a third plane). The reduced-precision kernels below use four products.
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

// Operand loads are split in two: load_a / load_b only issue the loads, from
// clamped (always valid) addresses and with the second K segment chosen by
// selects, so no instruction between the prefetch and the multiplication of
// the current tile needs the loaded values; fix_a / fix_b, called when the
// tile is staged into LDS one step later, zero the out-of-range elements and
// apply the Hermitian-operand mirroring.

// address of element (i, k) of op(A) (before conjugation), with the
// optional second K segment; (gi, gk) must be in range
template <int TA>
__device__ inline const cplx* addr_a(const ZGemm& g, const cplx* A, long gi, long gk) {
  const bool second = g.kcat && gk >= g.kcat;
  const cplx* P = second ? g.A2.p : A;
  const long ld = second ? g.A2.ld : g.A.ld;
  const long k = second ? gk - g.kcat : gk;
  return TA == 0 ? P + gi * ld + k : P + k * ld + gi;
}

template <int TB>
__device__ inline const cplx* addr_b(const ZGemm& g, const cplx* B, long gk, long gj) {
  const bool second = g.kcat && gk >= g.kcat;
  const cplx* P = second ? g.B2.p : B;
  const long ld = second ? g.B2.ld : g.B.ld;
  const long k = second ? gk - g.kcat : gk;
  return TB == 0 ? P + k * ld + gj : P + gj * ld + k;
}

// Hermitian operand with the lower triangle stored column-major: which
// lane layout a K-tile is loaded with. 0: the tile lies in the upper triangle
// (read the stored transpose, 4 consecutive k per thread); 1: otherwise (4
// consecutive i per thread; on tiles that cross the diagonal each element is
// read from the lower or the mirrored position).
__device__ inline int herm_tile_lower(int m0, long k0) { return k0 < (long)m0 + BM; }

// element coordinates handled by this thread for an A tile
template <int TA>
__device__ inline void coords_a(int m0, long k0, int u, long& gi, long& gk) {
  const int t = threadIdx.x;
  if (TA == 0 || (TA == 2 && !herm_tile_lower(m0, k0))) {
    gi = m0 + (t >> 2);
    gk = k0 + (t & 3) * 4 + u;
  } else {
    gk = k0 + (t >> 4);
    gi = m0 + (t & 15) * 4 + u;
  }
}

template <int TA>
__device__ inline void load_a(const ZGemm& g, const cplx* A, int m0, long k0, long kend,
                              cplx r[4]) {
  const long mlast = g.M - 1, klast = kend - 1;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    long gi, gk;
    coords_a<TA>(m0, k0, u, gi, gk);
    const long ci = min(gi, mlast), ck = min(gk, klast);
    if (TA == 2) {
      // stored lower element of (ci, ck) or of its mirror
      r[u] = A[(ci >= ck) ? ck * g.A.ld + ci : ci * g.A.ld + ck];
    } else {
      r[u] = *addr_a<TA>(g, A, ci, ck);
    }
  }
}

template <int TA>
__device__ inline void fix_a(const ZGemm& g, int m0, long k0, long kend, cplx r[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    long gi, gk;
    coords_a<TA>(m0, k0, u, gi, gk);
    cplx v = r[u];
    if (TA == 2) {
      if (gi < gk) v.y = -v.y;
      if (gi == gk) v.y = 0.0;
    }
    r[u] = (gi < g.M && gk < kend) ? v : make_double2(0.0, 0.0);
  }
}

template <int TB>
__device__ inline void coords_b(int n0, long k0, int u, long& gk, long& gj) {
  const int t = threadIdx.x;
  if (TB == 0) {
    gk = k0 + (t >> 4);
    gj = n0 + (t & 15) * 4 + u;
  } else {
    gj = n0 + (t >> 2);
    gk = k0 + (t & 3) * 4 + u;
  }
}

template <int TB>
__device__ inline void load_b(const ZGemm& g, const cplx* B, int n0, long k0, long kend,
                              cplx r[4]) {
  const long nlast = g.N - 1, klast = kend - 1;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    long gk, gj;
    coords_b<TB>(n0, k0, u, gk, gj);
    r[u] = *addr_b<TB>(g, B, min(gk, klast), min(gj, nlast));
  }
}

template <int TB>
__device__ inline void fix_b(const ZGemm& g, int n0, long k0, long kend, cplx r[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    long gk, gj;
    coords_b<TB>(n0, k0, u, gk, gj);
    r[u] = (gj < g.N && gk < kend) ? r[u] : make_double2(0.0, 0.0);
  }
}

// planes: 0 real, 1 imaginary, 2 real + imaginary (after conjugation)
template <int TA>
__device__ inline void store_a(double (*As)[BK][BM], const cplx r[4], int conj, int tile_lower = 1) {
  int t = threadIdx.x;
  double sg = conj ? -1.0 : 1.0;
  if (TA == 0 || (TA == 2 && !tile_lower)) {
    int i = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double re = r[u].x, im = sg * r[u].y;
      As[0][kk + u][i] = re; As[1][kk + u][i] = im; As[2][kk + u][i] = re + im;
    }
  } else {
    int k = t >> 4, ii = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double re = r[u].x, im = sg * r[u].y;
      As[0][k][ii + u] = re; As[1][k][ii + u] = im; As[2][k][ii + u] = re + im;
    }
  }
}

template <int TB>
__device__ inline void store_b(double (*Bs)[BK][BN], const cplx r[4], int conj) {
  int t = threadIdx.x;
  double sg = conj ? -1.0 : 1.0;
  if (TB == 0) {
    int k = t >> 4, jj = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double re = r[u].x, im = sg * r[u].y;
      Bs[0][k][jj + u] = re; Bs[1][k][jj + u] = im; Bs[2][k][jj + u] = re + im;
    }
  } else {
    int j = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double re = r[u].x, im = sg * r[u].y;
      Bs[0][kk + u][j] = re; Bs[1][kk + u][j] = im; Bs[2][kk + u][j] = re + im;
    }
  }
}

// The C value that an element's store epilogue adds (beta*C), read before
// any of the workgroup's stores: as far as the compiler knows C may alias
// the stored elements, so loads placed between the stores would each wait
// for their data in turn. Zero where the epilogue reads no C.
__device__ inline cplx load_c(const ZGemmDev& gd, int bat, long row, long col) {
  const ZGemm& g = gd.g;
  if (gd.ksplit > 1 || g.epi != EPI_STORE || (g.beta.x == 0.0 && g.beta.y == 0.0) || row >= g.M ||
      col >= g.N)
    return make_double2(0.0, 0.0);
  const cplx* C = g.C + (long)bat * g.strideC;
  return C[g.transC ? col * g.ldc + row : row * g.ldc + col];
}

// Store one result element: split-K partial, theta epilogue (phase, SWAP
// layout) or alpha*val + beta*C, with C read beforehand by load_c.
__device__ inline void store_out(const ZGemmDev& gd, int bz, int bat, long row, long col, cplx val,
                                 cplx cprev) {
  const ZGemm& g = gd.g;
  if (row >= g.M || col >= g.N) return;
  if (gd.ksplit > 1) {
    gd.partial[((long)bz * g.M + row) * g.N + col] = val;
    return;
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
    return;
  }
  const long idx = g.transC ? col * g.ldc + row : row * g.ldc + col;
  cplx out = cmul(g.alpha, val);
  if (g.beta.x != 0.0 || g.beta.y != 0.0) out = cadd(out, cmul(g.beta, cprev));
  C[idx] = out;
}

// WL selects the wave layout of the 64x64 tile: 0: 2x2 waves of 32x32;
// 1: 4x1 waves of 16x32, for outputs at most 32 columns wide (no MFMA work
// on columns past N).
template <int TA, int TB, int WL = 0>
__global__ __launch_bounds__(256, 2) void zgemm_kernel(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  __shared__ double As[3][BK][BM];
  __shared__ double Bs[3][BK][BN];
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
  constexpr int NA = WL ? 1 : 2;
  const int wr = WL ? w * 16 : (w >> 1) * 32, wc = WL ? 0 : (w & 1) * 32;
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }

  cplx ra[4], rb[4];
  if (kbeg < kend) {
    load_a<TA>(g, A, m0, kbeg, kend, ra);
    load_b<TB>(g, B, n0, kbeg, kend, rb);
  }
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    fix_a<TA>(g, m0, k0, kend, ra);
    fix_b<TB>(g, n0, k0, kend, rb);
    __syncthreads();
    store_a<TA>(As, ra, TA == 2 ? 0 : g.A.conj, TA == 2 ? herm_tile_lower(m0, k0) : 1);
    store_b<TB>(Bs, rb, g.B.conj);
    __syncthreads();
    if (k0 + BK < kend) {
      load_a<TA>(g, A, m0, k0 + BK, kend, ra);
      load_b<TB>(g, B, n0, k0 + BK, kend, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (l >> 4);
      double ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        ar[a] = As[0][kr][wr + a * 16 + (l & 15)];
        ai[a] = As[1][kr][wr + a * 16 + (l & 15)];
        as[a] = As[2][kr][wr + a * 16 + (l & 15)];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Bs[0][kr][wc + b * 16 + (l & 15)];
        bi[b] = Bs[1][kr][wc + b * 16 + (l & 15)];
        bs[b] = Bs[2][kr][wc + b * 16 + (l & 15)];
      }
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], t1[a][b], 0, 0, 0);
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], t2[a][b], 0, 0, 0);
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[a], bs[b], t3[a][b], 0, 0, 0);
        }
    }
  }

  // epilogue (f64 result layout: register v of lane l is row 4v + l/16)
  cplx cp[NA][2][4];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cp[a][b][v] = load_c(gd, bat, m0 + wr + a * 16 + 4 * v + (l >> 4), n0 + wc + b * 16 + (l & 15));
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        store_out(gd, bz, bat, m0 + wr + a * 16 + 4 * v + (l >> 4), n0 + wc + b * 16 + (l & 15),
                  make_double2(t1[a][b][v] - t2[a][b][v],
                               t3[a][b][v] - t1[a][b][v] - t2[a][b][v]),
                  cp[a][b][v]);
}


// ---------------------------------------------------------------------------
// Reduced-precision products. Operands are read as complex128 from HBM and
// rounded when staged into LDS.

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int TA>
__device__ inline void store_a_f32(float (*As)[BK][BM], const cplx r[4], int conj) {
  const int t = threadIdx.x;
  const float sg = conj ? -1.f : 1.f;
  if (TA == 0) {
    const int i = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { As[0][kk + u][i] = (float)r[u].x; As[1][kk + u][i] = sg * (float)r[u].y; }
  } else {
    const int k = t >> 4, ii = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { As[0][k][ii + u] = (float)r[u].x; As[1][k][ii + u] = sg * (float)r[u].y; }
  }
}

template <int TB>
__device__ inline void store_b_f32(float (*Bs)[BK][BN], const cplx r[4], int conj) {
  const int t = threadIdx.x;
  const float sg = conj ? -1.f : 1.f;
  if (TB == 0) {
    const int k = t >> 4, jj = (t & 15) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { Bs[0][k][jj + u] = (float)r[u].x; Bs[1][k][jj + u] = sg * (float)r[u].y; }
  } else {
    const int j = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) { Bs[0][kk + u][j] = (float)r[u].x; Bs[1][kk + u][j] = sg * (float)r[u].y; }
  }
}

// complex64 GEMM, FP32 accumulation, v_mfma_f32_16x16x4f32
// (result register v of lane l is row 4*(l/16) + v).
template <int TA, int TB>
__global__ __launch_bounds__(256) void cgemm_f32_kernel(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  __shared__ float As[2][BK][BM];
  __shared__ float Bs[2][BK][BN];
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
  f4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (f4){0, 0, 0, 0};
      ci[a][b] = (f4){0, 0, 0, 0};
    }
  cplx ra[4], rb[4];
  if (kbeg < kend) {
    load_a<TA>(g, A, m0, kbeg, kend, ra);
    load_b<TB>(g, B, n0, kbeg, kend, rb);
  }
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    fix_a<TA>(g, m0, k0, kend, ra);
    fix_b<TB>(g, n0, k0, kend, rb);
    store_a_f32<TA>(As, ra, g.A.conj);
    store_b_f32<TB>(Bs, rb, g.B.conj);
    __syncthreads();
    if (k0 + BK < kend) {
      load_a<TA>(g, A, m0, k0 + BK, kend, ra);
      load_b<TB>(g, B, n0, k0 + BK, kend, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (l >> 4);
      float ar[2], ai[2], br[2], bi[2];
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
          cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], br[b], cr[a][b], 0, 0, 0);
          cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[a], bi[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], bi[b], ci[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[a], br[b], ci[a][b], 0, 0, 0);
        }
    }
  }
  cplx cp[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cp[a][b][v] = load_c(gd, bat, m0 + wr + a * 16 + 4 * (l >> 4) + v, n0 + wc + b * 16 + (l & 15));
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        store_out(gd, bz, bat, m0 + wr + a * 16 + 4 * (l >> 4) + v, n0 + wc + b * 16 + (l & 15),
                  make_double2((double)cr[a][b][v], (double)ci[a][b][v]), cp[a][b][v]);
}

// Three-term bf16 split: x = hi + mid + lo with hi = bf16(x),
// mid = bf16(x - hi), lo = bf16(x - hi - mid) (24 significant bits, the
// precision of FP32). A product keeps the six partial products of relative
// order >= 2^-16 (hh, hm, mh, hl, lh, mm), accumulated in FP32 on
// v_mfma_f32_16x16x32_bf16. LDS planes per operand: re (h, m, l), im (h, m,
// l), and for B also -im; K = 32 per stage, k contiguous so that one lane
// reads its 8 consecutive k values at once.
#define BK2 32
#define KP (BK2 + 8)

__device__ inline void split3_bf16(float x, __bf16& h, __bf16& m, __bf16& lo) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  lo = (__bf16)(r1 - (float)m);
}

template <int TA>
__device__ inline void stage_a_bf(__bf16 (*As)[BM][KP], const cplx r[4], int kofs, int conj) {
  const int t = threadIdx.x;
  const float sg = conj ? -1.f : 1.f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int i, k;
    if (TA == 0) { i = t >> 2; k = (t & 3) * 4 + u; }
    else { k = t >> 4; i = (t & 15) * 4 + u; }
    __bf16 h, m, lo;
    split3_bf16((float)r[u].x, h, m, lo);
    As[0][i][kofs + k] = h; As[1][i][kofs + k] = m; As[2][i][kofs + k] = lo;
    split3_bf16(sg * (float)r[u].y, h, m, lo);
    As[3][i][kofs + k] = h; As[4][i][kofs + k] = m; As[5][i][kofs + k] = lo;
  }
}

template <int TB>
__device__ inline void stage_b_bf(__bf16 (*Bs)[BN][KP], const cplx r[4], int kofs, int conj) {
  const int t = threadIdx.x;
  const float sg = conj ? -1.f : 1.f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int j, k;
    if (TB == 0) { k = t >> 4; j = (t & 15) * 4 + u; }
    else { j = t >> 2; k = (t & 3) * 4 + u; }
    __bf16 h, m, lo;
    split3_bf16((float)r[u].x, h, m, lo);
    Bs[0][j][kofs + k] = h; Bs[1][j][kofs + k] = m; Bs[2][j][kofs + k] = lo;
    const float im = sg * (float)r[u].y;
    split3_bf16(im, h, m, lo);
    Bs[3][j][kofs + k] = h; Bs[4][j][kofs + k] = m; Bs[5][j][kofs + k] = lo;
    Bs[6][j][kofs + k] = -h; Bs[7][j][kofs + k] = -m; Bs[8][j][kofs + k] = -lo;
  }
}

// eight consecutive bf16 of an LDS row in one 128-bit load (rows are KP = 40
// elements long and the offsets multiples of 8, so every address is 16-byte
// aligned)
__device__ inline bf8 ld8(const __bf16* p) { return *reinterpret_cast<const bf8*>(p); }

// acc += x * y for split operands x = (xh, xm, xl), y = (yh, ym, yl)
__device__ inline f4 mfma_split3(const bf8* x, const bf8* y, f4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], y[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[2], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], y[1], acc, 0, 0, 0);
  return acc;
}

template <int TA, int TB>
__global__ __launch_bounds__(256) void cgemm_bf16x3_kernel(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  __shared__ __attribute__((aligned(16))) __bf16 As[6][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[9][BN][KP];
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
  f4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (f4){0, 0, 0, 0};
      ci[a][b] = (f4){0, 0, 0, 0};
    }
  // the operands of the next K stage are loaded (clamped addresses, always
  // valid) before the products of the current one and staged one step later
  cplx ra0[4], rb0[4], ra1[4], rb1[4];
  load_a<TA>(g, A, m0, kbeg, kend, ra0);
  load_b<TB>(g, B, n0, kbeg, kend, rb0);
  load_a<TA>(g, A, m0, kbeg + BK, kend, ra1);
  load_b<TB>(g, B, n0, kbeg + BK, kend, rb1);
  for (long k0 = kbeg; k0 < kend; k0 += BK2) {
    __syncthreads();
    fix_a<TA>(g, m0, k0, kend, ra0);
    fix_b<TB>(g, n0, k0, kend, rb0);
    stage_a_bf<TA>(As, ra0, 0, g.A.conj);
    stage_b_bf<TB>(Bs, rb0, 0, g.B.conj);
    fix_a<TA>(g, m0, k0 + BK, kend, ra1);
    fix_b<TB>(g, n0, k0 + BK, kend, rb1);
    stage_a_bf<TA>(As, ra1, BK, g.A.conj);
    stage_b_bf<TB>(Bs, rb1, BK, g.B.conj);
    __syncthreads();
    if (k0 + BK2 < kend) {
      load_a<TA>(g, A, m0, k0 + BK2, kend, ra0);
      load_b<TB>(g, B, n0, k0 + BK2, kend, rb0);
      load_a<TA>(g, A, m0, k0 + BK2 + BK, kend, ra1);
      load_b<TB>(g, B, n0, k0 + BK2 + BK, kend, rb1);
    }
    const int kq = 8 * (l >> 4);
    bf8 are[2][3], aim[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = wr + a * 16 + (l & 15);
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        are[a][p] = ld8(&As[p][i][kq]);
        aim[a][p] = ld8(&As[3 + p][i][kq]);
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = wc + b * 16 + (l & 15);
      bf8 bre[3], bim[3], bnim[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        bre[p] = ld8(&Bs[p][j][kq]);
        bim[p] = ld8(&Bs[3 + p][j][kq]);
        bnim[p] = ld8(&Bs[6 + p][j][kq]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        cr[a][b] = mfma_split3(are[a], bre, cr[a][b]);
        cr[a][b] = mfma_split3(aim[a], bnim, cr[a][b]);
        ci[a][b] = mfma_split3(are[a], bim, ci[a][b]);
        ci[a][b] = mfma_split3(aim[a], bre, ci[a][b]);
      }
    }
  }
  cplx cp[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cp[a][b][v] = load_c(gd, bat, m0 + wr + a * 16 + 4 * (l >> 4) + v, n0 + wc + b * 16 + (l & 15));
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        store_out(gd, bz, bat, m0 + wr + a * 16 + 4 * (l >> 4) + v, n0 + wc + b * 16 + (l & 15),
                  make_double2((double)cr[a][b][v], (double)ci[a][b][v]), cp[a][b][v]);
}

// ---------------------------------------------------------------------------
// Hermitian operand (lower triangle stored column-major) times a narrow
// operand of at most 32 columns: 128 x 32 outputs per workgroup, each wave
// 32 x 32 as 2 x 2 MFMA blocks, so that a wave issues as many products per
// staged K-tile as in the square tile (the 64 x 32 narrow layout issues half).
#define HM 128
#define HN 32
#define HMP (HM + 1)   // padded LDS rows: the k-major staging writes stay conflict-free
#define HNP (HN + 1)

template <int TB>
__global__ __launch_bounds__(256, 2) void zhemm_n32_kernel(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  __shared__ double As[3][BK][HMP];
  __shared__ double Bs[3][BK][HNP];
  const int n0 = blockIdx.x * HN, m0 = blockIdx.y * HM;
  const int bz = blockIdx.z;
  const int bat = bz / gd.ksplit, ks = bz % gd.ksplit;
  const cplx* A = g.A.p + (long)bat * g.A.stride;
  const cplx* B = g.B.p + (long)bat * g.B.stride;
  const long lda = g.A.ld, ldb = g.B.ld;
  const long kbeg = (long)ks * gd.kchunk;
  long kend = kbeg + gd.kchunk;
  if (kend > g.K) kend = g.K;
  const long mlast = g.M - 1, nlast = g.N - 1;

  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wr = w * 32;
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }

  // A tile element u of this thread, with neighbouring lanes on neighbouring
  // addresses: tiles reaching below the diagonal read stored columns (lane ->
  // row, t >> 7 and u -> column); tiles wholly above it read the stored
  // transpose (lane -> k within 16, t >> 4 and u -> row)
  auto a_coords = [&](long k0, int u, long& gi, long& gk) {
    if (k0 < (long)m0 + HM) {
      gi = m0 + (t & 127);
      gk = k0 + (t >> 7) + 2 * u;
    } else {
      gk = k0 + (t & 15);
      gi = m0 + (t >> 4) + 16 * u;
    }
  };
  auto b_coords = [&](long k0, int u, long& gk, long& gj) {
    if (TB == 0) {
      gj = n0 + (t & 31);
      gk = k0 + (t >> 5) + 8 * u;
    } else {
      gk = k0 + (t & 15);
      gj = n0 + (t >> 4) + 16 * u;
    }
  };
  auto load = [&](long k0, cplx ra[8], cplx rb[2]) {
    const long klast = kend - 1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      long gi, gk;
      a_coords(k0, u, gi, gk);
      const long ci = min(gi, mlast), ck = min(gk, klast);
      ra[u] = A[(ci >= ck) ? ck * lda + ci : ci * lda + ck];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      long gk, gj;
      b_coords(k0, u, gk, gj);
      const long ck = min(gk, klast), cj = min(gj, nlast);
      rb[u] = B[TB == 0 ? ck * ldb + cj : cj * ldb + ck];
    }
  };

  cplx ra[8], rb[2];
  if (kbeg < kend) load(kbeg, ra, rb);
  const double sgb = g.B.conj ? -1.0 : 1.0;
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    // mirror, zero out-of-range elements, stage the three planes
    const bool lower = k0 < (long)m0 + HM;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      long gi, gk;
      a_coords(k0, u, gi, gk);
      cplx v = ra[u];
      if (gi < gk) v.y = -v.y;
      if (gi == gk) v.y = 0.0;
      ra[u] = (gi < g.M && gk < kend) ? v : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      long gk, gj;
      b_coords(k0, u, gk, gj);
      rb[u] = (gj < g.N && gk < kend) ? rb[u] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int ii = lower ? (t & 127) : (t >> 4) + 16 * u;
      const int kk = lower ? (t >> 7) + 2 * u : (t & 15);
      As[0][kk][ii] = ra[u].x;
      As[1][kk][ii] = ra[u].y;
      As[2][kk][ii] = ra[u].x + ra[u].y;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int jj = TB == 0 ? (t & 31) : (t >> 4) + 16 * u;
      const int kk = TB == 0 ? (t >> 5) + 8 * u : (t & 15);
      const double re = rb[u].x, im = sgb * rb[u].y;
      Bs[0][kk][jj] = re;
      Bs[1][kk][jj] = im;
      Bs[2][kk][jj] = re + im;
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK, ra, rb);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (l >> 4);
      double ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = As[0][kr][wr + a * 16 + (l & 15)];
        ai[a] = As[1][kr][wr + a * 16 + (l & 15)];
        as[a] = As[2][kr][wr + a * 16 + (l & 15)];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Bs[0][kr][b * 16 + (l & 15)];
        bi[b] = Bs[1][kr][b * 16 + (l & 15)];
        bs[b] = Bs[2][kr][b * 16 + (l & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], t1[a][b], 0, 0, 0);
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], t2[a][b], 0, 0, 0);
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[a], bs[b], t3[a][b], 0, 0, 0);
        }
    }
  }
  cplx cp[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cp[a][b][v] = load_c(gd, bat, m0 + wr + a * 16 + 4 * v + (l >> 4), n0 + b * 16 + (l & 15));
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        store_out(gd, bz, bat, m0 + wr + a * 16 + 4 * v + (l >> 4), n0 + b * 16 + (l & 15),
                  make_double2(t1[a][b][v] - t2[a][b][v],
                               t3[a][b][v] - t1[a][b][v] - t2[a][b][v]),
                  cp[a][b][v]);
}

// Sum the split-K partials and apply the store epilogue.
__global__ void zgemm_reduce(ZGemmDev gd) {
  const ZGemm& g = gd.g;
  long total = (long)g.M * g.N;
  int bat = blockIdx.y;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    long row = e / g.N, col = e % g.N;
    cplx* C = g.C + (long)bat * g.strideC;
    const long idx = g.transC ? col * g.ldc + row : row * g.ldc + col;
    const bool addc = g.beta.x != 0.0 || g.beta.y != 0.0;
    const cplx cprev = addc ? C[idx] : make_double2(0.0, 0.0);
    cplx s = make_double2(0, 0);
    // 16 loads in flight per round; summation order k = 0, 1, ... as a plain loop
    for (int k0 = 0; k0 < gd.ksplit; k0 += 16) {
      cplx pv[16];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        pv[i] = (k0 + i < gd.ksplit) ? gd.partial[((long)(bat * gd.ksplit + k0 + i) * g.M + row) * g.N + col]
                                     : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 16; ++i) s = cadd(s, pv[i]);
    }
    cplx out = cmul(g.alpha, s);
    if (addc) out = cadd(out, cmul(g.beta, cprev));
    C[idx] = out;
  }
}

// The same product as its transpose: C^T = op(B)^T op(A)^T, with the result
// stored in the other orientation.
static void transpose_problem(ZGemm& g) {
  std::swap(g.A, g.B);
  g.A.trans ^= 1;
  g.B.trans ^= 1;
  std::swap(g.A2, g.B2);
  g.A2.trans ^= 1;
  g.B2.trans ^= 1;
  std::swap(g.M, g.N);
  g.transC ^= 1;
  std::swap(g.lower_only, g.upper_only);
}

// Operand extents of a product (host side, while operand checks are on):
// element (i, k), i < rows, k < cols, of o over `batch` batches.
static void require_op(const ZOp& o, long rows, long cols, int batch, const char* what) {
  if (rows <= 0 || cols <= 0) return;
  const long last = o.trans ? (cols - 1) * o.ld + (rows - 1) : (rows - 1) * o.ld + (cols - 1);
  const long bs = (long)(batch - 1) * o.stride;
  bounds_require(o.p, std::min(0L, bs), last + std::max(0L, bs), sizeof(cplx), what);
}

static void require_gemm_operands(const ZGemm& g, const cplx* partial, long partial_elems) {
  const long kc = g.kcat > 0 ? g.kcat : g.K;
  if (g.K > 0) {
    if (g.herm_a) {
      const long last = (long)(g.M - 1) * g.A.ld + (g.M - 1);
      const long bs = (long)(g.batch - 1) * g.A.stride;
      bounds_require(g.A.p, std::min(0L, bs), last + std::max(0L, bs), sizeof(cplx),
                     "product: Hermitian A");
    } else {
      require_op(g.A, g.M, kc, g.batch, "product: A");
      if (g.kcat > 0) require_op(g.A2, g.M, g.K - g.kcat, g.batch, "product: A2");
    }
    require_op(g.B, kc, g.N, g.batch, "product: B");
    if (g.kcat > 0 && !g.herm_a) require_op(g.B2, g.K - g.kcat, g.N, g.batch, "product: B2");
  }
  long clast;
  if (g.epi == EPI_THETA && g.swap)
    clast = ((long)(g.M - 1) / g.d1 * g.d2 + (g.N - 1) / g.b2) * ((long)g.d1 * g.b2) +
            (long)(g.d1 - 1) * g.b2 + (g.b2 - 1);
  else if (g.epi == EPI_THETA || !g.transC)
    clast = (long)(g.M - 1) * g.ldc + (g.N - 1);
  else
    clast = (long)(g.N - 1) * g.ldc + (g.M - 1);
  const long cs = (long)(g.batch - 1) * g.strideC;
  bounds_require(g.C, std::min(0L, cs), clast + std::max(0L, cs), sizeof(cplx), "product: C");
  if (g.epi == EPI_THETA && g.phase)
    bounds_require(g.phase, 0, (long)g.d1 * g.d2 - 1, sizeof(cplx), "product: phase table");
  if (partial && partial_elems > 0)
    bounds_require(partial, 0, partial_elems - 1, sizeof(cplx), "product: split-K partials");
}

void zgemm(const ZGemm& g0, cplx* partial, long partial_elems, hipStream_t s, Prof* prof) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return;
  if (bounds_checking()) require_gemm_operands(g0, partial, partial_elems);
  ZGemm g = g0;
  if (g.herm_a) {
    // only the plain float64 product with a row-major result
    g.prec = GEMM_F64;
    g.kcat = 0;
    g.transC = 0;
    g.K = g.M;
  }
  // A column-major result is stored as C^T, row-major, so that neighbouring
  // lanes write neighbouring addresses.
  if (g.transC && g.epi == EPI_STORE) transpose_problem(g);
  // A float64 result at most 32 rows high and wider than 32 is formed as its
  // transpose, whose at most 32 columns take the narrow wave layout (no MFMA
  // work on the empty half of each 64 x 64 tile); it is stored back through
  // transC.
  if (!g.herm_a && g.epi == EPI_STORE && g.prec == GEMM_F64 && !g.lower_only && !g.upper_only &&
      g.M <= 32 && g.N > 32)
    transpose_problem(g);
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
  // split-K for skinny outputs, until about 1024 workgroups run (four per
  // CU, so that operand loads overlap), in chunks of at least 256 (64 for a
  // handful of output tiles, whose K loop would otherwise run on a few dozen
  // workgroups)
  const long want = 1024;
  const long kmin = tiles <= 4 ? 64 : 256;
  if (partial && g.epi == EPI_STORE && !g.lower_only && !g.upper_only && !g.kcat &&
      (tiles < 128 || g.herm_a) && g.K >= 4 * kmin) {
    int ks = (int)std::min<long>(g.K / kmin, (want + tiles - 1) / tiles);
    while (ks > 1 && (long)ks * g.batch * g.M * g.N > partial_elems) --ks;
    if (ks > 1) {
      gd.ksplit = ks;
      gd.kchunk = ((g.K + ks - 1) / ks + BK2 - 1) / BK2 * BK2;
      gd.ksplit = (int)((g.K + gd.kchunk - 1) / gd.kchunk);
    }
  }
  dim3 grid(ceil_div(g.N, BN), ceil_div(g.M, BM), g.batch * gd.ksplit);
  const int ta = g.A.trans, tb = g.B.trans;
  const int pk = (prof && prof->kind == PROF_GEMM) ? PROF_GEMM : g.tag;
  double flops = 8.0 * g.M * (double)g.N * g.K * g.batch;
  if (g.lower_only || g.upper_only) flops = 8.0 * g.M * (g.M + 1.0) * 0.5 * g.K * g.batch;
  if (prof) prof->begin(pk, flops, s);
#define MPS_GEMM_DISPATCH(KER)                                                              \
  do {                                                                                      \
    if (ta == 0 && tb == 0) hipLaunchKernelGGL((KER<0, 0>), grid, dim3(256), 0, s, gd);     \
    else if (ta == 0 && tb == 1) hipLaunchKernelGGL((KER<0, 1>), grid, dim3(256), 0, s, gd); \
    else if (ta == 1 && tb == 0) hipLaunchKernelGGL((KER<1, 0>), grid, dim3(256), 0, s, gd); \
    else hipLaunchKernelGGL((KER<1, 1>), grid, dim3(256), 0, s, gd);                         \
  } while (0)
  const bool narrow = g.N <= 32 && g.epi == EPI_STORE;
  if (g.herm_a && narrow) {
    // 128 x 32 tiles; split K until about 1024 workgroups run
    const long htiles = (long)ceil_div(g.M, HM) * g.batch;
    ZGemmDev hd = gd;
    hd.ksplit = 1;
    hd.kchunk = g.K;
    if (partial && g.K >= 1024) {
      int ks = (int)std::min<long>(g.K / 256, (1024 + htiles - 1) / htiles);
      while (ks > 1 && (long)ks * g.batch * g.M * g.N > partial_elems) --ks;
      if (ks > 1) {
        hd.kchunk = ((g.K + ks - 1) / ks + BK2 - 1) / BK2 * BK2;
        hd.ksplit = (int)((g.K + hd.kchunk - 1) / hd.kchunk);
      }
    }
    dim3 hgrid(1, ceil_div(g.M, HM), g.batch * hd.ksplit);
    if (tb == 1) hipLaunchKernelGGL((zhemm_n32_kernel<1>), hgrid, dim3(256), 0, s, hd);
    else hipLaunchKernelGGL((zhemm_n32_kernel<0>), hgrid, dim3(256), 0, s, hd);
    if (hd.ksplit > 1) {
      long total = (long)g.M * g.N;
      int blocks = (int)std::min<long>((total + 255) / 256, 4096);
      hipLaunchKernelGGL(zgemm_reduce, dim3(blocks, g.batch), dim3(256), 0, s, hd);
    }
    if (prof) prof->end(pk, flops, s);
    return;
  }
  if (g.herm_a) {
    if (tb == 0) hipLaunchKernelGGL((zgemm_kernel<2, 0>), grid, dim3(256), 0, s, gd);
    else hipLaunchKernelGGL((zgemm_kernel<2, 1>), grid, dim3(256), 0, s, gd);
  } else if (narrow && g.prec == GEMM_F64) {
    if (ta == 0 && tb == 0) hipLaunchKernelGGL((zgemm_kernel<0, 0, 1>), grid, dim3(256), 0, s, gd);
    else if (ta == 0 && tb == 1) hipLaunchKernelGGL((zgemm_kernel<0, 1, 1>), grid, dim3(256), 0, s, gd);
    else if (ta == 1 && tb == 0) hipLaunchKernelGGL((zgemm_kernel<1, 0, 1>), grid, dim3(256), 0, s, gd);
    else hipLaunchKernelGGL((zgemm_kernel<1, 1, 1>), grid, dim3(256), 0, s, gd);
  } else if (g.prec == GEMM_F32) MPS_GEMM_DISPATCH(cgemm_f32_kernel);
  else if (g.prec == GEMM_BF16X3) MPS_GEMM_DISPATCH(cgemm_bf16x3_kernel);
  else MPS_GEMM_DISPATCH(zgemm_kernel);
#undef MPS_GEMM_DISPATCH
  if (gd.ksplit > 1) {
    long total = (long)g.M * g.N;
    int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(zgemm_reduce, dim3(blocks, g.batch), dim3(256), 0, s, gd);
  }
  if (prof) prof->end(pk, flops, s);
}

}  // namespace mpsim
