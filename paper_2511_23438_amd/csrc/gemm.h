// Complex float64 GEMM on gfx950 MFMA (v_mfma_f64_16x16x4f64).
#pragma once
#include "common.h"
#include "prof.h"

namespace mpsim {

// Logical operand: element (i, k) = trans ? p[k*ld + i] : p[i*ld + k], optionally conjugated.
struct ZOp {
  const cplx* p;
  long ld;
  long stride;  // batch stride (elements)
  int trans;
  int conj;
};

enum { EPI_STORE = 0, EPI_THETA = 1 };
// arithmetic of the product: float64, complex64 with FP32 accumulation, or a
// three-term bf16 split of each float64 operand (x = hi + mid + lo, each term
// the bf16 rounding of what the previous terms leave) whose six leading
// products (hh, hm, mh, hl, lh, mm) are accumulated in FP32
enum { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16X3 = 2 };

struct ZGemm {
  int M, N, K, batch;
  ZOp A, B;
  cplx* C;
  long ldc, strideC;
  int transC;       // logical (i, j) stored at transC ? C[j*ldc + i] : C[i*ldc + j]
  cplx alpha, beta;
  int lower_only;   // skip output tiles strictly above the diagonal
  int upper_only;   // skip output tiles strictly below the diagonal
  int epi;          // EPI_STORE or EPI_THETA
  // theta epilogue: row = a*d1 + s1, col = s2*b2 + g; value *= phase[s1][s2]
  // (phase_trans: phase[s2][s1]); swap: store at (a*d2 + s2, s1*b2 + g), ld d1*b2
  const cplx* phase;
  int phase_trans, d1, d2, b2, swap;
  int tag;          // launch class for the profiler (PROF_GRAM, PROF_THETA or 0)
  int prec;         // GEMM_F64 (default), GEMM_F32 or GEMM_BF16X3
  // optional second K segment: for k >= kcat the operands are A2 (i, k - kcat)
  // and B2 (k - kcat, j); A2/B2 share the trans and conj flags of A/B
  int kcat;
  ZOp A2, B2;
  // herm_a: op(A) is the M x M Hermitian matrix whose lower triangle is
  // stored column-major at A.p (ld A.ld); A.trans / A.conj are ignored.
  // Float64 only, row-major C, no second K segment.
  int herm_a;
};

// C = alpha*op(A)*op(B) + beta*C (or the theta epilogue). `partial` is a
// workspace of at least `partial_elems` complex values used for split-K on
// skinny outputs (may be NULL to disable split-K).
void zgemm(const ZGemm& g, cplx* partial, long partial_elems, hipStream_t s,
           Prof* prof = nullptr);

inline ZGemm zgemm_args(int M, int N, int K, ZOp A, ZOp B, cplx* C, long ldc, int transC,
                        cplx alpha, cplx beta) {
  ZGemm g{};
  g.M = M; g.N = N; g.K = K; g.batch = 1;
  g.A = A; g.B = B; g.C = C; g.ldc = ldc; g.transC = transC;
  g.alpha = alpha; g.beta = beta;
  g.epi = EPI_STORE;
  return g;
}

inline ZOp zop(const cplx* p, long ld, int trans, int conj = 0) {
  ZOp o{p, ld, 0, trans, conj};
  return o;
}

}  // namespace mpsim
