// Two-stage path to the top-q eigenspace of a Hermitian matrix (float64).
//
//   1. Dense -> band of half-width HB: for every panel of HB columns, a
//      Householder QR of the block below the band and the two-sided update
//      of the trailing matrix, A22 <- Q^H A22 Q = A22 - V W^H - W V^H with
//      W = A22 V T - 1/2 V T^H V^H A22 V T. The products run on MFMA GEMMs
//      (A22 V reads the stored lower triangle as a Hermitian operand), and
//      the rank-2k updates of a group of panels are applied together, so
//      the trailing matrix is read about 1.5 times per panel instead of once
//      per column as in the one-stage reduction.
//   2. Band -> real tridiagonal by bulge chasing, eigenvalues only. Sweep j
//      removes column j below the subdiagonal and chases the bulge down in
//      steps of HB rows. Each step touches a window of at most 2HB x 2HB
//      entries; sweep j+1 runs three steps behind sweep j, which keeps the
//      windows of one time slot disjoint, so one launch per time slot runs
//      all of its steps as independent workgroups.
//   3. Eigenvalues of the tridiagonal by bisection (shared with the one-stage
//      path).
//   4. Eigenvectors of the band matrix by inverse iteration: band LU with
//      partial pivoting of B - lambda I (one wave per vector, the active
//      window in LDS), back substitution, two iterations; then Householder QR
//      of the vectors (only the spanned subspace matters) and the stage-1
//      block reflectors applied in reverse order.
#include "linalg.h"

#include <algorithm>
#include <cfloat>

namespace mpsim {

constexpr int HB = TRD_NB;        // band half-width
constexpr int ABW = 2 * HB + 1;   // stored sub-diagonal offsets per band column
constexpr int URW = 2 * HB + 2;   // stored U row: 2HB+1 entries and the RHS value

static_assert(HB == 32, "the band kernels assume a half-width of 32");

// ---------------------------------------------------------------------------
// Stage 1

// Band of the reduced matrix: Ab[j*ABW + o] = A[j + o, j] for o <= HB, zero
// for the offsets that fill-in may reach later; diagonal made real.
__global__ void k_band_extract(int n, const cplx* A, long lda, cplx* Ab) {
  const long total = (long)n * ABW;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long j = idx / ABW;
    const int o = (int)(idx % ABW);
    cplx v = make_double2(0.0, 0.0);
    if (o <= HB && j + o < n) {
      v = A[j * lda + j + o];
      if (o == 0) v.y = 0.0;
    }
    Ab[idx] = v;
  }
}

// Panels are taken in groups of HB_GROUP. Within a group the trailing matrix
// is not rewritten: the group's reflectors V and their W accumulate, each
// panel's columns get the earlier updates of the group before its QR, and the
// product A22 V is formed from the stored matrix and corrected,
//   A22 V = A22_stored V - Vg (Wg^H V) - Wg (Vg^H V).
// One rank-2*HB*HB_GROUP update per group then brings the trailing matrix up
// to date, so it is read and written once per group instead of once per panel.
void he2hb_lower(int n, cplx* A, long lda, LinalgWork& w, hipStream_t s) {
  const cplx one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  const cplx mone = make_double2(-1.0, 0.0);
  constexpr int KG = HB_GROUP * HB;
  const long ld = w.nmax;                      // accumulator rows, offset by the group base
  cplx* Vg = w.acc;                            // ld x KG
  cplx* Wg = w.acc + ld * KG;                  // ld x KG
  cplx* Pw = w.acc + 2 * ld * KG;              // KG x HB row-major: Wg^H V
  cplx* Pv = Pw + (long)KG * HB;               // KG x HB row-major: Vg^H V
  int p = 0, i0 = 0;
  while (i0 + HB < n - 1) {
    const int base = i0 + HB;                  // first row of the group's reflectors
    int ka = 0;
    for (int g = 0; g < HB_GROUP && i0 + HB < n - 1; ++g, ++p, i0 += HB) {
      const int o = i0 + HB;
      const int m = n - o;
      const int kb = std::min(HB, m);
      cplx* T = w.T1 + (long)p * 4096;
      cplx* A22 = A + (long)o * lda + o;
      if (ka > 0) {
        // columns i0..i0+HB-1 (rows i0..n-1) receive the group's earlier updates
        const long r0 = i0 - base;
        ZGemm gc = zgemm_args(n - i0, HB, 2 * ka, zop(Vg + r0, ld, 1), zop(Wg + r0, ld, 0, 1),
                              A + (long)i0 * lda + i0, lda, 1, mone, one);
        gc.kcat = ka;
        gc.A2 = zop(Wg + r0, ld, 1);
        gc.B2 = zop(Vg + r0, ld, 0, 1);
        zgemm(gc, nullptr, 0, s, w.prof);
      }
      // panel QR; the explicit V (m x kb) lands in column ka of Vg
      cplx* V = Vg + (long)ka * ld + (o - base);
      cplx* W = Wg + (long)ka * ld + (o - base);
      LinalgWork wp = w;
      wp.T = T;
      wp.V = V;
      wp.vmax = ld;
      qr_factor(m, HB, A + (long)i0 * lda + o, 1, lda, wp, s);
      // X = A22 V (row-major, ld 64) from the stored lower triangle
      ZGemm gx = zgemm_args(m, kb, m, zop(A22, lda, 1), zop(V, ld, 1), w.X2, 64, 0, one, zero);
      gx.herm_a = 1;
      zgemm(gx, w.gpart, w.gpart_elems, s, w.prof);
      if (ka > 0) {
        const long r0 = o - base;
        // Pw = Wg^H V and Pv = Vg^H V as one batch of two (same V)
        ZGemm gp = zgemm_args(ka, kb, m, zop(Wg + r0, ld, 0, 1), zop(V, ld, 1), Pw, HB, 0, one,
                              zero);
        gp.batch = 2;
        gp.A.stride = (long)(Vg - Wg);
        gp.strideC = (long)(Pv - Pw);
        zgemm(gp, w.gpart, w.gpart_elems, s, w.prof);
        ZGemm gxc = zgemm_args(m, kb, 2 * ka, zop(Vg + r0, ld, 1), zop(Pw, HB, 0), w.X2, 64, 0, mone,
                               one);
        gxc.kcat = ka;
        gxc.A2 = zop(Wg + r0, ld, 1);
        gxc.B2 = zop(Pv, HB, 0);
        zgemm(gxc, nullptr, 0, s, w.prof);
      }
      // Y = X T (column-major, in column ka of Wg)
      ZGemm gy = zgemm_args(m, kb, kb, zop(w.X2, 64, 0), zop(T, 64, 0), W, ld, 1, one, zero);
      zgemm(gy, nullptr, 0, s, w.prof);
      // S = V^H Y, Z = T^H S
      ZGemm gs = zgemm_args(kb, kb, m, zop(V, ld, 0, 1), zop(W, ld, 1), w.S, 64, 0, one, zero);
      zgemm(gs, w.gpart, w.gpart_elems, s, w.prof);
      ZGemm gz = zgemm_args(kb, kb, kb, zop(T, 64, 1, 1), zop(w.S, 64, 0), w.S2, 64, 0, one, zero);
      zgemm(gz, nullptr, 0, s, w.prof);
      // W = Y - 1/2 V Z (in place)
      ZGemm gw = zgemm_args(m, kb, kb, zop(V, ld, 1), zop(w.S2, 64, 0), W, ld, 1,
                            make_double2(-0.5, 0.0), one);
      zgemm(gw, nullptr, 0, s, w.prof);
      ka += kb;
    }
    // trailing matrix from the next panel's first column: A22 -= [Vg Wg] [Wg Vg]^H
    const int o2 = i0;
    const int m2 = n - o2;
    if (m2 > 0) {
      const long r0 = o2 - base;
      cplx* A22 = A + (long)o2 * lda + o2;
      ZGemm g1 = zgemm_args(m2, m2, 2 * ka, zop(Vg + r0, ld, 1), zop(Wg + r0, ld, 0, 1), A22, lda, 1,
                            mone, one);
      g1.kcat = ka;
      g1.A2 = zop(Wg + r0, ld, 1);
      g1.B2 = zop(Vg + r0, ld, 0, 1);
      g1.lower_only = 1;
      zgemm(g1, nullptr, 0, s, w.prof);
    }
  }
}

// Block factor of two consecutive panels a, b: with H_a = I - Va Ta Va^H and
// H_b = I - Vb Tb Vb^H, H_a H_b = I - [Va Vb] T [Va Vb]^H for
// T = [[Ta, -Ta S Tb], [0, Tb]], S = Va^H Vb (HB x kb2, row-major ld 64).
// Ta, Tb and T are row-major in 64 x 64 blocks; T is zero past HB + kb2.
__global__ __launch_bounds__(256) void k_pair_t(const cplx* Ta, const cplx* Tb, const cplx* S, int kb2,
                                                cplx* T) {
  __shared__ cplx ta[HB][HB + 1], tb[HB][HB + 1], sm[HB][HB + 1], y[HB][HB + 1];
  const int t = threadIdx.x;
  const cplx zero = make_double2(0.0, 0.0);
  for (int e = t; e < HB * HB; e += 256) {
    const int i = e / HB, j = e % HB;
    ta[i][j] = Ta[i * 64 + j];
    tb[i][j] = (i < kb2 && j < kb2) ? Tb[i * 64 + j] : zero;
    sm[i][j] = (j < kb2) ? S[i * 64 + j] : zero;
  }
  __syncthreads();
  for (int e = t; e < HB * HB; e += 256) {
    const int i = e / HB, j = e % HB;
    cplx acc = zero;
    for (int l = 0; l < HB; ++l) acc = cadd(acc, cmul(ta[i][l], sm[l][j]));
    y[i][j] = acc;
  }
  __syncthreads();
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    cplx v = zero;
    if (i < HB && j < HB) {
      v = ta[i][j];
    } else if (i < HB) {
      cplx acc = zero;
      for (int l = 0; l < HB; ++l) acc = cadd(acc, cmul(y[i][l], tb[l][j - HB]));
      v = make_double2(-acc.x, -acc.y);
    } else if (j >= HB) {
      v = tb[i - HB][j - HB];
    }
    T[i * 64 + j] = v;
  }
}

// X (n x q row-major) <- Q1 X, Q1 = H_0 H_1 ... the product of the stage-1
// panel reflectors (stored below the band of A, block factors in w.T1).
// Panels are applied two at a time (the last one alone when their number is
// odd): the reflectors of panels a and a + 1 form one unit lower trapezoidal
// block of up to 2 HB columns from row a HB + HB, so X is read and written
// once per pair.
void he2hb_backtransform(int n, const cplx* A, long lda, int q, cplx* X, long ldx, LinalgWork& w,
                         hipStream_t s) {
  const cplx one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  int np = 0;
  for (int i0 = 0; i0 + HB < n - 1; i0 += HB) ++np;
  int p = np - 1;
  if (np % 2 == 1) {
    const int i0 = p * HB, o = i0 + HB, m = n - o;
    const int kb = std::min(HB, m);
    extract_v(A, 1, lda, o, i0, m, kb, w.V, w.vmax, s);
    apply_block_reflector(m, q, kb, w.T1 + (long)p * 4096, 0, X + (long)o * ldx, ldx, 1, w, s);
    --p;
  }
  for (; p >= 1; p -= 2) {
    const int a = p - 1;
    const int i0 = a * HB, o = i0 + HB, m = n - o;
    const int kb2 = std::min(HB, m - HB);
    const int ib = HB + kb2;
    extract_v(A, 1, lda, o, i0, m, ib, w.V, w.vmax, s);
    // S = Va^H Vb (HB x kb2, ld 64)
    ZGemm gs = zgemm_args(HB, kb2, m, zop(w.V, w.vmax, 0, 1), zop(w.V + (long)HB * w.vmax, w.vmax, 1),
                          w.S, 64, 0, one, zero);
    zgemm(gs, w.gpart, w.gpart_elems, s, w.prof);
    hipLaunchKernelGGL(k_pair_t, dim3(1), dim3(256), 0, s, (const cplx*)(w.T1 + (long)a * 4096),
                       (const cplx*)(w.T1 + (long)(a + 1) * 4096), (const cplx*)w.S, kb2, w.T);
    apply_block_reflector(m, q, ib, w.T, 0, X + (long)o * ldx, ldx, 1, w, s);
  }
}

// ---------------------------------------------------------------------------
// Stage 2: bulge chasing on the band (lower storage Ab[col*ABW + row - col])

__device__ inline int hb_steps(int n, int j) { return (n - 1 - j + HB - 1) / HB; }

// One step of sweep j = jlo + blockIdx.x at time slot `slot` (step k =
// slot - 3j): reflector from column c, rows r..r+L-1; applied from the left
// to rows R = [r, r+L) of columns c+1..r-1 (block Bl), from both sides to the
// diagonal block R x R (D), and from the right to rows [r+L, r+L+Lb) of
// columns R (Bb). Thread t keeps the elements (t % 32, t / 32 + 8 it) of the
// three blocks in registers for the update; LDS holds copies for the
// products, which 8-lane groups form in four-term pieces.
__global__ __launch_bounds__(256) void k_hb2st(int n, cplx* Ab, int slot, int jlo) {
  const int j = jlo + blockIdx.x;
  if (j > n - 3) return;
  const int k = slot - 3 * j;
  if (k < 0 || k >= hb_steps(n, j)) return;
  const int r = j + 1 + k * HB;
  const int c = (k == 0) ? j : r - HB;
  const int L = min(HB, n - r);
  if (L < 2) return;
  const int Lb = min(HB, n - r - L);
  const int nl = r - c - 1;
  __shared__ cplx Bl[HB][HB + 1];
  __shared__ cplx D[HB][HB + 1];
  __shared__ cplx Bb[HB][HB + 1];
  __shared__ cplx x[HB], v[HB], pv[HB], qv[HB], wl[HB];
  __shared__ double sc[8];
  __shared__ double ssum[4];
  const int t = threadIdx.x, lane = t & 63;
  const int ri = t % HB, cj0 = t / HB;
#define AB(row, col) Ab[(long)(col) * ABW + ((row) - (col))]
  cplx rl[4], rd[4], rb[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int jj = cj0 + 8 * it;
    rl[it] = (ri < L && jj < nl) ? AB(r + ri, c + 1 + jj) : make_double2(0.0, 0.0);
    rd[it] = (ri < L && jj < L && ri >= jj) ? AB(r + ri, r + jj) : make_double2(0.0, 0.0);
    rb[it] = (ri < Lb && jj < L) ? AB(r + L + ri, r + jj) : make_double2(0.0, 0.0);
  }
  if (t < HB) x[t] = (t < L) ? AB(r + t, c) : make_double2(0.0, 0.0);
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int jj = cj0 + 8 * it;
    Bl[ri][jj] = rl[it];
    Bb[ri][jj] = rb[it];
    if (ri == jj) rd[it].y = 0.0;
    if (ri >= jj) {
      D[ri][jj] = rd[it];
      D[jj][ri] = cconj(rd[it]);
    }
  }
  __syncthreads();
  if (t < 64) {
    // reflector; lanes 0..L-1 then form v
    double xn = (t >= 1 && t < L) ? cabs2(x[t]) : 0.0;
    xn = wave_sum(xn);
    double beta = 0.0;
    cplx tau = make_double2(0.0, 0.0), scl = make_double2(0.0, 0.0);
    if (t == 0) reflector(x[0], xn, beta, tau, scl);
    scl.x = wave_bcast0(scl.x);
    scl.y = wave_bcast0(scl.y);
    if (t < HB) v[t] = (t == 0) ? make_double2(1.0, 0.0) : (t < L ? cmul(x[t], scl) : make_double2(0.0, 0.0));
    if (t == 0) {
      sc[0] = beta; sc[1] = tau.x; sc[2] = tau.y;
    }
  }
  __syncthreads();
  {
    // row / column q = t / 8 of the products, terms 4 (t % 8) .. 4 (t % 8) + 3
    const int q = t >> 3, part = t & 7;
    cplx pp = make_double2(0.0, 0.0), qq = pp, ww = pp;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = part * 4 + u;
      const cplx vm = v[m];
      pp = cadd(pp, cmul(D[q][m], vm));
      qq = cadd(qq, cmul(Bb[q][m], vm));
      ww = cadd(ww, cmulc(vm, Bl[m][q]));
    }
    // v^H D v (real): every piece of p times conj(v_q)
    double sp = cmulc(v[q], pp).x;
    pp.x = oct_sum(pp.x);
    pp.y = oct_sum(pp.y);
    qq.x = oct_sum(qq.x);
    qq.y = oct_sum(qq.y);
    ww.x = oct_sum(ww.x);
    ww.y = oct_sum(ww.y);
    if (part == 0) {
      pv[q] = pp;
      qv[q] = qq;
      wl[q] = ww;
    }
    sp = wave_sum(sp);
    if (lane == 0) ssum[t >> 6] = sp;
  }
  __syncthreads();
  const cplx tau = make_double2(sc[1], sc[2]);
  const cplx ctau = cconj(tau);
  const double hs = 0.5 * cabs2(tau) * (ssum[0] + ssum[1] + ssum[2] + ssum[3]);
  // w = tau p - 1/2 |tau|^2 (v^H p) v
  const cplx vi = v[ri];
  const cplx wi = csub(cmul(tau, pv[ri]), cscale(vi, hs));
  const cplx qi = qv[ri];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int jj = cj0 + 8 * it;
    const cplx vj = v[jj];
    if (ri < L && jj < nl) AB(r + ri, c + 1 + jj) = csub(rl[it], cmul(ctau, cmul(vi, wl[jj])));
    if (ri < L && jj < L && ri >= jj) {
      const cplx wj = csub(cmul(tau, pv[jj]), cscale(vj, hs));
      cplx dv = csub(rd[it], cadd(cmul(wi, cconj(vj)), cmul(vi, cconj(wj))));
      if (ri == jj) dv.y = 0.0;
      AB(r + ri, r + jj) = dv;
    }
    if (ri < Lb && jj < L) AB(r + L + ri, r + jj) = csub(rb[it], cmul(tau, cmul(qi, cconj(vj))));
  }
  if (t < L) AB(r + t, c) = (t == 0) ? make_double2(sc[0], 0.0) : make_double2(0.0, 0.0);
#undef AB
}

__global__ void k_hb_tridiag(int n, const cplx* Ab, double* d, double* e) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    d[i] = Ab[(long)i * ABW].x;
    if (i < n - 1) e[i] = sqrt(cabs2(Ab[(long)i * ABW + 1]));
  }
}

static void hb2st_launches(int n, cplx* Ab, hipStream_t s) {
  if (n < 3) return;
  const int st0 = (n - 1 + HB - 1) / HB;  // steps of sweep 0 (the most)
  int nslots = 0;
  for (int j = 0; j <= n - 3; ++j) nslots = std::max(nslots, 3 * j + (n - 1 - j + HB - 1) / HB);
  for (int slot = 0; slot < nslots; ++slot) {
    const int jhi = std::min(n - 3, slot / 3);
    const int jlo = std::max(0, (slot - st0 + 1 + 2) / 3);
    if (jhi < jlo) continue;
    hipLaunchKernelGGL(k_hb2st, dim3(jhi - jlo + 1), dim3(256), 0, s, n, Ab, slot, jlo);
  }
}

// The launch sequence depends only on n and the band's address, so it is
// captured once into a HIP graph (on a private stream) and replayed; if
// capture or instantiation fails the kernels are launched directly.
static hipGraphExec_t hb2st_graph(int n, cplx* Ab, LinalgWork& w, hipStream_t s) {
  for (auto& g : w.hbg)
    if (g.exec && g.n == n && g.ab == Ab) return g.exec;
  if (!w.cap_stream && hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking) != hipSuccess) {
    w.cap_stream = nullptr;
    return nullptr;
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(w.cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
  hb2st_launches(n, Ab, w.cap_stream);
  if (hipStreamEndCapture(w.cap_stream, &graph) != hipSuccess || !graph) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return nullptr;
  }
  auto& slot = w.hbg[w.hbg_next];
  w.hbg_next = (w.hbg_next + 1) % 2;
  // the evicted graph may still be queued or running on the handle's stream
  if (slot.exec) (void)hipStreamSynchronize(s);
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  if (slot.graph) (void)hipGraphDestroy(slot.graph);
  slot.n = n;
  slot.ab = Ab;
  slot.graph = graph;
  slot.exec = exec;
  return exec;
}

void hb2st(int n, cplx* Ab, LinalgWork& w, hipStream_t s) {
  if (n >= 3) {
    hipGraphExec_t exec = hb2st_graph(n, Ab, w, s);
    if (!exec || hipGraphLaunch(exec, s) != hipSuccess) {
      (void)hipGetLastError();
      hb2st_launches(n, Ab, s);
    }
  }
  hipLaunchKernelGGL(k_hb_tridiag, dim3(std::max(1, std::min(ceil_div(n, 256), 1024))), dim3(256), 0,
                     s, n, (const cplx*)Ab, w.d, w.e);
}

void linalg_release(LinalgWork& w) {
  for (auto& g : w.hbg) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = LinalgWork::HbGraph{};
  }
  if (w.cap_stream) (void)hipStreamDestroy(w.cap_stream);
  w.cap_stream = nullptr;
}

// ---------------------------------------------------------------------------
// Band inverse iteration

// Row-major copy of the Hermitian band: Br[i*ABW + o] = B[i, i - HB + o].
__global__ void k_band_rows(int n, const cplx* Ab, cplx* Br) {
  const long total = (long)n * ABW;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long i = idx / ABW;
    const int o = (int)(idx % ABW);
    const long jc = i - HB + o;
    cplx v = make_double2(0.0, 0.0);
    if (jc >= 0 && jc < n) {
      if (jc <= i) v = Ab[jc * ABW + (i - jc)];
      else v = cconj(Ab[i * ABW + (jc - i)]);
    }
    Br[idx] = v;
  }
}

__device__ inline double band_hash(uint64_t seed, uint64_t a, uint64_t b) {
  uint64_t z = seed ^ (a * 0x9E3779B97F4A7C15ULL) ^ (b * 0xC2B2AE3D27D4EB4FULL);
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

template <int M>
__device__ inline void argmax_step(double& best, int& bi) {
  const double ob = lane_xch<M>(best);
  const int oi = lane_xch<M>(bi);
  if (ob > best || (ob == best && oi < bi)) {
    best = ob;
    bi = oi;
  }
}

constexpr int WR = HB + 1;        // window rows
constexpr int WC = 2 * HB + 1;    // window columns
constexpr int CH = 4;             // rows staged per chunk (LDS: 4 waves per CU)
constexpr int LRW = HB + 1;       // stored L row: HB multipliers, then the pivot offset
constexpr int CHL = 16;           // L rows loaded ahead in the substitution-only passes

// One wave per eigenvector (vector index v0 + blockIdx.x, column kq of X for
// the kq-th largest eigenvalue). Window W[row % WR][col % WC] holds rows
// k..k+HB and columns k..k+2HB of the partially eliminated B - lambda I.
// The first pass factors B - lambda I and keeps U (with the transformed
// right-hand side) and L (multipliers and pivot offset per row); later passes
// only repeat the forward substitution with the kept L on the new
// right-hand side, the same operations on the same values as a refactoring.
__global__ __launch_bounds__(64) void k_band_invit(int n, const cplx* Br, int q, const double* lam,
                                                  int lam_off, const double* bounds, cplx* Ubuf,
                                                  int v0, cplx* X, long ldx, uint64_t seed,
                                                  int iters) {
  __shared__ cplx Wn[WR][WC];
  __shared__ cplx yv[WR];
  __shared__ cplx lb[HB];
  __shared__ cplx stage[CH][URW];
  const int kq = v0 + blockIdx.x;
  if (kq >= q) return;
  const int l = threadIdx.x;
  cplx* U = Ubuf + (long)blockIdx.x * n * (URW + LRW);
  cplx* Lr = U + (long)n * URW;
  const double lmb = lam[lam_off + q - 1 - kq];
  double epsp = DBL_EPSILON * bounds[2];
  if (epsp == 0.0) epsp = DBL_MIN;
  for (int it = 0; it < iters; ++it) {
    if (it == 0) {
      // ---- forward: LU with partial pivoting, RHS carried along
      for (int e = l; e < WR * WC; e += 64) Wn[e / WC][e % WC] = make_double2(0.0, 0.0);
      __syncthreads();
      // rows 0..HB: B[i, jc] for jc in [0, 2HB] (Br offset o = jc - i + HB)
      for (int e = l; e < WR * WC; e += 64) {
        const int i = e / WC, jc = e % WC;
        if (i < n && jc < n) {
          const int o = jc - i + HB;
          if (o >= 0 && o < ABW) {
            cplx b = Br[(long)i * ABW + o];
            if (o == HB) b.x -= lmb;
            Wn[i % WR][jc % WC] = b;
          }
        }
      }
      if (l < WR && l < n) {
        if (it == 0) yv[l] = make_double2(band_hash(seed, (uint64_t)kq, (uint64_t)l), 0.0);
        else yv[l] = X[(long)l * ldx + kq];
      }
      // rows entering the window in chunk kc (rows kc+WR .. kc+WR+CH-1): loaded
      // into registers one chunk ahead, so the loads are in flight while the
      // previous chunk's rows are eliminated; the shift by lambda is applied
      // when they are written to LDS
      constexpr int NPF = (CH * ABW + 63) / 64;
      cplx pf[NPF], pfy = make_double2(0.0, 0.0);
      auto fetch = [&](int kc) {
  #pragma unroll
        for (int j = 0; j < NPF; ++j) {
          const int e = l + 64 * j;
          const long i = (long)kc + WR + e / ABW;
          pf[j] = make_double2(0.0, 0.0);
          if (e < CH * ABW && i < n) pf[j] = Br[i * ABW + e % ABW];
        }
        pfy = make_double2(0.0, 0.0);
        if (l < CH) {
          const long i = (long)kc + WR + l;
          if (i < n) {
            if (it == 0) pfy = make_double2(band_hash(seed, (uint64_t)kq, (uint64_t)i), 0.0);
            else pfy = X[i * ldx + kq];
          }
        }
      };
      auto stage_fetched = [&](int kc) {
  #pragma unroll
        for (int j = 0; j < NPF; ++j) {
          const int e = l + 64 * j;
          if (e < CH * ABW) {
            cplx b = pf[j];
            if (e % ABW == HB && (long)kc + WR + e / ABW < n) b.x -= lmb;
            stage[e / ABW][e % ABW] = b;
          }
        }
        if (l < CH) stage[l][ABW] = pfy;
      };
      fetch(0);
      __syncthreads();
      stage_fetched(0);
      __syncthreads();
      for (int k0 = 0; k0 < n; k0 += CH) {
        const bool more = k0 + CH < n;
        if (more) fetch(k0 + CH);
        const int kend = min(n, k0 + CH);
        for (int k = k0; k < kend; ++k) {
          const int cs = k % WC;
          // pivot: largest |W[i][k]| over rows k..min(n-1, k+HB)
          double best = -1.0;
          int bi = k;
          if (l < WR && k + l < n) {
            best = cabs2(Wn[(k + l) % WR][cs]);
            bi = k + l;
          }
          // (largest |W|^2, then lowest row): the same in every lane whatever
          // the exchange order
          argmax_step<1>(best, bi);
          argmax_step<2>(best, bi);
          argmax_step<4>(best, bi);
          argmax_step<8>(best, bi);
          argmax_step<16>(best, bi);
          argmax_step<32>(best, bi);
          const int ks = k % WR;
          if (bi != k) {
            const int ps = bi % WR;
            for (int cc = l; cc < WC; cc += 64) {
              const cplx a = Wn[ks][cc];
              Wn[ks][cc] = Wn[ps][cc];
              Wn[ps][cc] = a;
            }
            if (l == 0) {
              const cplx a = yv[ks];
              yv[ks] = yv[ps];
              yv[ps] = a;
            }
          }
          __syncthreads();
          cplx ukk = Wn[ks][cs];
          if (cabs2(ukk) < epsp * epsp) ukk = make_double2(ukk.x < 0.0 ? -epsp : epsp, 0.0);
          const cplx yk = yv[ks];
          // U row k: offsets 0..2HB, then the eliminated RHS value
          for (int o = l; o < WC; o += 64) U[(long)k * URW + o] = (o == 0) ? ukk : Wn[ks][(k + o) % WC];
          if (l == 0) U[(long)k * URW + WC] = yk;
          // multipliers of rows k+1..k+HB (kept with the pivot offset)
          if (l < HB) {
            const int i = k + 1 + l;
            cplx li = make_double2(0.0, 0.0);
            if (i < n) li = cmul(Wn[i % WR][cs], cinv(ukk));
            lb[l] = li;
            Lr[(long)k * LRW + l] = li;
            if (i < n) yv[i % WR] = csub(yv[i % WR], cmul(li, yk));
          }
          if (l == HB) Lr[(long)k * LRW + HB] = make_double2((double)(bi - k), 0.0);
          __syncthreads();
          {
            // lane l updates column k+1+l of rows k+1..k+HB, eight rows at a
            // time: all reads of a group, then all writes (rows past n hold
            // zeros and zero multipliers, so they are updated harmlessly)
            const int cl = (k + 1 + l) % WC;
            const cplx u = Wn[ks][cl];
            int slot = (k + 1) % WR;
  #pragma unroll
            for (int g8 = 0; g8 < HB / 8; ++g8) {
              cplx wv[8], lv[8];
              int sl[8];
  #pragma unroll
              for (int q = 0; q < 8; ++q) {
                sl[q] = slot;
                slot = (slot + 1 == WR) ? 0 : slot + 1;
                lv[q] = lb[g8 * 8 + q];
                wv[q] = Wn[sl[q]][cl];
              }
  #pragma unroll
              for (int q = 0; q < 8; ++q) Wn[sl[q]][cl] = csub(wv[q], cmul(lv[q], u));
            }
          }
          __syncthreads();
          // advance: row k+WR takes row k's slot, column k+WC takes column k's
          {
            const int ni = k + WR;
            const int rr = ni - (k0 + WR);   // its index in the staged chunk
            for (int cc = l; cc < WC; cc += 64) {
              // column index of slot cc in the new window [k+1, k+WC]
              const int jc = k + 1 + ((cc - (k + 1) % WC) + WC) % WC;
              cplx b = make_double2(0.0, 0.0);
              if (ni < n) {
                const int o = jc - ni + HB;
                if (o >= 0 && o < ABW) b = stage[rr][o];
              }
              Wn[ks][cc] = b;
            }
            // the entering column is zero in every other row
            for (int i2 = l; i2 < WR; i2 += 64)
              if (i2 != ks) Wn[i2][cs] = make_double2(0.0, 0.0);
            if (l == 0) yv[ks] = (ni < n) ? stage[rr][ABW] : make_double2(0.0, 0.0);
          }
          __syncthreads();
        }
        if (more) {
          stage_fetched(k0 + CH);
          __syncthreads();
        }
      }
    } else {
      // ---- forward substitution with the kept L on the right-hand side X
      if (l < WR && l < n) yv[l] = X[(long)l * ldx + kq];
      // lane l < LRW holds entry l of the chunk's L rows; lane j < CHL the
      // right-hand side of row k0 + WR + j, which enters after row k0 + j
      cplx lc[CHL], ln[CHL], xc, xn;
      auto fetch_l = [&](int k0, cplx (&dst)[CHL], cplx& xv) {
#pragma unroll
        for (int j = 0; j < CHL; ++j)
          dst[j] = (l < LRW && k0 + j < n) ? Lr[(long)(k0 + j) * LRW + l] : make_double2(0.0, 0.0);
        const long ie = (long)k0 + WR + l;
        xv = (l < CHL && ie < n) ? X[ie * ldx + kq] : make_double2(0.0, 0.0);
      };
      fetch_l(0, lc, xc);
      __syncthreads();
      for (int k0 = 0; k0 < n; k0 += CHL) {
        if (k0 + CHL < n) fetch_l(k0 + CHL, ln, xn);
#pragma unroll
        for (int j = 0; j < CHL; ++j) {
          const int k = k0 + j;
          if (k < n) {
            const int ks = k % WR;
            const int po = (int)wave_readlane(lc[j].x, HB);
            if (po != 0 && l == 0) {
              const int ps = (k + po) % WR;
              const cplx a = yv[ks];
              yv[ks] = yv[ps];
              yv[ps] = a;
            }
            __syncthreads();
            const cplx yk = yv[ks];
            if (l == 0) U[(long)k * URW + WC] = yk;
            if (l < HB && k + 1 + l < n) {
              const int is = (k + 1 + l) % WR;
              yv[is] = csub(yv[is], cmul(lc[j], yk));
            }
            __syncthreads();
            if (l == j) yv[ks] = xc;
            __syncthreads();
          }
        }
#pragma unroll
        for (int j = 0; j < CHL; ++j) lc[j] = ln[j];
        xc = xn;
      }
    }
    // ---- back substitution: lane l holds x[jc] for the jc = l (mod 64) in
    // [k+1, k+64]; rows staged CH at a time from U
    cplx xr = make_double2(0.0, 0.0);
    double mx = 0.0;
    // U rows of the next chunk are loaded one chunk ahead, like the forward rows
    constexpr int NPB = (CH * URW + 63) / 64;
    cplx pb[NPB];
    auto fetch_u = [&](int kb) {
      const int klo = max(0, kb - CH + 1);
      const int cnt = (kb - klo + 1) * URW;
#pragma unroll
      for (int j = 0; j < NPB; ++j) {
        const int e = l + 64 * j;
        pb[j] = (e < cnt) ? U[(long)klo * URW + e] : make_double2(0.0, 0.0);
      }
    };
    fetch_u(n - 1);
    for (int kb = n - 1; kb >= 0; kb -= CH) {
      const int klo = max(0, kb - CH + 1);
      {
        const int cnt = (kb - klo + 1) * URW;
#pragma unroll
        for (int j = 0; j < NPB; ++j) {
          const int e = l + 64 * j;
          if (e < cnt) stage[e / URW][e % URW] = pb[j];
        }
      }
      __syncthreads();
      if (kb - CH >= 0) fetch_u(kb - CH);
      for (int k = kb; k >= klo; --k) {
        const int rr = k - klo;
        const int o = ((l - (k + 1)) % 64 + 64) % 64 + 1;   // jc = k + o
        cplx p = make_double2(0.0, 0.0);
        if (k + o < n) p = cmul(stage[rr][o], xr);
        p.x = wave_sum(p.x);
        p.y = wave_sum(p.y);
        const cplx xk = cmul(csub(stage[rr][WC], p), cinv(stage[rr][0]));
        if (l == (k & 63)) xr = xk;
        if (l == 0) {
          X[(long)k * ldx + kq] = xk;
          mx = fmax(mx, fmax(fabs(xk.x), fabs(xk.y)));
        }
      }
      __syncthreads();
    }
    // normalise (the scale first, against overflow)
    mx = wave_bcast0(mx);
    if (!(mx > 0.0) || !isfinite(mx)) mx = 1.0;
    double s2 = 0.0;
    for (int i = l; i < n; i += 64) {
      const cplx a = X[(long)i * ldx + kq];
      s2 += cabs2(make_double2(a.x / mx, a.y / mx));
    }
    s2 = wave_sum(s2);
    double nrm = sqrt(s2);
    if (!(nrm > 0.0)) nrm = 1.0;
    const double scv = 1.0 / (mx * nrm);
    for (int i = l; i < n; i += 64) {
      const cplx a = X[(long)i * ldx + kq];
      X[(long)i * ldx + kq] = make_double2(a.x * scv, a.y * scv);
    }
    __syncthreads();
  }
}

// vectors per inverse-iteration launch (bounds the U workspace); every
// vector's iteration depends only on its own index, so the batching does not
// change the results
static int band_invit_batch(int q, int batch) { return std::max(1, std::min(q, batch)); }

long band_invit_work_elems(long n, int q, int batch) {
  return (long)band_invit_batch(q, batch) * n * (URW + LRW);
}

void band_invit(int n, const cplx* Br, int q, int lam_off, LinalgWork& w, cplx* X, long ldx,
                uint64_t seed, hipStream_t s) {
  const int bs = band_invit_batch(q, w.invit_batch);
  require_strided(Br, ABW, 1, 0, 0, n, ABW, "band inverse iteration: band rows");
  require_strided(w.Ubuf, (long)n * (URW + LRW), 1, 0, 0, bs, (long)n * (URW + LRW),
                  "band inverse iteration: LU rows");
  require_strided(X, ldx, 1, 0, 0, n, q, "band inverse iteration: vectors");
  for (int v0 = 0; v0 < q; v0 += bs) {
    const int cnt = std::min(bs, q - v0);
    hipLaunchKernelGGL(k_band_invit, dim3(cnt), dim3(64), 0, s, n, Br, q, (const double*)w.lam,
                       lam_off, (const double*)(w.scal + 8), w.Ubuf, v0, X, ldx, seed, 2);
  }
}

void heev_top_2stage(int n, cplx* G, long ldg, int q, cplx* U, long ldu, cplx* Xtmp, LinalgWork& w,
                     uint64_t seed, hipStream_t s) {
  require_strided(G, 1, ldg, 0, 0, n, n, "two-stage eigensolver: Gram matrix");
  require_strided(U, ldu, 1, 0, 0, n, q, "two-stage eigensolver: eigenvectors");
  require_strided(Xtmp, q, 1, 0, 0, n, q, "two-stage eigensolver: work vectors");
  require_strided(w.Ab, ABW, 1, 0, 0, n, ABW, "two-stage eigensolver: band");
  require_strided(w.Br, ABW, 1, 0, 0, n, ABW, "two-stage eigensolver: band rows");
  he2hb_lower(n, G, ldg, w, s);
  const long tot = (long)n * ABW;
  const int bl = (int)std::min<long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_band_extract, dim3(bl), dim3(256), 0, s, n, (const cplx*)G, ldg, w.Ab);
  hipLaunchKernelGGL(k_band_rows, dim3(bl), dim3(256), 0, s, n, (const cplx*)w.Ab, w.Br);
  hb2st(n, w.Ab, w, s);
  const int extra = (q < n) ? 1 : 0;
  tridiag_eigvals(n, n - q - extra, q + extra, w, s);
  band_invit(n, w.Br, q, extra, w, Xtmp, q, seed, s);
  qr_factor(n, q, Xtmp, q, 1, w, s);
  qr_form_q(n, q, Xtmp, q, 1, w, U, ldu, s);
  he2hb_backtransform(n, G, ldg, q, U, ldu, w, s);
}

}  // namespace mpsim
