// C-ABI of the block-MPS Trotter evolution (see include/mpsim.h).
//
// One handle = one MPS instance resident in HBM. Bond dimensions, block
// order and the orthogonality centre are tracked on the host (they follow
// from the schedule and chi alone), so a Trotter step is a pure sequence of
// asynchronous launches on the handle's stream; device-side failures are
// raised through a flag checked at the synchronising calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mpsim.h"
#include "common.h"
#include "gemm.h"
#include "linalg.h"
#include "mps_kernels.h"
#include "planner.h"
#include "prof.h"

using namespace mpsim;

static thread_local std::string g_tl_error;

namespace mpsim {
// Message returned by mps_last_error(NULL) on this thread (calls without a handle).
void set_thread_error(const std::string& msg) { g_tl_error = msg; }
}  // namespace mpsim

struct mps_sim {
  mps_config cfg{};
  Plan plan;
  hipStream_t stream = nullptr;
  int device = 0;
  mps_allocator alloc{};
  bool has_alloc = false;
  std::vector<void*> allocations;

  std::vector<cplx*> site;
  std::vector<int> bond, pos;
  int centre = 0;
  int steps = 0;
  uint64_t nupdates = 0;
  uint64_t step_upd = 0;   // truncations since the start of the current step (seeds the eigensolver)

  long tmp_elems = 0, theta_elems = 0, gram_elems = 0, env_elems = 0, envx_elems = 0;
  cplx* theta = nullptr;
  cplx* gram = nullptr;
  cplx* tmpA = nullptr;
  cplx* tmpB = nullptr;
  cplx* tmpC = nullptr;
  cplx* env[2] = {nullptr, nullptr};
  cplx* envx = nullptr;
  double* dscal = nullptr;   // [0] logF [1] min gap [2] |M|^2 [3] |C|^2 [4] 1/|C|
  double* dpartial = nullptr;
  double* flog = nullptr;
  int* dlogn = nullptr;     // [0] next log position (device copy of nlog), [1] suspect truncations
  long log_cap = 0, nlog = 0;
  LinalgWork lw;
  Prof prof;

  cplx* d_pairs = nullptr;
  std::vector<long> pair_off;
  cplx* d_gates = nullptr;
  std::vector<long> gate_off[4];
  cplx* d_xy = nullptr;  // XY model: gates 1..4, 16 complex each
  cplx* d_wt = nullptr;  // factored Gram: weights (<= 136 x 16) and the oriented phase table
  double* d_zsum = nullptr;
  std::vector<long> zsum_off;

  int gprec = GEMM_F64;     // arithmetic of the contractions (theta, C, measurement)

  mps_progress_fn progress = nullptr;
  void* progress_ctx = nullptr;

  std::string err;
  int failed = 0;
};

// ---------------------------------------------------------------------------
namespace {

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) throw HipError{_e, #expr};  \
  } while (0)

struct NoMem {};

void* dev_alloc(mps_sim* h, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (h->has_alloc) {
    p = h->alloc.alloc(h->alloc.ctx, bytes, (void*)h->stream);
    if (!p) throw NoMem{};
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw NoMem{};
    }
  }
  h->allocations.push_back(p);
  bounds_register(p, bytes);
  return p;
}

template <typename T>
T* dalloc(mps_sim* h, long count) {
  return (T*)dev_alloc(h, sizeof(T) * (size_t)std::max<long>(count, 1));
}

struct Sizes {
  long site_max = 0, sites_total = 0, theta = 0, gram = 0, nmax = 1, qmax = 1, mmax = 1,
       colmax = 1, tmp = 0, env = 0, envx = 0;
  int eig_path = 0, eig_batch = 1024;
};

Sizes plan_sizes(const Plan& p) {
  Sizes z;
  z.eig_path = p.eig_path;
  z.eig_batch = p.eig_batch;
  const long D = p.dmax;
  for (int s = 0; s < p.N; ++s) {
    long e = (long)p.xcap[s] * D * p.xcap[s + 1];
    z.site_max = std::max(z.site_max, e);
    z.sites_total += e;
    z.mmax = std::max(z.mmax, std::max((long)p.xcap[s] * D, D * p.xcap[s + 1]));
    z.colmax = std::max(z.colmax, (long)std::max(p.xcap[s], p.xcap[s + 1]));
  }
  if (p.schedule == 4) {
    // bond truncations: the site (cap D) x (2 cap) and its Gram on the smaller
    // side; C = (kept) x (2 cap)
    for (int b = 1; b < p.N; ++b) {
      long kg = std::min((long)p.cap[b - 1] * D, (long)p.xcap[b]);
      z.theta = std::max(z.theta, (long)p.cap[b] * p.xcap[b]);
      z.gram = std::max(z.gram, kg * kg);
      z.nmax = std::max(z.nmax, kg);
      z.qmax = std::max(z.qmax, std::min<long>(p.chi, kg));
    }
  } else {
    for (int i = 0; i + 1 < p.N; ++i) {
      long mo = (long)p.cap[i] * D, no = D * p.cap[i + 2];
      z.theta = std::max(z.theta, mo * no);
      long kg = std::min(mo, no);
      z.gram = std::max(z.gram, kg * kg);
      z.nmax = std::max(z.nmax, kg);
      z.qmax = std::max(z.qmax, std::min<long>(p.chi, kg));
    }
  }
  // bond spectrum Gram (cap x cap)
  for (int b = 1; b < p.N; ++b) {
    z.nmax = std::max(z.nmax, (long)p.cap[b]);
    z.gram = std::max(z.gram, (long)p.cap[b] * p.cap[b]);
  }
  z.mmax = std::max(z.mmax, z.nmax);
  z.colmax = std::max(z.colmax, z.qmax);
  // the two-stage panels factor TRD_NB columns at a time
  z.colmax = std::max<long>(z.colmax, TRD_NB);
  z.tmp = std::max(z.site_max, z.nmax * z.qmax);
  long cmax = 1;
  for (int s = 0; s <= p.N; ++s) cmax = std::max(cmax, (long)p.cap[s]);
  z.env = 3 * cmax * cmax;
  z.envx = 3 * z.site_max;
  return z;
}

struct LwSizes {
  long W, tpart, P, dpart, npart, iwork, T, V, W12, gpart;
  long T1, X2, band, ubuf, acc;  // two-stage path (zero when it is never taken)
};

// whether a Gram side of n takes the two-stage eigensolver
static bool use_two_stage(int eig_path, long n) {
  return eig_path == 2 || (eig_path == 0 && n >= MPS_EIG2_MIN);
}

LwSizes lw_sizes(const Sizes& z) {
  LwSizes l;
  l.W = z.nmax * TRD_NB;
  long nparts = (long)ceil_div(z.mmax, 256) * 4;
  // QR column steps: two halves of (pivot row copy, nparts x QR_NB partials)
  l.tpart = std::max(nparts * (2 * TRD_NB + 1), 2 * (QR_NB + nparts * QR_NB));
  long nt = ceil_div(z.nmax, 64);
  l.P = nt * nt * 64;
  l.dpart = std::max(nparts, nt + 1);
  l.npart = nparts;
  l.iwork = 6 * z.nmax * z.qmax;
  l.T = ((long)z.colmax / QR_NB + 2) * 4096;
  l.V = std::max(z.nmax, z.mmax) * 64;
  l.W12 = 64 * z.colmax;
  l.gpart = 4L << 20;
  l.T1 = l.X2 = l.band = l.ubuf = l.acc = 0;
  if (use_two_stage(z.eig_path, z.nmax)) {
    l.T1 = (z.nmax / TRD_NB + 2) * 4096;
    l.X2 = z.nmax * 64;
    l.band = z.nmax * BAND_W;
    l.ubuf = band_invit_work_elems(z.nmax, (int)z.qmax, z.eig_batch);
    l.acc = he2hb_acc_elems(z.nmax);
  }
  return l;
}

// The eigensolver, QR and reflector workspaces of one handle.
void alloc_linalg(mps_sim* h, const Sizes& z, const LwSizes& l) {
  LinalgWork& w = h->lw;
  w.nmax = z.nmax; w.qmax = z.qmax; w.mmax = z.mmax;
  w.W = dalloc<cplx>(h, l.W);
  w.tpart = dalloc<cplx>(h, l.tpart);
  w.tpart_elems = l.tpart;
  w.P = dalloc<cplx>(h, l.P);
  w.P_elems = l.P;
  w.dpart = dalloc<cplx>(h, l.dpart);
  w.tsum = dalloc<cplx>(h, 2 * TRD_NB + 2);
  w.npart = dalloc<double>(h, l.npart);
  w.d = dalloc<double>(h, z.nmax);
  w.e = dalloc<double>(h, z.nmax);
  w.e2 = dalloc<double>(h, z.nmax);
  w.tau = dalloc<cplx>(h, z.nmax);
  w.qtau = dalloc<cplx>(h, z.colmax);
  w.scal = dalloc<double>(h, 16);
  w.lam = dalloc<double>(h, z.qmax + 2);
  w.iwork = dalloc<double>(h, l.iwork);
  w.T = dalloc<cplx>(h, l.T);
  w.T_elems = l.T;
  w.S = dalloc<cplx>(h, 4096);
  w.wmax = z.colmax;
  w.W1 = dalloc<cplx>(h, l.W12);
  w.W2 = dalloc<cplx>(h, l.W12);
  w.vmax = std::max(z.nmax, z.mmax);
  w.V = dalloc<cplx>(h, l.V);
  w.gpart = dalloc<cplx>(h, l.gpart);
  w.gpart_elems = l.gpart;
  w.flag = dalloc<int>(h, 4);
  w.prof = &h->prof;
  if (l.T1) {
    w.T1 = dalloc<cplx>(h, l.T1);
    w.X2 = dalloc<cplx>(h, l.X2);
    w.S2 = dalloc<cplx>(h, 4096);
    w.Ab = dalloc<cplx>(h, l.band);
    w.Br = dalloc<cplx>(h, l.band);
    w.Ubuf = dalloc<cplx>(h, l.ubuf);
    w.invit_batch = z.eig_batch;
    w.acc = dalloc<cplx>(h, l.acc);
  }
}

size_t footprint(const Plan& p) {
  Sizes z = plan_sizes(p);
  LwSizes l = lw_sizes(z);
  size_t c = sizeof(cplx), d = sizeof(double);
  size_t total = 0;
  total += (size_t)z.sites_total * c;
  total += (size_t)(z.theta + z.gram + 3 * z.tmp + 2 * z.env + z.envx) * c;
  total += (size_t)(l.W + l.tpart + l.P + l.dpart + l.T + 4096 + 2 * l.W12 + l.V + l.gpart) * c;
  total += (size_t)(l.T1 + l.X2 + 4096 + 2 * l.band + l.ubuf + l.acc) * c;
  total += (size_t)(l.npart + l.iwork + 4 * z.nmax + z.qmax + 2 + 16 + 2 * 4096) * d;
  total += (size_t)(z.nmax + z.colmax) * c;
  return total;
}

// Stream-ordered copy followed by a wait on the handle's stream only.
hipError_t copy_sync(mps_sim* h, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e;
}

mps_status fail(mps_sim* h, mps_status st, const std::string& msg) {
  if (h) {
    h->err = msg;
    if (st == MPS_E_DEVICE || st == MPS_E_NUMERIC) h->failed = 1;
  } else {
    g_tl_error = msg;
  }
  return st;
}

// ---------------------------------------------------------------------------
// building blocks

// Bound on | |C|^2 - sum of the kept eigenvalues | / |M|^2 above which a
// truncation counts as suspect: float64 contractions agree to ~1e-13, the
// reduced-precision ones to their own rounding (~1e-7).
double eig_check_tol(const mps_sim* h) { return h->gprec == GEMM_F64 ? 1e-9 : 1e-5; }

void norm2(mps_sim* h, const cplx* x, long len, int slot) {
  launch_norm2(x, len, h->dpartial, h->dscal + slot, h->stream);
}

void dev_free(mps_sim* h, void* p) {
  auto it = std::find(h->allocations.begin(), h->allocations.end(), p);
  if (it == h->allocations.end()) return;
  h->allocations.erase(it);
  bounds_unregister(p);
  if (h->has_alloc) {
    h->alloc.free(h->alloc.ctx, p, (void*)h->stream);   // stream-ordered
  } else {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(p);
  }
}

// Capacity of the truncation log (growing it moves the log and frees the old
// buffer).
void ensure_log(mps_sim* h, long need) {
  if (need <= h->log_cap) return;
  long ncap = std::max(need, 2 * h->log_cap);
  double* nl = dalloc<double>(h, 2 * ncap);
  if (h->nlog > 0)
    HIPCHK(hipMemcpyAsync(nl, h->flog, sizeof(double) * 2 * h->nlog, hipMemcpyDeviceToDevice, h->stream));
  if (h->flog) dev_free(h, h->flog);
  h->flog = nl;
  h->log_cap = ncap;
}

// Move the orthogonality centre one site right: QR of site c.
void move_right(mps_sim* h) {
  const int c = h->centre;
  const Plan& p = h->plan;
  const int b0 = h->bond[c], d = p.dim(h->pos[c]), b1 = h->bond[c + 1];
  const int m = b0 * d, k = b1, kmin = std::min(m, k);
  const int d2 = p.dim(h->pos[c + 1]), b2 = h->bond[c + 2];
  hipStream_t s = h->stream;
  HIPCHK(hipMemcpyAsync(h->tmpA, h->site[c], sizeof(cplx) * (size_t)m * k, hipMemcpyDeviceToDevice, s));
  qr_factor(m, k, h->tmpA, k, 1, h->lw, s);
  qr_form_q(m, k, h->tmpA, k, 1, h->lw, h->site[c], kmin, s);
  qr_get_r(m, k, h->tmpA, k, 1, h->tmpB, k, s);
  // site c+1 <- R * site c+1  (kmin x k) (k x d2*b2)
  ZGemm g = zgemm_args(kmin, d2 * b2, k, zop(h->tmpB, k, 0), zop(h->site[c + 1], (long)d2 * b2, 0),
                       h->tmpC, (long)d2 * b2, 0, make_double2(1, 0), make_double2(0, 0));
  zgemm(g, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
  HIPCHK(hipMemcpyAsync(h->site[c + 1], h->tmpC, sizeof(cplx) * (size_t)kmin * d2 * b2,
                        hipMemcpyDeviceToDevice, s));
  h->bond[c + 1] = kmin;
  h->centre = c + 1;
}

// Move the centre one site left: LQ of site c (QR of its conjugate transpose).
void move_left(mps_sim* h) {
  const int c = h->centre;
  const Plan& p = h->plan;
  const int b0 = h->bond[c], d = p.dim(h->pos[c]), b1 = h->bond[c + 1];
  const int rows = b0, cols = d * b1;  // site as b0 x (d*b1)
  const int m = cols, k = rows, kmin = std::min(m, k);
  const int bp = h->bond[c - 1], dp = p.dim(h->pos[c - 1]);
  hipStream_t s = h->stream;
  // Y = site^H (m x k row-major)
  launch_conj_transpose(h->site[c], rows, cols, cols, h->tmpA, k, s);
  qr_factor(m, k, h->tmpA, k, 1, h->lw, s);
  qr_form_q(m, k, h->tmpA, k, 1, h->lw, h->tmpB, kmin, s);  // Q: m x kmin
  // new site c = Q^H (kmin x m)
  launch_conj_transpose(h->tmpB, m, kmin, kmin, h->site[c], m, s);
  qr_get_r(m, k, h->tmpA, k, 1, h->tmpB, k, s);  // R: kmin x k
  // site c-1 <- site c-1 * R^H : (bp*dp x k) (k x kmin)
  ZGemm g = zgemm_args(bp * dp, kmin, k, zop(h->site[c - 1], k, 0), zop(h->tmpB, k, 1, 1), h->tmpC,
                       kmin, 0, make_double2(1, 0), make_double2(0, 0));
  zgemm(g, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
  HIPCHK(hipMemcpyAsync(h->site[c - 1], h->tmpC, sizeof(cplx) * (size_t)bp * dp * kmin,
                        hipMemcpyDeviceToDevice, s));
  h->bond[c] = kmin;
  h->centre = c - 1;
}

void move_centre(mps_sim* h, int target) {
  while (h->centre < target) move_right(h);
  while (h->centre > target) move_left(h);
}

// Two-site update on (i, i+1): theta = A_i A_{i+1} with the block-pair phase
// (and SWAP) fused into the GEMM epilogue, then truncation to
// q = min(chi, rows, cols) through the top-q eigenspace of the Gram matrix on
// the smaller side, fidelity bookkeeping and renormalisation.
// Top-q eigenspace of the Gram matrix (kg x kg in h->gram) into U (kg x q).
void heev(mps_sim* h, int kg, int q, cplx* U, uint64_t seed) {
  if (use_two_stage(h->plan.eig_path, kg))
    heev_top_2stage(kg, h->gram, kg, q, U, q, h->tmpA, h->lw, seed, h->stream);
  else
    heev_top(kg, h->gram, kg, q, U, q, h->tmpA, h->lw, seed, h->stream);
}

// Two-site update without SWAP through the factored Gram matrix. With
// theta[(a s1), (s2 c)] = D[s1][s2] (A_s1 B_s2)[a, c] (A_s1: rows a d + s1 of
// site i, B_s2: columns s2 b2 + c of site i+1), the Gram matrix on the rows,
// taken in the order (s1, a), has the blocks
//   G_{s1 s1'} = A_s1 (sum_s2 D[s1][s2] conj(D[s1'][s2]) B_s2 B_s2^H) A_s1'^H,
// and the one on the columns
//   G_{s2 s2'} = B_s2^H (sum_s1 conj(D[s1][s2]) D[s1][s2'] A_s1^H A_s1) B_s2';
// the truncation products factor the same way (C = U^H theta from
// U_s1^H A_s1, C = theta V from B_s2 V_s2), so theta is never formed and the
// Gram costs two chi^3 products per block pair instead of d chi^3.
// The Gram products run in float64 whatever the precision mode; the
// products that form C take the mode's contraction precision.
// Returns false (nothing done) when the shape does not qualify.
constexpr long FACTORED_MIN = 2048;  // Gram side from which the factored form pays
bool two_site_factored(mps_sim* h, int i, int gate, bool left, int q, uint64_t seed) {
  const Plan& p = h->plan;
  const int ba = h->pos[i], bb = h->pos[i + 1];
  const int d = p.dim(ba);
  if (p.dim(bb) != d || d < 4 || p.model != 0) return false;
  const long b0 = h->bond[i], b1 = h->bond[i + 1], b2 = h->bond[i + 2];
  const long kg = left ? b0 * d : (long)d * b2;
  if (kg < FACTORED_MIN) return false;
  const long np = (long)d * (d + 1) / 2;
  if ((long)(d + np) * b1 * b1 > h->theta_elems) return false;
  hipStream_t s = h->stream;
  const cplx one = make_double2(1, 0), zero = make_double2(0, 0);
  cplx* A = h->site[i];
  cplx* B = h->site[i + 1];
  const long lda = (long)d * b1, ldb = (long)d * b2;
  const cplx* table = nullptr;
  int trans = 0;
  if (gate) {
    const int pi = p.coupled(ba, bb);
    if (pi >= 0) {
      table = h->d_pairs + h->pair_off[pi];
      trans = (ba > bb) ? 1 : 0;
    }
  }
  cplx* W = h->d_wt;
  cplx* Dfull = h->d_wt + 136 * 16;
  launch_pair_weights(table, trans, d, left ? 0 : 1, W, Dfull, s);
  cplx* Mb = h->theta;                      // d products, b1 x b1 each
  cplx* Kb = h->theta + (long)d * b1 * b1;  // np weighted sums, b1 x b1 each
  const int extra = (q < kg) ? 1 : 0;
  if (left) {
    // M_s2 = B_s2 B_s2^H
    ZGemm gm = zgemm_args((int)b1, (int)b1, (int)b2, zop(B, ldb, 0), zop(B, ldb, 1, 1), Mb, b1, 0, one, zero);
    gm.batch = d; gm.A.stride = b2; gm.B.stride = b2; gm.strideC = b1 * b1;
    zgemm(gm, nullptr, 0, s, &h->prof);
  } else {
    // N_s1 = A_s1^H A_s1
    ZGemm gm = zgemm_args((int)b1, (int)b1, (int)b0, zop(A, lda, 1, 1), zop(A, lda, 0), Mb, b1, 0, one, zero);
    gm.batch = d; gm.A.stride = b1; gm.B.stride = b1; gm.strideC = b1 * b1;
    zgemm(gm, nullptr, 0, s, &h->prof);
  }
  // weighted sums of all block pairs at once: (np x d) (d x b1^2)
  ZGemm gk = zgemm_args((int)np, (int)(b1 * b1), d, zop(W, d, 0), zop(Mb, b1 * b1, 0), Kb, b1 * b1, 0, one,
                        zero);
  zgemm(gk, nullptr, 0, s, &h->prof);
  // Gram blocks (lower block triangle, diagonal blocks in full), column-major
  for (int x = 0; x < d; ++x) {
    cplx* Kx = Kb + (long)x * (x + 1) / 2 * b1 * b1;
    if (left) {
      // T_y = A_x K_xy (b0 x b1), G_xy = T_y A_y^H
      ZGemm gt = zgemm_args((int)b0, (int)b1, (int)b1, zop(A + (long)x * b1, lda, 0), zop(Kx, b1, 0), h->tmpA,
                            b1, 0, one, zero);
      gt.batch = x + 1; gt.A.stride = 0; gt.B.stride = b1 * b1; gt.strideC = b0 * b1;
      zgemm(gt, nullptr, 0, s, &h->prof);
      ZGemm gg = zgemm_args((int)b0, (int)b0, (int)b1, zop(h->tmpA, b1, 0), zop(A, lda, 1, 1),
                            h->gram + (long)x * b0, kg, 1, one, zero);
      gg.batch = x + 1; gg.A.stride = b0 * b1; gg.B.stride = b1; gg.strideC = b0 * kg;
      gg.tag = PROF_GRAM;
      zgemm(gg, nullptr, 0, s, &h->prof);
    } else {
      // T_y = B_x^H L_xy (b2 x b1), G_xy = T_y B_y
      ZGemm gt = zgemm_args((int)b2, (int)b1, (int)b1, zop(B + (long)x * b2, ldb, 1, 1), zop(Kx, b1, 0),
                            h->tmpA, b1, 0, one, zero);
      gt.batch = x + 1; gt.A.stride = 0; gt.B.stride = b1 * b1; gt.strideC = b2 * b1;
      zgemm(gt, nullptr, 0, s, &h->prof);
      ZGemm gg = zgemm_args((int)b2, (int)b2, (int)b1, zop(h->tmpA, b1, 0), zop(B, ldb, 0),
                            h->gram + (long)x * b2, kg, 1, one, zero);
      gg.batch = x + 1; gg.A.stride = b2 * b1; gg.B.stride = b2; gg.strideC = b2 * kg;
      gg.tag = PROF_GRAM;
      zgemm(gg, nullptr, 0, s, &h->prof);
    }
  }
  launch_trace_real(h->gram, kg, kg, h->dscal + 2, s);
  heev(h, (int)kg, q, h->tmpB, seed);
  ensure_log(h, h->nlog + 1);
  if (left) {
    // P_s1 = U_s1^H A_s1 (q x b1), U in (s1, a) row order
    ZGemm gp = zgemm_args(q, (int)b1, (int)b0, zop(h->tmpB, q, 1, 1), zop(A, lda, 0), h->tmpC, b1, 0, one,
                          zero);
    gp.batch = d; gp.A.stride = b0 * q; gp.B.stride = b1; gp.strideC = (long)q * b1;
    gp.prec = h->gprec;
    zgemm(gp, nullptr, 0, s, &h->prof);
    // Q_s2 = sum_s1 D[s1][s2] P_s1: (d x d)^T (d x q b1)
    ZGemm gq = zgemm_args(d, (int)(q * b1), d, zop(Dfull, d, 1), zop(h->tmpC, q * b1, 0), h->tmpA, q * b1, 0,
                          one, zero);
    zgemm(gq, nullptr, 0, s, &h->prof);
    // C_s2 = Q_s2 B_s2 -> columns s2 b2 .. of C (q x d b2)
    ZGemm gc = zgemm_args(q, (int)b2, (int)b1, zop(h->tmpA, b1, 0), zop(B, ldb, 0), h->theta, ldb, 0, one,
                          zero);
    gc.batch = d; gc.A.stride = (long)q * b1; gc.B.stride = b2; gc.strideC = b2;
    gc.prec = h->gprec;
    zgemm(gc, nullptr, 0, s, &h->prof);
    launch_unpermute_rows(h->tmpB, A, (int)b0, d, q, s);
    norm2(h, h->theta, (long)q * ldb, 3);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    launch_scale_by(h->theta, (long)q * ldb, h->dscal, s);
    HIPCHK(hipMemcpyAsync(B, h->theta, sizeof(cplx) * (size_t)q * ldb, hipMemcpyDeviceToDevice, s));
    h->centre = i + 1;
  } else {
    // R_s2 = B_s2 V_s2 (b1 x q), V in natural (s2, c) row order
    ZGemm gr = zgemm_args((int)b1, q, (int)b2, zop(B, ldb, 0), zop(h->tmpB, q, 0), h->tmpC, q, 0, one, zero);
    gr.batch = d; gr.A.stride = b2; gr.B.stride = b2 * q; gr.strideC = b1 * q;
    gr.prec = h->gprec;
    zgemm(gr, nullptr, 0, s, &h->prof);
    // Q_s1 = sum_s2 D[s1][s2] R_s2: (d x d) (d x b1 q)
    ZGemm gq = zgemm_args(d, (int)(b1 * q), d, zop(Dfull, d, 0), zop(h->tmpC, b1 * q, 0), h->tmpA, b1 * q, 0,
                          one, zero);
    zgemm(gq, nullptr, 0, s, &h->prof);
    // C_s1 = A_s1 Q_s1 -> rows a d + s1 of C (b0 d x q)
    ZGemm gc = zgemm_args((int)b0, q, (int)b1, zop(A, lda, 0), zop(h->tmpA, q, 0), h->theta, (long)d * q, 0,
                          one, zero);
    gc.batch = d; gc.A.stride = b1; gc.B.stride = b1 * q; gc.strideC = q;
    gc.prec = h->gprec;
    zgemm(gc, nullptr, 0, s, &h->prof);
    // site i+1 = V^H (q x d b2)
    launch_conj_transpose(h->tmpB, (int)kg, q, q, B, kg, s);
    norm2(h, h->theta, b0 * d * q, 3);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    launch_scale_by(h->theta, b0 * d * q, h->dscal, s);
    HIPCHK(hipMemcpyAsync(A, h->theta, sizeof(cplx) * (size_t)(b0 * d * q), hipMemcpyDeviceToDevice, s));
    h->centre = i;
  }
  h->nlog += 1;
  h->nupdates += 1;
  h->step_upd += 1;
  h->bond[i + 1] = q;
  return true;
}

void two_site(mps_sim* h, int i, int swap, int gate, int next_site) {
  const Plan& p = h->plan;
  if (h->centre < i) move_centre(h, i);
  else if (h->centre > i + 1) move_centre(h, i + 1);
  hipStream_t s = h->stream;
  const int ba = h->pos[i], bb = h->pos[i + 1];
  const int b0 = h->bond[i], d1 = p.dim(ba), b1 = h->bond[i + 1], d2 = p.dim(bb), b2 = h->bond[i + 2];
  const long m = (long)b0 * d1, n = (long)d2 * b2;
  const long mo = swap ? (long)b0 * d2 : m, no = swap ? (long)d1 * b2 : n;
  const int q = (int)std::min<long>(p.chi, std::min(mo, no));
  bool left;
  if (mo != no) left = mo < no;
  else left = !(next_site >= 0 && next_site < i);
  const uint64_t seed = h->cfg.seed * 0x9E3779B97F4A7C15ULL + h->step_upd;
  if (!swap && two_site_factored(h, i, gate, left, q, seed)) return;

  // theta
  ZGemm g = zgemm_args((int)m, (int)n, b1, zop(h->site[i], b1, 0), zop(h->site[i + 1], n, 0), h->theta,
                       n, 0, make_double2(1, 0), make_double2(0, 0));
  g.epi = EPI_THETA;
  g.d1 = d1; g.d2 = d2; g.b2 = b2; g.swap = swap;
  g.phase = nullptr;
  g.tag = PROF_THETA;
  g.prec = h->gprec;
  const bool dense_gate = p.model == 1 && gate;
  if (dense_gate) g.swap = 0;  // the dense gate kernel applies the SWAP
  if (gate && p.model == 0) {
    int pi = p.coupled(ba, bb);
    if (pi >= 0) {
      g.phase = h->d_pairs + h->pair_off[pi];
      g.phase_trans = (ba > bb) ? 1 : 0;
    }
  }
  zgemm(g, nullptr, 0, s, &h->prof);
  if (dense_gate) launch_theta_gate4(h->theta, b0, b2, h->d_xy + 16 * gate, swap, s);
  norm2(h, h->theta, mo * no, 2);

  const int extra = (q < (left ? mo : no)) ? 1 : 0;
  const cplx one = make_double2(1, 0), zero = make_double2(0, 0);
  if (left) {
    const int kg = (int)mo;
    // G = M M^H stored column-major (lower triangle)
    ZGemm gg = zgemm_args(kg, kg, (int)no, zop(h->theta, no, 0), zop(h->theta, no, 1, 1), h->gram, kg, 1,
                          one, zero);
    gg.lower_only = 1;
    gg.tag = PROF_GRAM;
    zgemm(gg, nullptr, 0, s, &h->prof);
    heev(h, kg, q, h->site[i], seed);
    // C = U^H M -> site i+1 (q x no)
    ZGemm gc = zgemm_args(q, (int)no, kg, zop(h->site[i], q, 1, 1), zop(h->theta, no, 0), h->site[i + 1],
                          no, 0, one, zero);
    gc.prec = h->gprec;
    zgemm(gc, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
    norm2(h, h->site[i + 1], (long)q * no, 3);
    ensure_log(h, h->nlog + 1);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    launch_scale_by(h->site[i + 1], (long)q * no, h->dscal, s);
    h->centre = i + 1;
  } else {
    const int kg = (int)no;
    // G = M^H M stored column-major (lower triangle)
    ZGemm gg = zgemm_args(kg, kg, (int)mo, zop(h->theta, no, 1, 1), zop(h->theta, no, 0), h->gram, kg, 1,
                          one, zero);
    gg.lower_only = 1;
    gg.tag = PROF_GRAM;
    zgemm(gg, nullptr, 0, s, &h->prof);
    heev(h, kg, q, h->tmpB, seed);
    launch_conj_transpose(h->tmpB, kg, q, q, h->site[i + 1], kg, s);
    // C = M V -> site i (mo x q)
    ZGemm gc = zgemm_args((int)mo, q, kg, zop(h->theta, no, 0), zop(h->tmpB, q, 0), h->site[i], q, 0, one,
                          zero);
    gc.prec = h->gprec;
    zgemm(gc, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
    norm2(h, h->site[i], mo * q, 3);
    ensure_log(h, h->nlog + 1);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    launch_scale_by(h->site[i], mo * q, h->dscal, s);
    h->centre = i;
  }
  h->nlog += 1;
  h->nupdates += 1;
  h->step_upd += 1;
  h->bond[i + 1] = q;
  if (swap) std::swap(h->pos[i], h->pos[i + 1]);
}

// Truncate the bond between sites i and i+1 with the orthogonality centre on
// site i and every site right of it right-orthonormal: the site M
// ((b d) x b') keeps the top q = min(chi, rank bound, b d, b') singular
// directions of the bond (results section: the centre is moved onto the bond
// before the decomposition, so its cost depends on the bond only). The Gram
// matrix is taken on the smaller side; on the column side the kept part
// M V = Q R' is re-orthonormalised by QR, site i <- Q, and R' V^H moves into
// site i+1, which becomes the centre.
void truncate_bond(mps_sim* h, int i) {
  const Plan& p = h->plan;
  hipStream_t s = h->stream;
  const int b0 = h->bond[i], d = p.dim(h->pos[i]), k = h->bond[i + 1];
  const int d2 = p.dim(h->pos[i + 1]), b2 = h->bond[i + 2];
  const long m = (long)b0 * d, n2 = (long)d2 * b2;
  const int q = (int)std::min<long>(std::min<long>(p.chi, p.rank_cap[i + 1]), std::min<long>(m, k));
  const cplx one = make_double2(1, 0), zero = make_double2(0, 0);
  const uint64_t seed = h->cfg.seed * 0x9E3779B97F4A7C15ULL + h->step_upd;
  cplx* M = h->site[i];
  norm2(h, M, m * k, 2);
  ensure_log(h, h->nlog + 1);
  if (m < k) {
    const int kg = (int)m;
    const int extra = (q < kg) ? 1 : 0;
    ZGemm gg = zgemm_args(kg, kg, k, zop(M, k, 0), zop(M, k, 1, 1), h->gram, kg, 1, one, zero);
    gg.lower_only = 1;
    gg.tag = PROF_GRAM;
    zgemm(gg, nullptr, 0, s, &h->prof);
    heev(h, kg, q, h->tmpB, seed);
    // C = U^H M (q x k)
    ZGemm gc = zgemm_args(q, k, kg, zop(h->tmpB, q, 1, 1), zop(M, k, 0), h->theta, k, 0, one, zero);
    zgemm(gc, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
    norm2(h, h->theta, (long)q * k, 3);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    HIPCHK(hipMemcpyAsync(M, h->tmpB, sizeof(cplx) * (size_t)m * q, hipMemcpyDeviceToDevice, s));
  } else {
    const int kg = k;
    const int extra = (q < kg) ? 1 : 0;
    ZGemm gg = zgemm_args(kg, kg, (int)m, zop(M, k, 1, 1), zop(M, k, 0), h->gram, kg, 1, one, zero);
    gg.lower_only = 1;
    gg.tag = PROF_GRAM;
    zgemm(gg, nullptr, 0, s, &h->prof);
    heev(h, kg, q, h->tmpB, seed);
    // X = M V (m x q), kept weight |X|^2
    ZGemm gx = zgemm_args((int)m, q, kg, zop(M, k, 0), zop(h->tmpB, q, 0), h->tmpA, q, 0, one, zero);
    zgemm(gx, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
    norm2(h, h->tmpA, m * q, 3);
    launch_trunc_finalize(h->dscal, h->flog, h->dlogn, h->lw.lam, q, extra, h->lw.flag, eig_check_tol(h), s);
    // X = Q R': site i <- Q, C = R' V^H (q x k)
    qr_factor((int)m, q, h->tmpA, q, 1, h->lw, s);
    qr_form_q((int)m, q, h->tmpA, q, 1, h->lw, M, q, s);
    qr_get_r((int)m, q, h->tmpA, q, 1, h->tmpC, q, s);
    ZGemm gc = zgemm_args(q, k, q, zop(h->tmpC, q, 0), zop(h->tmpB, q, 1, 1), h->theta, k, 0, one, zero);
    zgemm(gc, nullptr, 0, s, &h->prof);
  }
  launch_scale_by(h->theta, (long)q * k, h->dscal, s);
  // site i+1 <- C * site i+1 (q x d2 b2)
  ZGemm gn = zgemm_args(q, (int)n2, k, zop(h->theta, k, 0), zop(h->site[i + 1], n2, 0), h->tmpA, n2, 0,
                        one, zero);
  gn.prec = h->gprec;
  zgemm(gn, h->lw.gpart, h->lw.gpart_elems, s, &h->prof);
  HIPCHK(hipMemcpyAsync(h->site[i + 1], h->tmpA, sizeof(cplx) * (size_t)q * n2, hipMemcpyDeviceToDevice, s));
  h->nlog += 1;
  h->nupdates += 1;
  h->step_upd += 1;
  h->bond[i + 1] = q;
  h->centre = i + 1;
}

// One ZZ gate exp(-i J dt Z Z') between bit ja of the block at site sa and
// bit jb of the block at site sb > sa, applied as a rank-2 matrix product
// operator (results section: a gate between two blocks doubles every bond
// between them), then canonical form again (LQ steps from sb down to sa) and
// truncation of the doubled bonds from left to right.
void zz_mpo(mps_sim* h, int sa, int sb, int ja, int jb) {
  const Plan& p = h->plan;
  hipStream_t s = h->stream;
  move_centre(h, sa);
  const double phi = p.J * p.dt;
  const double c = std::cos(phi), sn = std::sin(phi);
  for (int t = sa; t <= sb; ++t) {
    const int blk = h->pos[t];
    const int b0 = h->bond[t], d = p.dim(blk), b1 = h->bond[t + 1];
    const int mode = (t == sa) ? 0 : (t == sb ? 2 : 1);
    const int bit = (t == sa) ? ja : jb;
    launch_mpo_site(h->site[t], h->tmpA, b0, d, b1, mode, p.block_width[blk], bit, c, sn, s);
    const long ob0 = mode == 0 ? b0 : 2L * b0, ob1 = mode == 2 ? b1 : 2L * b1;
    HIPCHK(hipMemcpyAsync(h->site[t], h->tmpA, sizeof(cplx) * (size_t)(ob0 * d * ob1),
                          hipMemcpyDeviceToDevice, s));
  }
  for (int b = sa + 1; b <= sb; ++b) h->bond[b] *= 2;
  h->centre = sb;
  move_centre(h, sa);
  for (int t = sa; t < sb; ++t) truncate_bond(h, t);
}

void single_site(mps_sim* h, int site, int variant) {
  const Plan& p = h->plan;
  const int b = h->pos[site];
  launch_apply_u1(h->site[site], h->bond[site], p.dim(b), h->bond[site + 1],
                  h->d_gates + h->gate_off[variant][b], h->stream);
}

void run_step(mps_sim* h) {
  std::vector<Op> ops;
  std::vector<int> pos = h->pos;
  h->plan.step_ops(pos, ops);
  h->step_upd = 0;
  int nu2 = 0, done = 0;
  for (const Op& o : ops) nu2 += (o.kind == 1 || o.kind == 3);
  for (size_t k = 0; k < ops.size(); ++k) {
    const Op& o = ops[k];
    if (o.kind == 1) {
      int next = -1;
      for (size_t k2 = k + 1; k2 < ops.size(); ++k2)
        if (ops[k2].kind == 1) { next = ops[k2].site; break; }
      two_site(h, o.site, o.swap, o.gate, next);
      ++done;
      if (h->progress) h->progress(h->progress_ctx, h->steps, done, nu2);
    } else if (o.kind == 3) {
      zz_mpo(h, o.site, o.site_b, o.bit_a, o.bit_b);
      ++done;
      if (h->progress) h->progress(h->progress_ctx, h->steps, done, nu2);
    } else {
      single_site(h, o.site, o.variant);
    }
  }
  h->steps += 1;
}

mps_status check_device(mps_sim* h) {
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, MPS_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  int flag = 0;
  e = hipMemcpyAsync(&flag, h->lw.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, MPS_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  if (flag) return fail(h, MPS_E_NUMERIC, "non-finite or zero norm in a truncation");
  return MPS_OK;
}

// Measurement sweep: three left environments for 1, Z_tot and Z_tot^2.
// XY model preparation (eq. "xy_init"): the Trotter steps of size dtau from
// the Neel state, then exp(-i pi/8 H_Z) on every site.
void xy_prepare(mps_sim* h) {
  const Plan& p = h->plan;
  for (int k = 0; k < p.nprep; ++k) {
    std::vector<Op> ops;
    p.xy_ops(h->pos, ops, true);
    for (size_t i = 0; i < ops.size(); ++i) {
      int next = -1;
      for (size_t i2 = i + 1; i2 < ops.size(); ++i2) { next = ops[i2].site; break; }
      two_site(h, ops[i].site, ops[i].swap, ops[i].gate, next);
    }
  }
  for (int st = 0; st < p.N; ++st) single_site(h, st, 3);
}

// op 0: Z_tot moments (diagonal z sums); op 1: staggered X (XY model)
void measure_sweep(mps_sim* h, double out[3], int op = 0);
void measure_sweep(mps_sim* h, double out[3], int op) {
  const Plan& p = h->plan;
  hipStream_t s = h->stream;
  launch_env_init(h->env[0], s);
  int cur = 0;
  const cplx one = make_double2(1, 0), zero = make_double2(0, 0);
  for (int st = 0; st < p.N; ++st) {
    const int b = h->bond[st], blk = h->pos[st], d = p.dim(blk), b2 = h->bond[st + 1];
    const long xs = (long)b * d * b2;
    // X_k = E_k A
    ZGemm g1 = zgemm_args(b, d * b2, b, zop(h->env[cur], b, 0), zop(h->site[st], (long)d * b2, 0), h->envx,
                          (long)d * b2, 0, one, zero);
    g1.batch = 3;
    g1.prec = h->gprec;
    g1.A.stride = (long)b * b;
    g1.B.stride = 0;
    g1.strideC = xs;
    zgemm(g1, nullptr, 0, s, &h->prof);
    if (op == 1) launch_meas_combine_x(h->envx, b, b2, (double)p.stagger[blk], s);
    else launch_meas_combine(h->envx, b, d, b2, h->d_zsum + h->zsum_off[blk], s);
    // E'_k = A^H Y_k
    ZGemm g2 = zgemm_args(b2, b2, b * d, zop(h->site[st], b2, 1, 1), zop(h->envx, b2, 0), h->env[1 - cur], b2,
                          0, one, zero);
    g2.batch = 3;
    g2.prec = h->gprec;
    g2.A.stride = 0;
    g2.B.stride = xs;
    g2.strideC = (long)b2 * b2;
    zgemm(g2, nullptr, 0, s, &h->prof);
    cur = 1 - cur;
  }
  cplx host[3];
  HIPCHK(hipMemcpyAsync(host, h->env[cur], sizeof(cplx) * 3, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) out[k] = host[k].x;
}

void upload_product_state(mps_sim* h) {
  const Plan& p = h->plan;
  const double c = std::cos(p.theta0 / 2), sn = std::sin(p.theta0 / 2);
  for (int st = 0; st < p.N; ++st) {
    const int blk = h->pos[st], w = p.block_width[blk], d = p.dim(blk);
    std::vector<cplx> v(d);
    for (int idx = 0; idx < d; ++idx) {
      double amp = 1.0;
      for (int j = 0; j < w; ++j) amp *= (((idx >> (w - 1 - j)) & 1) == 0) ? c : sn;
      v[idx] = make_double2(amp, 0.0);
    }
    if (p.model == 1) {
      // Neel state, the ground state of H_Z = sum_j (-1)^j Z_j: |1> where the
      // checkerboard sign is +1, |0> where it is -1
      v[0] = make_double2(p.stagger[blk] == 1 ? 0.0 : 1.0, 0.0);
      v[1] = make_double2(p.stagger[blk] == 1 ? 1.0 : 0.0, 0.0);
    }
    HIPCHK(copy_sync(h, h->site[st], v.data(), sizeof(cplx) * d, hipMemcpyHostToDevice));
  }
}

void reset_bookkeeping(mps_sim* h) {
  double sc[5] = {0.0, INFINITY, 0.0, 0.0, 0.0};
  HIPCHK(copy_sync(h, h->dscal, sc, sizeof(sc), hipMemcpyHostToDevice));
  int zero = 0;
  HIPCHK(copy_sync(h, h->lw.flag, &zero, sizeof(int), hipMemcpyHostToDevice));
  int zeros[2] = {0, 0};
  HIPCHK(copy_sync(h, h->dlogn, zeros, sizeof(zeros), hipMemcpyHostToDevice));
  h->nlog = 0;
  h->steps = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

mps_status mps_footprint_bytes(const mps_config* cfg, size_t* bytes) {
  const char* msg;
  mps_status st = validate(cfg, &msg);
  if (st != MPS_OK) return fail(nullptr, st, msg);
  if (!bytes) return fail(nullptr, MPS_E_INVAL, "bytes is NULL");
  Plan p;
  build_plan(cfg, p);
  *bytes = footprint(p);
  return MPS_OK;
}

mps_status mps_schedule_dump(const mps_config* cfg, int32_t nsteps, int32_t* ops, int32_t cap,
                             int32_t* len) {
  const char* msg;
  mps_status st = validate(cfg, &msg);
  if (st != MPS_OK) return fail(nullptr, st, msg);
  if (!len || nsteps < 0 || (cap > 0 && !ops)) return fail(nullptr, MPS_E_INVAL, "bad arguments");
  Plan p;
  build_plan(cfg, p);
  std::vector<int> pos = p.snake();
  std::vector<Op> all;
  for (int k = 0; k < nsteps; ++k) p.step_ops(pos, all);
  const long need = 6L * (long)all.size();
  *len = (int32_t)need;
  if (need > cap) return fail(nullptr, MPS_E_INVAL, "ops buffer too small");
  for (size_t k = 0; k < all.size(); ++k) {
    const Op& o = all[k];
    int32_t* r = ops + 6 * k;
    if (o.kind == 1) {
      r[0] = 1; r[1] = o.site; r[2] = o.swap; r[3] = o.gate; r[4] = o.block_a; r[5] = o.block_b;
    } else if (o.kind == 3) {
      r[0] = 3; r[1] = o.site; r[2] = o.site_b; r[3] = o.bit_a; r[4] = o.bit_b; r[5] = 0;
    } else {
      r[0] = 2; r[1] = o.site; r[2] = o.variant; r[3] = o.block_a; r[4] = 0; r[5] = 0;
    }
  }
  return MPS_OK;
}

mps_status mps_init_product(const mps_config* cfg, const mps_allocator* alloc, void* hip_stream,
                            mps_handle* out) {
  if (!out) return fail(nullptr, MPS_E_INVAL, "out is NULL");
  *out = nullptr;
  const char* msg;
  mps_status st = validate(cfg, &msg);
  if (st != MPS_OK) return fail(nullptr, st, msg);
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, MPS_E_INVAL, "allocator incomplete");
  mps_sim* h = new mps_sim();
  h->cfg = *cfg;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  h->gprec = cfg->precision == MPS_C64_FP32ACC ? GEMM_F32
           : cfg->precision == MPS_BF16X3_FP32ACC ? GEMM_BF16X3 : GEMM_F64;
  if (alloc) {
    h->alloc = *alloc;
    h->has_alloc = true;
  }
  try {
    build_plan(cfg, h->plan);
    const Plan& p = h->plan;
    Sizes z = plan_sizes(p);
    LwSizes l = lw_sizes(z);
    h->site.resize(p.N);
    for (int s = 0; s < p.N; ++s) h->site[s] = dalloc<cplx>(h, (long)p.xcap[s] * p.dmax * p.xcap[s + 1]);
    h->theta = dalloc<cplx>(h, z.theta);
    h->theta_elems = z.theta;
    h->gram = dalloc<cplx>(h, z.gram);
    h->tmpA = dalloc<cplx>(h, z.tmp);
    h->tmpB = dalloc<cplx>(h, z.tmp);
    h->tmpC = dalloc<cplx>(h, z.tmp);
    h->env[0] = dalloc<cplx>(h, z.env);
    h->env[1] = dalloc<cplx>(h, z.env);
    h->envx = dalloc<cplx>(h, z.envx);
    h->dscal = dalloc<double>(h, 16);
    h->dlogn = dalloc<int>(h, 2);
    h->dpartial = dalloc<double>(h, 4096);
    alloc_linalg(h, z, l);
    // gate tables
    long off = 0;
    for (auto& t : p.pair_phase) { h->pair_off.push_back(off); off += (long)t.size(); }
    h->d_pairs = dalloc<cplx>(h, off);
    {
      std::vector<cplx> hp(std::max<long>(off, 1));
      long o2 = 0;
      for (auto& t : p.pair_phase)
        for (auto& z2 : t) hp[o2++] = make_double2(z2.real(), z2.imag());
      if (off) HIPCHK(copy_sync(h, h->d_pairs, hp.data(), sizeof(cplx) * off, hipMemcpyHostToDevice));
    }
    long goff = 0;
    std::vector<cplx> hg;
    for (int v = 0; v < 4; ++v)
      for (int b = 0; b < p.nblocks(); ++b) {
        h->gate_off[v].push_back(goff);
        for (auto& z2 : p.site_gate[v][b]) hg.push_back(make_double2(z2.real(), z2.imag()));
        goff += (long)p.site_gate[v][b].size();
      }
    h->d_gates = dalloc<cplx>(h, goff);
    HIPCHK(copy_sync(h, h->d_gates, hg.data(), sizeof(cplx) * goff, hipMemcpyHostToDevice));
    std::vector<double> hz;
    for (int b = 0; b < p.nblocks(); ++b) {
      h->zsum_off.push_back((long)hz.size());
      for (double zz : p.zsum[b]) hz.push_back(zz);
    }
    h->d_zsum = dalloc<double>(h, (long)hz.size());
    HIPCHK(copy_sync(h, h->d_zsum, hz.data(), sizeof(double) * hz.size(), hipMemcpyHostToDevice));
    h->d_wt = dalloc<cplx>(h, 136 * 16 + 256);
    if (p.model == 1) {
      std::vector<cplx> hx(5 * 16, make_double2(0.0, 0.0));
      for (int v = 1; v <= 4; ++v)
        for (int k = 0; k < 16; ++k) hx[v * 16 + k] = make_double2(p.xy_gate[v][k].real(), p.xy_gate[v][k].imag());
      h->d_xy = dalloc<cplx>(h, 5 * 16);
      HIPCHK(copy_sync(h, h->d_xy, hx.data(), sizeof(cplx) * hx.size(), hipMemcpyHostToDevice));
    }
    // state
    h->pos = p.snake();
    h->bond.assign(p.N + 1, 1);
    h->centre = 0;
    upload_product_state(h);
    h->log_cap = 0;
    ensure_log(h, 64L * (11 * p.R + 4));
    reset_bookkeeping(h);
    if (p.model == 1) xy_prepare(h);
    HIPCHK(hipStreamSynchronize(h->stream));
  } catch (NoMem&) {
    mps_free(h);
    return fail(nullptr, MPS_E_NOMEM, "device allocation failed");
  } catch (HipError& e) {
    std::string m = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    mps_free(h);
    return fail(nullptr, MPS_E_DEVICE, m);
  } catch (BoundsError& e) {
    mps_free(h);
    return fail(nullptr, MPS_E_DEVICE, "operand out of bounds, not launched: " + e.msg);
  }
  *out = h;
  return MPS_OK;
}

#define GUARD(h)                                                     \
  if (!(h)) return fail(nullptr, MPS_E_INVAL, "handle is NULL");     \
  if ((h)->failed) return fail((h), MPS_E_STATE, "handle has failed")

#define TRYDEV(h, ...)                                                                       \
  try {                                                                                      \
    __VA_ARGS__;                                                                             \
  } catch (HipError & e) {                                                                   \
    return fail((h), MPS_E_DEVICE, std::string("HIP error in ") + e.what + ": " +            \
                                       hipGetErrorString(e.e));                              \
  } catch (NoMem&) {                                                                         \
    return fail((h), MPS_E_DEVICE, "device allocation failed");                              \
  } catch (BoundsError & e) {                                                                \
    return fail((h), MPS_E_DEVICE, "operand out of bounds, not launched: " + e.msg);         \
  }

mps_status mps_apply_trotter_step(mps_handle h, int32_t nsteps) {
  GUARD(h);
  if (nsteps < 0) return fail(h, MPS_E_INVAL, "nsteps < 0");
  TRYDEV(h, for (int k = 0; k < nsteps; ++k) run_step(h); HIPCHK(hipGetLastError()));
  return MPS_OK;
}

mps_status mps_apply_trotter_step_batched(mps_handle* hs, int32_t count, int32_t nsteps) {
  if (!hs || count < 0 || nsteps < 0) return fail(nullptr, MPS_E_INVAL, "bad arguments");
  for (int k = 0; k < count; ++k) {
    if (!hs[k]) return fail(nullptr, MPS_E_INVAL, "NULL handle in batch");
    if (hs[k]->failed) return fail(hs[k], MPS_E_STATE, "handle has failed");
    for (int k2 = 0; k2 < k; ++k2)
      if (hs[k2] == hs[k]) return fail(nullptr, MPS_E_INVAL, "handle repeated in batch");
  }
  // One host thread per instance, each enqueueing on its instance's own
  // stream: a single thread would block on one instance's full launch queue
  // while the other instances' queues drain.
  std::vector<mps_status> st(count, MPS_OK);
  auto run = [&](int k) {
    mps_sim* h = hs[k];
    if (hipSetDevice(h->device) != hipSuccess) {
      st[k] = fail(h, MPS_E_DEVICE, "hipSetDevice failed");
      return;
    }
    st[k] = mps_apply_trotter_step(h, nsteps);
  };
  if (count == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    th.reserve(count);
    for (int k = 0; k < count; ++k) th.emplace_back(run, k);
    for (auto& t : th) t.join();
  }
  for (int k = 0; k < count; ++k)
    if (st[k] != MPS_OK) return st[k];
  return MPS_OK;
}

mps_status mps_sync(mps_handle h) {
  GUARD(h);
  return check_device(h);
}

mps_status mps_measure(mps_handle h, double gamma, mps_obs* out) {
  GUARD(h);
  if (!out) return fail(h, MPS_E_INVAL, "out is NULL");
  double e[3], ex[3] = {0.0, 0.0, 0.0};
  double sc[2];
  int counts[2] = {0, 0};
  const bool xy = h->plan.model == 1;
  TRYDEV(h, measure_sweep(h, e, 0);
         if (xy) measure_sweep(h, ex, 1);
         HIPCHK(copy_sync(h, sc, h->dscal, sizeof(sc), hipMemcpyDeviceToHost));
         HIPCHK(copy_sync(h, counts, h->dlogn, sizeof(counts), hipMemcpyDeviceToHost)));
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  const double n = h->plan.n;
  mps_obs o{};
  o.step = h->steps;
  o.eig_suspect = counts[1];
  o.norm = e[0];
  o.z = e[1] / (n * e[0]);
  o.z2 = xy ? ex[2] / (n * n * ex[0]) : e[2] / (n * n * e[0]);
  if (!std::isfinite(o.z) || !std::isfinite(o.z2)) return fail(h, MPS_E_NUMERIC, "non-finite observable");
  o.log_fidelity = sc[0];
  o.fidelity = std::exp(sc[0]);
  o.min_gap = sc[1];
  o.z_rescaled = o.fidelity * o.z;
  o.gamma = gamma;
  o.z2_rescaled = gamma >= 0 ? o.z2 * std::pow(o.fidelity, gamma) : NAN;
  *out = o;
  return MPS_OK;
}

mps_status mps_fidelity(mps_handle h, double* fidelity, double* log_fidelity) {
  GUARD(h);
  if (!fidelity || !log_fidelity) return fail(h, MPS_E_INVAL, "NULL output");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  double sc = 0;
  if (copy_sync(h, &sc, h->dscal, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, MPS_E_DEVICE, "copy failed");
  *log_fidelity = sc;
  *fidelity = std::exp(sc);
  return MPS_OK;
}

void mps_free(mps_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  linalg_release(h->lw);
  for (void* p : h->allocations) {
    bounds_unregister(p);
    if (h->has_alloc) h->alloc.free(h->alloc.ctx, p, (void*)h->stream);
    else (void)hipFree(p);
  }
  delete h;
}

mps_status mps_bond_dims(mps_handle h, int32_t* dims, int32_t cap, int32_t* len) {
  GUARD(h);
  if (!len) return fail(h, MPS_E_INVAL, "len is NULL");
  *len = (int32_t)h->bond.size();
  if (cap < *len || !dims) return fail(h, MPS_E_INVAL, "buffer too small");
  for (size_t k = 0; k < h->bond.size(); ++k) dims[k] = h->bond[k];
  return MPS_OK;
}

mps_status mps_site_blocks(mps_handle h, int32_t* blocks, int32_t cap, int32_t* len) {
  GUARD(h);
  if (!len) return fail(h, MPS_E_INVAL, "len is NULL");
  *len = (int32_t)h->pos.size();
  if (cap < *len || !blocks) return fail(h, MPS_E_INVAL, "buffer too small");
  for (size_t k = 0; k < h->pos.size(); ++k) blocks[k] = h->pos[k];
  return MPS_OK;
}

mps_status mps_get_site(mps_handle h, int32_t p, double* re_im, int64_t cap, int32_t* dims) {
  GUARD(h);
  if (p < 0 || p >= h->plan.N || !dims) return fail(h, MPS_E_INVAL, "bad site");
  const int b0 = h->bond[p], d = h->plan.dim(h->pos[p]), b1 = h->bond[p + 1];
  dims[0] = b0; dims[1] = d; dims[2] = b1;
  const long len = (long)b0 * d * b1;
  if (cap < len || !re_im) return fail(h, MPS_E_INVAL, "buffer too small");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  if (copy_sync(h, re_im, h->site[p], sizeof(cplx) * len, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, MPS_E_DEVICE, "copy failed");
  return MPS_OK;
}

mps_status mps_set_state(mps_handle h, const int32_t* bonds, const double* const* sites, int32_t centre) {
  GUARD(h);
  const Plan& p = h->plan;
  if (!bonds || !sites || centre < 0 || centre >= p.N) return fail(h, MPS_E_INVAL, "bad arguments");
  if (bonds[0] != 1 || bonds[p.N] != 1) return fail(h, MPS_E_INVAL, "end bonds must be 1");
  for (int b = 0; b <= p.N; ++b)
    if (bonds[b] < 1 || bonds[b] > p.cap[b]) return fail(h, MPS_E_INVAL, "bond exceeds its cap");
  for (int s = 0; s < p.N; ++s)
    if (!sites[s]) return fail(h, MPS_E_INVAL, "NULL site");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  TRYDEV(h, {
    std::vector<int> pos = p.snake();
    for (int s = 0; s < p.N; ++s) {
      long len = (long)bonds[s] * p.dim(pos[s]) * bonds[s + 1];
      HIPCHK(copy_sync(h, h->site[s], sites[s], sizeof(cplx) * len, hipMemcpyHostToDevice));
    }
    h->pos = pos;
    h->bond.assign(bonds, bonds + p.N + 1);
    h->centre = centre;
    reset_bookkeeping(h);
  });
  return MPS_OK;
}

mps_status mps_apply_two_site(mps_handle h, int32_t site, int32_t swap, int32_t gate) {
  GUARD(h);
  if (site < 0 || site + 1 >= h->plan.N) return fail(h, MPS_E_INVAL, "bad site");
  if (h->plan.schedule == 4)
    return fail(h, MPS_E_UNSUPPORTED, "two-site updates are not sized for the gate-by-gate schedule");
  TRYDEV(h, two_site(h, site, swap ? 1 : 0, gate ? 1 : 0, -1); HIPCHK(hipGetLastError()));
  return MPS_OK;
}

mps_status mps_apply_two_site_toward(mps_handle h, int32_t site, int32_t swap, int32_t gate,
                                     int32_t next_site) {
  GUARD(h);
  if (site < 0 || site + 1 >= h->plan.N) return fail(h, MPS_E_INVAL, "bad site");
  if (h->plan.schedule == 4)
    return fail(h, MPS_E_UNSUPPORTED, "two-site updates are not sized for the gate-by-gate schedule");
  TRYDEV(h, two_site(h, site, swap ? 1 : 0, gate ? 1 : 0, next_site); HIPCHK(hipGetLastError()));
  return MPS_OK;
}

mps_status mps_apply_single_site(mps_handle h, int32_t site, int32_t variant) {
  GUARD(h);
  if (site < 0 || site >= h->plan.N) return fail(h, MPS_E_INVAL, "bad site");
  if (variant < 0 || variant > 2) return fail(h, MPS_E_INVAL, "variant must be 0, 1 or 2");
  if (h->plan.model == 1) return fail(h, MPS_E_UNSUPPORTED, "no single-site layer in the XY step");
  TRYDEV(h, single_site(h, site, variant); HIPCHK(hipGetLastError()));
  return MPS_OK;
}

mps_status mps_truncation_log(mps_handle h, double* f, double* gap, int32_t cap, int32_t* len) {
  GUARD(h);
  if (!len) return fail(h, MPS_E_INVAL, "len is NULL");
  *len = (int32_t)h->nlog;
  if (cap < h->nlog || (h->nlog > 0 && (!f || !gap))) return fail(h, MPS_E_INVAL, "buffer too small");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  std::vector<double> buf(2 * std::max<long>(h->nlog, 1));
  if (h->nlog > 0 &&
      copy_sync(h, buf.data(), h->flog, sizeof(double) * 2 * h->nlog, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, MPS_E_DEVICE, "copy failed");
  for (long k = 0; k < h->nlog; ++k) {
    f[k] = buf[2 * k];
    gap[k] = buf[2 * k + 1];
  }
  return MPS_OK;
}

mps_status mps_bond_spectrum(mps_handle h, int32_t bond, double* sv, int32_t cap, int32_t* len) {
  GUARD(h);
  const Plan& p = h->plan;
  if (bond < 1 || bond >= p.N || !len) return fail(h, MPS_E_INVAL, "bad bond");
  TRYDEV(h, {
    move_centre(h, bond - 1);
    const int c = bond - 1;
    const int b0 = h->bond[c], d = p.dim(h->pos[c]), b1 = h->bond[c + 1];
    const int m = b0 * d;
    *len = b1;
    if (cap < b1 || !sv) return fail(h, MPS_E_INVAL, "buffer too small");
    // G = A^H A (b1 x b1), eigenvalues = squared Schmidt values
    ZGemm gg = zgemm_args(b1, b1, m, zop(h->site[c], b1, 1, 1), zop(h->site[c], b1, 0), h->gram, b1, 1,
                          make_double2(1, 0), make_double2(0, 0));
    gg.lower_only = 1;
    zgemm(gg, nullptr, 0, h->stream, &h->prof);
    hetrd_lower(b1, h->gram, b1, h->lw, h->stream);
    tridiag_eigvals(b1, 0, b1, h->lw, h->stream);
    std::vector<double> lam(b1);
    HIPCHK(hipMemcpyAsync(lam.data(), h->lw.lam, sizeof(double) * b1, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < b1; ++k) sv[k] = std::sqrt(std::max(lam[b1 - 1 - k], 0.0));
  });
  return check_device(h);
}

mps_status mps_to_statevector(mps_handle h, double* re_im, int64_t len) {
  GUARD(h);
  const Plan& p = h->plan;
  if (p.n > 20) return fail(h, MPS_E_UNSUPPORTED, "state vector limited to 20 qubits");
  if (!re_im || len != (1LL << p.n)) return fail(h, MPS_E_INVAL, "len must be 2^n");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  typedef std::complex<double> zc;
  // contract on the host (diagnostic only): T has shape (prod d) x b
  std::vector<zc> T(1, zc(1, 0));
  long left = 1;
  for (int s = 0; s < p.N; ++s) {
    const int b0 = h->bond[s], d = p.dim(h->pos[s]), b1 = h->bond[s + 1];
    std::vector<zc> A((size_t)b0 * d * b1);
    if (copy_sync(h, A.data(), h->site[s], sizeof(zc) * A.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(h, MPS_E_DEVICE, "copy failed");
    std::vector<zc> U((size_t)left * d * b1, zc(0, 0));
    for (long x = 0; x < left; ++x)
      for (int a = 0; a < b0; ++a) {
        const zc t = T[(size_t)x * b0 + a];
        if (t == zc(0, 0)) continue;
        for (int sidx = 0; sidx < d; ++sidx)
          for (int c = 0; c < b1; ++c)
            U[((size_t)x * d + sidx) * b1 + c] += t * A[((size_t)a * d + sidx) * b1 + c];
      }
    T.swap(U);
    left *= d;
  }
  const int n = p.n;
  for (long x = 0; x < (1L << n); ++x) {
    long flat = 0;
    for (int s = 0; s < p.N; ++s) {
      const auto& qs = p.block_qubits[h->pos[s]];
      const int w = (int)qs.size();
      long sidx = 0;
      for (int j = 0; j < w; ++j) sidx |= ((x >> (n - 1 - qs[j])) & 1L) << (w - 1 - j);
      flat = flat * (1L << w) + sidx;
    }
    re_im[2 * x] = T[flat].real();
    re_im[2 * x + 1] = T[flat].imag();
  }
  return MPS_OK;
}

mps_status mps_set_progress(mps_handle h, mps_progress_fn fn, void* ctx) {
  GUARD(h);
  h->progress = fn;
  h->progress_ctx = ctx;
  return MPS_OK;
}

mps_status mps_eigh_top(int32_t n, int32_t q, int32_t eig_path, uint64_t seed, const double* gram,
                        double* lam, double* vecs, void* hip_stream) {
  if (n < 1 || q < 1 || q > n || (eig_path != 1 && eig_path != 2) || !gram || !lam || !vecs)
    return fail(nullptr, MPS_E_INVAL, "mps_eigh_top: bad arguments");
  mps_sim* h = new mps_sim();
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  mps_status st = MPS_OK;
  std::string msg;
  try {
    Sizes z;
    z.nmax = n; z.qmax = q; z.mmax = n;
    z.colmax = std::max<long>(q, TRD_NB);
    z.eig_path = eig_path;
    const LwSizes l = lw_sizes(z);
    alloc_linalg(h, z, l);
    h->gram = dalloc<cplx>(h, (long)n * n);
    h->tmpA = dalloc<cplx>(h, (long)n * q);
    h->tmpB = dalloc<cplx>(h, (long)n * q);
    HIPCHK(hipMemsetAsync(h->lw.flag, 0, 4 * sizeof(int), h->stream));
    HIPCHK(hipMemcpyAsync(h->gram, gram, sizeof(cplx) * (size_t)n * n, hipMemcpyHostToDevice, h->stream));
    if (eig_path == 2) heev_top_2stage(n, h->gram, n, q, h->tmpB, q, h->tmpA, h->lw, seed, h->stream);
    else heev_top(n, h->gram, n, q, h->tmpB, q, h->tmpA, h->lw, seed, h->stream);
    HIPCHK(hipGetLastError());
    const int extra = (q < n) ? 1 : 0;
    std::vector<double> asc(q + extra);
    HIPCHK(hipMemcpyAsync(asc.data(), h->lw.lam, sizeof(double) * asc.size(), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipMemcpyAsync(vecs, h->tmpB, sizeof(cplx) * (size_t)n * q, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int j = 0; j < q; ++j) lam[j] = asc[extra + q - 1 - j];
  } catch (NoMem&) {
    st = MPS_E_NOMEM;
    msg = "mps_eigh_top: device allocation failed";
  } catch (HipError& e) {
    st = MPS_E_DEVICE;
    msg = std::string("mps_eigh_top: HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
  } catch (BoundsError& e) {
    st = MPS_E_DEVICE;
    msg = "mps_eigh_top: operand out of bounds, not launched: " + e.msg;
  }
  mps_free(h);
  if (st != MPS_OK) return fail(nullptr, st, msg);
  return MPS_OK;
}

mps_status mps_debug_check_bounds(int32_t enable) {
  bounds_set_checking(enable != 0);
  return MPS_OK;
}

mps_status mps_profile(mps_handle h, int32_t kind) {
  GUARD(h);
  if (kind < PROF_OFF || kind > PROF_THETA) return fail(h, MPS_E_INVAL, "unknown launch class");
  h->prof.reset(kind);
  return MPS_OK;
}

mps_status mps_profile_min_work(mps_handle h, double min_work) {
  GUARD(h);
  if (!(min_work >= 0.0)) return fail(h, MPS_E_INVAL, "min_work must be >= 0");
  h->prof.flush();
  h->prof.min_work = min_work;
  return MPS_OK;
}

mps_status mps_profile_read(mps_handle h, double* total_ms, int64_t* launches, double* work) {
  GUARD(h);
  if (!total_ms || !launches || !work) return fail(h, MPS_E_INVAL, "NULL output");
  mps_status st = check_device(h);
  if (st != MPS_OK) return st;
  h->prof.flush();
  *total_ms = h->prof.ms;
  *launches = h->prof.launches;
  *work = h->prof.work;
  return MPS_OK;
}

const char* mps_last_error(mps_handle h) {
  if (h) return h->err.c_str();
  return g_tl_error.c_str();
}

}  // extern "C"
