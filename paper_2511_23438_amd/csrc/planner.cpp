// Host planning: geometry, schedule and gate tables of the block MPS.
//
// Model: H = J sum_<ij> Z_i Z_j + h sum_i X_i on an R x C grid with periodic
// wrap (eq. "hamiltonian"); one Trotter step exp(-i dt H_X) exp(-i dt H_ZZ)
// (first order) or exp(-i dt H_X/2) exp(-i dt H_ZZ) exp(-i dt H_X/2)
// (eq. "trotter_step"). Blocks are half rows fused into sites of local
// dimension 2^width (results section, figure of the 7x8 grouping) on a row
// snake (supplement, "MPS Ordering").
#include "planner.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <set>

namespace mpsim {

mps_status validate(const mps_config* cfg, const char** msg) {
  if (!cfg) { *msg = "config is NULL"; return MPS_E_INVAL; }
  if (cfg->layers < 0) { *msg = "layers must be >= 0"; return MPS_E_INVAL; }
  if (cfg->model != 0 && cfg->model != 1) { *msg = "model must be 0 (TFIM) or 1 (XY)"; return MPS_E_INVAL; }
  if (cfg->model == 1) {
    if (cfg->layers != 0) { *msg = "the XY model runs on the grid (layers 0)"; return MPS_E_INVAL; }
    if (cfg->periodic != 0) { *msg = "the XY model has open boundaries (periodic 0)"; return MPS_E_INVAL; }
    if (cfg->trotter_order != 2) { *msg = "the XY step is second order (trotter_order 2)"; return MPS_E_INVAL; }
    if (cfg->schedule != 3) { *msg = "the XY model uses schedule 3"; return MPS_E_INVAL; }
    if (cfg->rows < 1 || cfg->cols < 1 || cfg->rows * cfg->cols < 2) { *msg = "need at least 2 qubits"; return MPS_E_INVAL; }
    if ((long)cfg->rows * cfg->cols > 256) { *msg = "XY grid with > 256 qubits unsupported"; return MPS_E_UNSUPPORTED; }
  } else if (cfg->layers >= 2) {
    if (cfg->rows < 1 || cfg->cols < 1) { *msg = "cube extents must be >= 1"; return MPS_E_INVAL; }
    if ((long)cfg->rows * cfg->cols * cfg->layers > 256) { *msg = "cube with > 256 sites unsupported"; return MPS_E_UNSUPPORTED; }
    if (cfg->schedule != 3 && cfg->schedule != 4) { *msg = "the cube needs schedule 3 or 4"; return MPS_E_INVAL; }
  } else {
    if (cfg->rows < 1 || cfg->cols < 2) { *msg = "need rows >= 1 and cols >= 2"; return MPS_E_INVAL; }
    if (cfg->cols > 8) { *msg = "cols > 8 (block width > 4, d > 16) unsupported"; return MPS_E_UNSUPPORTED; }
    if (cfg->rows > 64) { *msg = "rows > 64 unsupported"; return MPS_E_UNSUPPORTED; }
  }
  if (cfg->chi_max < 1) { *msg = "chi_max must be >= 1"; return MPS_E_INVAL; }
  if (cfg->chi_max > 4096) { *msg = "chi_max > 4096 unsupported"; return MPS_E_UNSUPPORTED; }
  if (cfg->precision < 0 || cfg->precision > 2) { *msg = "bad precision"; return MPS_E_INVAL; }
  if (cfg->trotter_order != 1 && cfg->trotter_order != 2) { *msg = "trotter_order must be 1 or 2"; return MPS_E_INVAL; }
  if (cfg->schedule < 1 || cfg->schedule > 4) { *msg = "schedule must be 1, 2, 3 or 4"; return MPS_E_INVAL; }
  if (cfg->periodic != 0 && cfg->periodic != 1) { *msg = "periodic must be 0 or 1"; return MPS_E_INVAL; }
  if (cfg->eig_path < 0 || cfg->eig_path > 2) { *msg = "eig_path must be 0, 1 or 2"; return MPS_E_INVAL; }
  if (cfg->eig_batch < 0 || cfg->eig_batch > 1024) { *msg = "eig_batch must be in 0..1024"; return MPS_E_INVAL; }
  if (!std::isfinite(cfg->J) || !std::isfinite(cfg->h) || !std::isfinite(cfg->dt) ||
      !std::isfinite(cfg->theta0)) { *msg = "non-finite parameter"; return MPS_E_INVAL; }
  *msg = "";
  return MPS_OK;
}

std::vector<int> Plan::snake() const { return snake_order; }

// XY model, one step (supplement, eq. "xy_trotter_step"): sublayers
// A/2 B/2 C/2 D C/2 B/2 A/2; inside a sublayer the bonds are taken in the
// order of their chain positions, and each is routed and returned: the qubit
// at pb is swapped leftwards to pa+1, the gate acts on (pa, pa+1), and it is
// swapped back.
void Plan::xy_ops(std::vector<int>& pos, std::vector<Op>& out, bool prep) const {
  static const int layer[7] = {0, 1, 2, 3, 2, 1, 0};
  static const int variant[7] = {1, 1, 1, 2, 1, 1, 1};
  auto u2 = [&](int site, int swap, int gate) {
    Op o{};
    o.kind = 1; o.site = site; o.swap = swap; o.gate = gate;
    o.block_a = pos[site]; o.block_b = pos[site + 1];
    out.push_back(o);
    if (swap) std::swap(pos[site], pos[site + 1]);
  };
  for (int k = 0; k < 7; ++k) {
    std::vector<int> where(nb, 0);
    for (int p = 0; p < N; ++p) where[pos[p]] = p;
    std::vector<std::pair<int, int>> pairs;
    for (auto& bd : xy_sub[layer[k]])
      pairs.push_back({std::min(where[bd.first], where[bd.second]),
                       std::max(where[bd.first], where[bd.second])});
    std::sort(pairs.begin(), pairs.end());
    const int gv = variant[k] + (prep ? 2 : 0);
    for (auto& pr : pairs) {
      const int pa = pr.first, pb = pr.second;
      for (int p = pb - 1; p > pa; --p) u2(p, 1, 0);
      u2(pa, 0, gv);
      for (int p = pa + 1; p < pb; ++p) u2(p, 1, 0);
    }
  }
}

void Plan::step_ops(std::vector<int>& pos, std::vector<Op>& out) const {
  if (model == 1) {
    xy_ops(pos, out, false);
    return;
  }
  auto u2 = [&](int site, int swap, int gate) {
    Op o{};
    o.kind = 1; o.site = site; o.swap = swap;
    o.block_a = pos[site]; o.block_b = pos[site + 1];
    o.gate = (gate && coupled(o.block_a, o.block_b) >= 0) ? 1 : 0;
    out.push_back(o);
    if (swap) std::swap(pos[site], pos[site + 1]);
  };
  auto u1 = [&](int site, int variant) {
    Op o{};
    o.kind = 2; o.site = site; o.variant = variant; o.block_a = pos[site]; o.block_b = -1;
    out.push_back(o);
  };
  if (schedule == 4) {
    // gate by gate: every ZZ bond between two blocks is its own gate, a
    // rank-2 operator on the span of sites between them; blocks never move.
    // Order: (first site, second site, bit in the first block, bit in the
    // second block).
    if (order == 2)
      for (int p = 0; p < N; ++p) u1(p, 1);
    std::vector<int> where(nb, 0), blk_of(n, 0), idx_in(n, 0);
    for (int p = 0; p < N; ++p) where[pos[p]] = p;
    for (int b = 0; b < nb; ++b)
      for (size_t j = 0; j < block_qubits[b].size(); ++j) {
        blk_of[block_qubits[b][j]] = b;
        idx_in[block_qubits[b][j]] = (int)j;
      }
    std::vector<std::array<int, 4>> gates;
    for (auto& bd : bonds) {
      int a = blk_of[bd.first], b = blk_of[bd.second];
      if (a == b) continue;
      int sa = where[a], sb = where[b], ja = idx_in[bd.first], jb = idx_in[bd.second];
      if (sa > sb) { std::swap(sa, sb); std::swap(ja, jb); }
      gates.push_back({sa, sb, ja, jb});
    }
    std::sort(gates.begin(), gates.end());
    for (auto& gt : gates) {
      Op o{};
      o.kind = 3; o.site = gt[0]; o.site_b = gt[1]; o.bit_a = gt[2]; o.bit_b = gt[3];
      o.block_a = pos[gt[0]]; o.block_b = pos[gt[1]];
      out.push_back(o);
    }
    for (int p = 0; p < N; ++p) u1(p, order == 1 ? 0 : 2);
    return;
  }
  if (schedule == 3) {
    // route and return: coupled pairs in the order of their chain positions
    // at the start of the step; the block at pb travels to pa+1 by SWAP
    // updates, the phase gate acts on (pa, pa+1), and the block travels back
    if (order == 2)
      for (int p = 0; p < N; ++p) u1(p, 1);
    std::vector<int> where(nb, 0);
    for (int p = 0; p < N; ++p) where[pos[p]] = p;
    std::vector<std::pair<int, int>> pairs;  // (pa, pb)
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b)
        if (coupled(a, b) >= 0)
          pairs.push_back({std::min(where[a], where[b]), std::max(where[a], where[b])});
    std::sort(pairs.begin(), pairs.end());
    for (auto& pr : pairs) {
      const int pa = pr.first, pb = pr.second;
      for (int p = pb - 1; p > pa; --p) u2(p, 1, 0);
      u2(pa, 0, 1);
      for (int p = pa + 1; p < pb; ++p) u2(p, 1, 0);
    }
    for (int p = 0; p < N; ++p) u1(p, order == 1 ? 0 : 2);
    return;
  }
  const bool rotating = schedule == 2 && periodic && R >= 3;
  const int nfacing = rotating ? R - 2 : R - 1;
  if (order == 2)
    for (int p = 0; p < N; ++p) u1(p, 1);
  // vertical neighbours facing each other between chain rows r and r+1
  for (int r = 0; r < nfacing; ++r) u2(2 * r + 1, 0, 1);
  // the two blocks of every row, fused with a SWAP
  for (int r = 0; r < R; ++r) u2(2 * r, 1, 1);
  // the other vertical neighbours, now facing each other
  for (int r = 0; r < nfacing; ++r) u2(2 * r + 1, 0, 1);
  if (rotating) {
    // rotating rows: the last chain row moves to the chain front; crossings
    // with the blocks it is coupled to (chain rows R-2 and 0) carry the gate.
    // For odd R the row is reversed first so chain rows keep facing
    // same-side blocks.
    if (R % 2 == 1) u2(2 * R - 2, 1, 0);
    for (int p = 2 * R - 3; p >= 0; --p) u2(p, 1, 1);
    for (int p = 2 * R - 2; p >= 1; --p) u2(p, 1, 1);
  } else if (periodic && R >= 3) {
    // periodic wrap between the last and the first row: route the last-row
    // block next to its row-0 partner, gate, route back
    for (int p0 = 1; p0 >= 0; --p0) {
      int want = 2 * (R - 1) + (pos[p0] & 1);
      int t = (int)(std::find(pos.begin(), pos.end(), want) - pos.begin());
      for (int p = t - 1; p > p0; --p) u2(p, 1, 0);
      u2(p0, 0, 1);
      for (int p = p0 + 1; p < t; ++p) u2(p, 1, 0);
    }
  }
  for (int p = 0; p < N; ++p) u1(p, order == 1 ? 0 : 2);
}

static int zval(int s, int w, int j) { return 1 - 2 * ((s >> (w - 1 - j)) & 1); }

// Cube: qubit (x, y, z) -> (x*Ly + y)*Lz + z, one qubit per block; snake
// with x slowest, rows y alternating direction per layer, z alternating per
// row visited; neighbours along each axis (wrap only when periodic).
static void cube_geometry(const mps_config* cfg, Plan& p) {
  const int lx = cfg->rows, ly = cfg->cols, lz = cfg->layers;
  p.R = lx; p.C = ly; p.Lz = lz;
  p.n = lx * ly * lz; p.N = p.n; p.nb = p.n;
  p.wL = p.wR = 1;
  p.dmax = 2;
  p.block_width.assign(p.nb, 1);
  p.block_qubits.assign(p.nb, {});
  for (int q = 0; q < p.n; ++q) p.block_qubits[q].push_back(q);
  auto idx = [&](int x, int y, int z) { return (x * ly + y) * lz + z; };
  p.snake_order.clear();
  int t = 0;
  for (int x = 0; x < lx; ++x)
    for (int yy = 0; yy < ly; ++yy, ++t) {
      const int y = (x % 2 == 0) ? yy : ly - 1 - yy;
      for (int zz = 0; zz < lz; ++zz) p.snake_order.push_back(idx(x, y, (t % 2 == 0) ? zz : lz - 1 - zz));
    }
  std::set<std::pair<int, int>> seen;
  p.bonds.clear();
  const int dims[3] = {lx, ly, lz};
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y)
      for (int z = 0; z < lz; ++z)
        for (int ax = 0; ax < 3; ++ax) {
          int c[3] = {x, y, z};
          c[ax] += 1;
          if (c[ax] >= dims[ax]) {
            if (!p.periodic || dims[ax] < 2) continue;
            c[ax] = 0;
          }
          const int q = idx(x, y, z), q2 = idx(c[0], c[1], c[2]);
          if (q == q2) continue;
          std::pair<int, int> key(std::min(q, q2), std::max(q, q2));
          if (seen.insert(key).second) p.bonds.push_back(key);
        }
}

// XY model: one qubit per site on the rows x cols grid, row snake (even rows
// left to right, odd rows right to left), open boundaries; sublayers A / B:
// horizontal bonds whose first column is even / odd, C / D: vertical bonds
// whose first row is even / odd.
static void xy_geometry(const mps_config* cfg, Plan& p) {
  const int R = cfg->rows, C = cfg->cols;
  p.R = R; p.C = C; p.Lz = 0;
  p.n = R * C; p.N = p.n; p.nb = p.n;
  p.wL = p.wR = 1;
  p.dmax = 2;
  p.block_width.assign(p.nb, 1);
  p.block_qubits.assign(p.nb, {});
  for (int q = 0; q < p.n; ++q) p.block_qubits[q].push_back(q);
  p.snake_order.clear();
  for (int r = 0; r < R; ++r)
    for (int cc = 0; cc < C; ++cc) p.snake_order.push_back(r * C + ((r % 2 == 0) ? cc : C - 1 - cc));
  p.xy_sub.assign(4, {});
  p.bonds.clear();
  for (int r = 0; r < R; ++r)
    for (int c = 0; c < C; ++c) {
      if (c + 1 < C) p.xy_sub[c % 2].push_back({r * C + c, r * C + c + 1});
      if (r + 1 < R) p.xy_sub[2 + r % 2].push_back({r * C + c, (r + 1) * C + c});
    }
  p.stagger.assign(p.n, 1);
  for (int q = 0; q < p.n; ++q) p.stagger[q] = ((q / C + q % C) % 2 == 0) ? 1 : -1;
}

// Grid: half-row blocks (ceil(C/2) and floor(C/2) columns), row snake of
// blocks, right and down neighbours with wrap.
static void grid_geometry(const mps_config* cfg, Plan& p) {
  p.R = cfg->rows; p.C = cfg->cols; p.Lz = 0;
  p.n = p.R * p.C; p.N = 2 * p.R; p.nb = 2 * p.R;
  p.wL = (p.C + 1) / 2; p.wR = p.C / 2;
  p.dmax = 1 << p.wL;
  const int nb = p.nb;
  p.block_width.assign(nb, 0);
  p.block_qubits.assign(nb, {});
  for (int r = 0; r < p.R; ++r) {
    p.block_width[2 * r] = p.wL;
    p.block_width[2 * r + 1] = p.wR;
    for (int c = 0; c < p.wL; ++c) p.block_qubits[2 * r].push_back(r * p.C + c);
    for (int c = p.wL; c < p.C; ++c) p.block_qubits[2 * r + 1].push_back(r * p.C + c);
  }
  p.snake_order.clear();
  for (int r = 0; r < p.R; ++r) {
    if (r % 2 == 0) { p.snake_order.push_back(2 * r); p.snake_order.push_back(2 * r + 1); }
    else { p.snake_order.push_back(2 * r + 1); p.snake_order.push_back(2 * r); }
  }
  // ZZ bonds: right and down neighbours with wrap, unordered pairs kept once
  std::set<std::pair<int, int>> seen;
  p.bonds.clear();
  for (int r = 0; r < p.R; ++r)
    for (int c = 0; c < p.C; ++c) {
      int q = r * p.C + c;
      int cand[2] = {-1, -1};
      if (c + 1 < p.C) cand[0] = r * p.C + c + 1;
      else if (p.periodic) cand[0] = r * p.C;
      if (r + 1 < p.R) cand[1] = (r + 1) * p.C + c;
      else if (p.periodic) cand[1] = c;
      for (int k = 0; k < 2; ++k) {
        int q2 = cand[k];
        if (q2 < 0 || q2 == q) continue;
        std::pair<int, int> key(std::min(q, q2), std::max(q, q2));
        if (seen.insert(key).second) p.bonds.push_back(key);
      }
    }
}

void build_plan(const mps_config* cfg, Plan& p) {
  p.chi = cfg->chi_max; p.order = cfg->trotter_order; p.periodic = cfg->periodic;
  p.schedule = cfg->schedule;
  p.eig_path = cfg->eig_path;
  p.eig_batch = cfg->eig_batch > 0 ? cfg->eig_batch : 1024;
  p.J = cfg->J; p.h = cfg->h; p.dt = cfg->dt; p.theta0 = cfg->theta0;
  p.model = cfg->model;
  if (cfg->model == 1) xy_geometry(cfg, p);
  else if (cfg->layers >= 2) cube_geometry(cfg, p);
  else grid_geometry(cfg, p);
  const int nb = p.nb;
  std::vector<int> blk_of(p.n), idx_in(p.n);
  for (int b = 0; b < nb; ++b)
    for (size_t j = 0; j < p.block_qubits[b].size(); ++j) {
      blk_of[p.block_qubits[b][j]] = b;
      idx_in[p.block_qubits[b][j]] = (int)j;
    }
  // block-pair phases D_ab[s_a][s_b] = exp(-i J dt sum_crossing z z')
  p.pair_index.assign(nb * nb, -1);
  p.pair_phase.clear();
  std::vector<std::vector<double>> energy_pair;
  std::vector<std::vector<double>> energy_intra(nb);
  for (int b = 0; b < nb; ++b) energy_intra[b].assign(p.dim(b), 0.0);
  for (auto& bd : p.bonds) {
    int a = blk_of[bd.first], b = blk_of[bd.second];
    int ja = idx_in[bd.first], jb = idx_in[bd.second];
    if (a == b) {
      int w = p.block_width[a];
      for (int s = 0; s < p.dim(a); ++s) energy_intra[a][s] += zval(s, w, ja) * zval(s, w, jb);
      continue;
    }
    if (a > b) { std::swap(a, b); std::swap(ja, jb); }
    int& pi = p.pair_index[a * nb + b];
    if (pi < 0) {
      pi = (int)energy_pair.size();
      energy_pair.push_back(std::vector<double>(p.dim(a) * p.dim(b), 0.0));
    }
    int wa = p.block_width[a], wb = p.block_width[b];
    for (int sa = 0; sa < p.dim(a); ++sa)
      for (int sb = 0; sb < p.dim(b); ++sb)
        energy_pair[pi][sa * p.dim(b) + sb] += zval(sa, wa, ja) * zval(sb, wb, jb);
  }
  for (auto& e : energy_pair) {
    std::vector<zc> ph(e.size());
    for (size_t k = 0; k < e.size(); ++k) ph[k] = std::exp(zc(0.0, -p.J * p.dt * e[k]));
    p.pair_phase.push_back(ph);
  }
  // single-site gates
  for (int v = 0; v < 4; ++v) p.site_gate[v].assign(nb, {});
  p.zsum.assign(nb, {});
  for (int b = 0; b < nb; ++b) {
    int w = p.block_width[b], d = p.dim(b);
    auto xlayer = [&](double phi) {
      // Kronecker power of exp(-i phi X), first qubit most significant
      std::vector<zc> u(d * d);
      double c = std::cos(phi), s = std::sin(phi);
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          zc val(1.0, 0.0);
          for (int k = 0; k < w; ++k) {
            int bi = (i >> k) & 1, bj = (j >> k) & 1;
            val *= (bi == bj) ? zc(c, 0.0) : zc(0.0, -s);
          }
          u[i * d + j] = val;
        }
      return u;
    };
    std::vector<zc> dintra(d);
    for (int s = 0; s < d; ++s) dintra[s] = std::exp(zc(0.0, -p.J * p.dt * energy_intra[b][s]));
    auto full = xlayer(p.h * p.dt), half = xlayer(0.5 * p.h * p.dt);
    p.site_gate[0][b].resize(d * d);
    p.site_gate[1][b].resize(d * d);
    p.site_gate[2][b] = half;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        p.site_gate[0][b][i * d + j] = full[i * d + j] * dintra[j];  // U_X * D_intra
        p.site_gate[1][b][i * d + j] = dintra[i] * half[i * d + j];  // D_intra * U_X(half)
      }
    // XY preparation's last factor exp(-i pi/8 H_Z), H_Z = sum_j (-1)^j Z_j
    // (identity outside the XY model)
    p.site_gate[3][b].assign(d * d, zc(0.0, 0.0));
    for (int i = 0; i < d; ++i) {
      double hz = 0.0;
      if (p.model == 1) hz = p.stagger[b] * zval(i, w, 0);
      p.site_gate[3][b][i * d + i] = std::exp(zc(0.0, -0.125 * M_PI * hz));
    }
    p.zsum[b].resize(d);
    for (int s = 0; s < d; ++s) {
      double z = 0;
      for (int k = 0; k < w; ++k) z += zval(s, w, k);
      p.zsum[b][s] = z;
    }
  }
  // bond caps (valid for any block order): min(chi, dmax^p, dmax^(N-p))
  p.cap.assign(p.N + 1, 1);
  for (int b = 1; b < p.N; ++b) {
    double lim = std::min((double)p.chi, std::min(std::pow((double)p.dmax, b),
                                                   std::pow((double)p.dmax, p.N - b)));
    p.cap[b] = (int)lim;
  }
  // XY gates exp(-i phi (XX + YY)): XX + YY = 2 (|01><10| + |10><01|)
  if (p.model == 1) {
    long k = 0;
    double dtau = 0.0;
    if (p.theta0 != 0.0) {
      k = std::lround(std::fabs(p.J * p.theta0) / (0.02 * M_PI));
      if (k < 1) k = 1;
      dtau = p.theta0 / (double)k;
    }
    p.nprep = (int)k;
    p.dtau = dtau;
    const double phis[5] = {0.0, p.J * p.dt / 4, p.J * p.dt / 2, p.J * dtau / 4, p.J * dtau / 2};
    for (int v = 1; v <= 4; ++v) {
      const double c = std::cos(2 * phis[v]), sn = std::sin(2 * phis[v]);
      std::vector<zc> G(16, zc(0.0, 0.0));
      G[0] = G[15] = 1.0;
      G[5] = G[10] = c;
      G[6] = G[9] = zc(0.0, -sn);
      p.xy_gate[v] = G;
    }
  }
  // rank bound of each bond in the start order (blocks keep their sites
  // under schedule 4): the smaller product of local dimensions on its sides
  p.rank_cap.assign(p.N + 1, 1);
  for (int b = 1; b < p.N; ++b) {
    double left = 1, right = 1;
    for (int s = 0; s < b; ++s) left *= p.dim(p.snake_order[s]);
    for (int s = b; s < p.N; ++s) right *= p.dim(p.snake_order[s]);
    p.rank_cap[b] = (long)std::min(std::min(left, right), 1e15);
  }
  // bonds between the two blocks of a schedule-4 gate double before they
  // are truncated again
  p.xcap = p.cap;
  if (p.schedule == 4)
    for (int b = 1; b < p.N; ++b) p.xcap[b] = 2 * p.cap[b];
}

}  // namespace mpsim
