// Host-side planning of a block-MPS instance: lattice geometry (a grid with
// half-row blocks, or a cube with one qubit per site), snake order, the
// two-site update schedule, gate tables and buffer sizes.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

#include "../../include/mpsim.h"

namespace mpsim {

typedef std::complex<double> zc;

struct Op {          // one entry of the step schedule
  int kind;          // 1 = two-site update, 2 = single-site gate, 3 = ZZ gate as a rank-2 MPO
  int site;
  int swap;          // kind 1
  int gate;          // kind 1: block-pair phase applied
  int variant;       // kind 2
  int block_a, block_b;  // blocks at site, site+1 before the op (kind 1); block (kind 2)
  int site_b, bit_a, bit_b;  // kind 3: sites site < site_b, bit of each block's fused index
};

struct Plan {
  int R = 0, C = 0, n = 0, N = 0;  // grid, qubits, sites
  int Lz = 0;                      // cube depth (0: two-dimensional grid)
  int nb = 0;                      // blocks
  std::vector<int> snake_order;    // block held by each site at the start
  int chi = 0, order = 1, periodic = 1, schedule = 1, eig_path = 0;
  int eig_batch = 1024;            // vectors per band inverse-iteration launch
  double J = 0, h = 0, dt = 0, theta0 = 0;
  int wL = 0, wR = 0, dmax = 1;
  std::vector<int> block_width;               // per block id
  std::vector<int> cap;                       // bond caps b_0..b_N
  std::vector<int> xcap;                      // transient caps: 2 cap inside the chain for schedule 4
  std::vector<long> rank_cap;                 // smaller Hilbert-space dimension on either side of a bond
  std::vector<std::vector<int>> block_qubits; // per block, in column order
  std::vector<std::pair<int, int>> bonds;     // ZZ bonds (q1 < q2), each once

  // gate tables: pair index of ordered (a, b) with a < b; -1 = not coupled
  std::vector<int> pair_index;                // [a * nblocks + b]
  std::vector<std::vector<zc>> pair_phase;    // [pair] d_a x d_b, row-major
  std::vector<std::vector<zc>> site_gate[4];  // [variant][block] d x d (3: XY staggered Z phase)
  // XY model (model 1): sublayers A, B, C, D of bonds (qubit pairs), the
  // dense two-qubit gates exp(-i phi (XX + YY)) (row-major 4 x 4; variant
  // 1 / 2: half / full step dt, 3 / 4: half / full preparation step dtau),
  // the checkerboard sign of every qubit and the preparation step count
  int model = 0;
  std::vector<std::vector<std::pair<int, int>>> xy_sub;
  std::vector<zc> xy_gate[5];
  std::vector<int> stagger;
  int nprep = 0;
  double dtau = 0.0;
  std::vector<std::vector<double>> zsum;      // [block] d entries

  int nblocks() const { return nb; }
  int dim(int block) const { return 1 << block_width[block]; }
  int coupled(int a, int b) const {
    if (a == b) return -1;
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return pair_index[lo * nblocks() + hi];
  }
  std::vector<int> snake() const;
  // ops of one step from order `pos`; pos is updated to the end order
  void step_ops(std::vector<int>& pos, std::vector<Op>& out) const;
  // XY model: ops of one step (prep: with the preparation step's gates)
  void xy_ops(std::vector<int>& pos, std::vector<Op>& out, bool prep) const;
};

// Validate a config; returns MPS_OK or an error code with a message.
mps_status validate(const mps_config* cfg, const char** msg);
// Build the plan (geometry, tables, caps) for a validated config.
void build_plan(const mps_config* cfg, Plan& p);

}  // namespace mpsim
