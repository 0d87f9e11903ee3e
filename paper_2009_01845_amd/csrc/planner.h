// Host-side circuit representation and pass planner (no HIP dependency).
#pragma once
#include <complex>
#include <string>
#include <vector>

#include "qs_types.h"

namespace qs {

using cd = std::complex<double>;

// A user gate in qubit terms (qubit q <-> index bit n-1-q).
struct Gate {
  int k = 0;
  int tq[5] = {0, 0, 0, 0, 0};
  std::vector<int> cq;
  bool is_rot = false;
  char pauli = 0;
  int pidx = -1;
  int rsign = 1;        // rotations: theta = rsign * params[pidx]
  std::vector<cd> mat;  // 2^k x 2^k row-major, MAT gates only
  // a diagonal exp(i scales[scale_slot] * E(x)) with E a polynomial owned by
  // the caller (adiabatic steps); k and the target list are unused
  const struct PhasePoly* spoly = nullptr;
  int scale_slot = -1;
};

struct TuneOpts {
  int tile_bits = 0;
  int fuse_k = 0;
  int use_mfma = -1;
  int low_bits = 0;
  int grid_bits = kGridBits;  // log2 of the workgroups walking a pass's tiles (0: one workgroup)
  bool force_stage = false;   // register-blocked stages also for tiles below 2^12
  bool lane_ops = false;      // one-qubit ops on lane bits inside register stages
};

enum PassKind : int { PASS_TILE = 1, PASS_PHASE = 2, PASS_PERM = 3, PASS_MFMA = 4, PASS_DENSE = 5 };

struct Pass {
  int kind = PASS_TILE;
  PassGeom geom{};
  std::vector<TileOp> ops;
  std::vector<int> sigma;  // PASS_PERM: data at bit a moves to bit sigma[a] (an involution)
  // staged passes whose forward stages hold lane ops: the same ops staged
  // without lane ops, for the two-state (adjoint) kernel
  bool has_adj = false;
  PassGeom geom_adj{};
  std::vector<TileOp> ops_adj;
  const PassGeom& adj_geom() const { return has_adj ? geom_adj : geom; }
  const std::vector<TileOp>& adj_ops() const { return has_adj ? ops_adj : ops; }
};

// Quadratic phase polynomial over global index bits.
struct PhasePoly {
  double c = 0.0;
  std::vector<double> mu;   // n
  std::vector<double> lam;  // n*n symmetric, zero diagonal
  bool empty = true;
  void init(int n) { mu.assign(n, 0.0); lam.assign(size_t(n) * n, 0.0); c = 0.0; empty = true; }
  // index bits that appear in a non-constant term
  uint64_t support() const {
    if (empty) return 0;
    const int n = (int)mu.size();
    uint64_t s = 0;
    for (int p = 0; p < n; ++p) {
      if (mu[p] != 0.0) s |= 1ull << p;
      for (int q = p + 1; q < n; ++q)
        if (lam[size_t(p) * n + q] != 0.0) s |= (1ull << p) | (1ull << q);
    }
    return s;
  }
};

struct Plan {
  int n = 0;
  bool dbl = false;  // state precision the tables were built for
  std::vector<Pass> passes;
  std::vector<cd> matpool;       // gate matrices
  std::vector<double> dpool;     // phase polynomials: c, mu[n], lam[n*n]
  std::vector<PhaseRec> phases;
  std::vector<cd> qtab;          // exp(i theta_T(j)) per phase op
  std::vector<double> qang;      // theta_T(j) per phase op (same offsets as qtab)
  std::vector<cd> ctab;          // per-thread-group phase factors of staged phase ops
  std::vector<StageRec> stages;  // staged passes
  std::vector<int32_t> phlist;   // staged passes: phase record of each per-pass phase slot
  std::vector<double> btab;      // staged passes: per-group phase constants (PhaseRec::bt_off)
  int nparams = 0;
  int ngates = 0;
  int ngrad_slots = 0;           // ops carrying a trainable parameter
  int grid_bits = kGridBits;
  bool force_stage = false;
  bool lane_ops = false;         // stages may hold lane ops (TuneOpts::lane_ops)
  int schedule = 0;              // high-bit choice that produced the plan: 0 index order,
                                 // 1 greedy lookahead, 2 one-step rollout
};

// Circuit description kept by the C ABI.
struct HostCircuit {
  int n = 0;
  std::vector<Gate> gates;
  int nparams = 0;
  TuneOpts opts;
  const PhasePoly* tail_phase = nullptr;  // appended with scale slot 0 (adiabatic steps)
  bool compiled = false;
  Plan plan;
};

// Validation used by the ABI (returns empty string when fine).
std::string validate_gate(int n, int k, const int* targets, int nctrl, const int* controls);

// Plan a circuit for a state of the given precision.  Throws std::runtime_error.
Plan plan_circuit(const HostCircuit& c, const TuneOpts& opts, bool dbl);

// Default tile geometry for n qubits and a precision.
void default_tile(int n, bool dbl, const TuneOpts& o, int* m, int* L);

// Build an OP_PHASE op (and its tables) for a pass geometry.  scale_idx >= 0
// multiplies theta by scales[scale_idx] at run time.
TileOp make_phase_op(Plan& plan, const PassGeom& g, const PhasePoly& P, int scale_idx);
// Ising energy E(z) as a polynomial in the index bits.
PhasePoly ising_poly(int n, const double* J, const double* h);
// `steps` Trotter steps in one plan: for s = 0..steps-1, RX(params[s]) on every
// qubit then exp(i scales[s] E(x)); consecutive steps share passes.  With
// final_layer, RX(params[steps]) on every qubit closes the plan.
Plan plan_trotter(int n, bool dbl, const TuneOpts& opts, const PhasePoly* poly, int steps,
                  bool final_layer = false);

// The op records of staged passes (StagedOp), one per op of `ops`, whose phase
// ops index `phases` (the plan's phase records).  Ops of other passes get
// records with opc = -1 and no gradient.
std::vector<StagedOp> staged_records(const std::vector<TileOp>& ops, const std::vector<PhaseRec>& phases);
// Greedy fusion of consecutive fixed gates into blocks of at most K qubits.
std::vector<Gate> fuse_gates(const std::vector<Gate>& in, int K);

// Named gate matrices (row-major complex); returns k or 0 for an unknown name.
int named_gate(const std::string& name, double theta, std::vector<cd>& out);

}  // namespace qs
