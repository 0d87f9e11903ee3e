// Host pass planner: turns a gate queue into a short list of passes over the
// state (paper Sec. 2.4.5 fuses gates into at most 4x4 matrices; here every
// gate whose targets fit one on-chip tile shares a single HBM read+write).
//
//  1. SWAP gates become a relabelling of qubits to index bits; the data is
//     moved once at the end by at most two involutive bit-permutation passes.
//  2. Diagonal gates with unit-modulus entries on at most two index bits
//     (Z, S, T, RZ, U1, CZ, CU1 -- the paper's sparse gates, Sec. 2.3) are
//     collected into a quadratic phase polynomial theta(x) that is applied
//     element-wise, deferred until a non-diagonal gate touches one of its bits.
//  3. The other gates are scheduled greedily, in dependency order, into tiled
//     passes: the tile bit set T = {0..L-1} U (up to m-L high bits); a gate
//     joins the open pass when its targets fit in T.  The high bits are those
//     the first gates in index order ask for, or are picked ahead by how many
//     gates they unlock (two ways); the plan with the fewest passes is kept.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <stdexcept>

namespace qs {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;
constexpr int kRolloutMaxGates = 6000;  // longer gate lists skip the rollout schedule
constexpr int kRolloutMaxFront = 48;    // first choices tried per pass by the rollout
constexpr int kMaxHighBits = 7;         // a tile holds at most 2^7 rows

bool is_diag(const std::vector<cd>& m, int dim) {
  for (int r = 0; r < dim; ++r)
    for (int c = 0; c < dim; ++c)
      if (r != c && m[size_t(r) * dim + c] != cd(0, 0)) return false;
  return true;
}

bool is_swap(const std::vector<cd>& m) {
  static const int one[4][4] = {{1, 0, 0, 0}, {0, 0, 1, 0}, {0, 1, 0, 0}, {0, 0, 0, 1}};
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      if (m[r * 4 + c] != cd(one[r][c], 0)) return false;
  return true;
}

std::vector<cd> matmul(const std::vector<cd>& a, const std::vector<cd>& b, int dim) {
  std::vector<cd> o(size_t(dim) * dim, cd(0, 0));
  for (int i = 0; i < dim; ++i)
    for (int k = 0; k < dim; ++k) {
      cd v = a[size_t(i) * dim + k];
      if (v == cd(0, 0)) continue;
      for (int j = 0; j < dim; ++j) o[size_t(i) * dim + j] += v * b[size_t(k) * dim + j];
    }
  return o;
}

std::vector<cd> dagger(const std::vector<cd>& a, int dim) {
  std::vector<cd> o(size_t(dim) * dim);
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) o[size_t(j) * dim + i] = std::conj(a[size_t(i) * dim + j]);
  return o;
}

enum BKind { BK_DENSE = 0, BK_ROT = 1, BK_PHASE = 2, BK_SPHASE = 3 };

struct Term {  // theta contribution: ang * x_p * x_q (p == q: linear)
  int p, q;
  double ang;
};

struct BitGate {
  int kind = BK_DENSE;
  int k = 0;
  int tb[5] = {0, 0, 0, 0, 0};
  uint64_t cmask = 0;
  std::vector<cd> mat;
  char pauli = 0;
  int pidx = -1;
  int rsign = 1;
  double cphase = 0.0;
  std::vector<Term> terms;
  uint64_t nmask = 0;  // bits where the gate is not diagonal
  uint64_t dmask = 0;  // bits where it is diagonal (controls, diagonal targets)
  bool mfma = false;   // applied as a dense block on matrix cores (own pass)
  const PhasePoly* spoly = nullptr;  // BK_SPHASE: run-time scaled phase
  int scale_slot = -1;
};

// Pending op inside an open pass, in global bit terms.
struct RawOp {
  int kind;  // OP_*
  BitGate g;
  PhasePoly poly;  // OP_PHASE
  int scale_idx = -1;
};

}  // namespace

std::string validate_gate(int n, int k, const int* targets, int nctrl, const int* controls) {
  if (k < 1 || k > 5) return "number of targets must be in [1, 5]";
  if (nctrl < 0) return "negative number of controls";
  if (k + nctrl > n) return "targets + controls exceed the number of qubits";
  if (!targets) return "null targets";
  if (nctrl > 0 && !controls) return "null controls";
  uint64_t seen = 0;
  for (int i = 0; i < k + nctrl; ++i) {
    int q = i < k ? targets[i] : controls[i - k];
    if (q < 0 || q >= n) return "qubit index out of range";
    if ((seen >> q) & 1) return "duplicate qubit among targets and controls";
    seen |= 1ull << q;
  }
  return "";
}

int named_gate(const std::string& name, double theta, std::vector<cd>& out) {
  const double c = std::cos(theta / 2), s = std::sin(theta / 2);
  const double r2 = 1.0 / std::sqrt(2.0);
  const cd I(0, 1);
  if (name == "H") { out = {r2, r2, r2, -r2}; return 1; }
  if (name == "X") { out = {0.0, 1.0, 1.0, 0.0}; return 1; }
  if (name == "Y") { out = {0.0, -I, I, 0.0}; return 1; }
  if (name == "Z") { out = {1.0, 0.0, 0.0, -1.0}; return 1; }
  if (name == "S") { out = {1.0, 0.0, 0.0, I}; return 1; }
  if (name == "T") { out = {1.0, 0.0, 0.0, std::polar(1.0, M_PI / 4)}; return 1; }
  if (name == "RX") { out = {c, -I * s, -I * s, c}; return 1; }
  if (name == "RY") { out = {c, -s, s, c}; return 1; }
  if (name == "RZ") { out = {std::polar(1.0, -theta / 2), 0.0, 0.0, std::polar(1.0, theta / 2)}; return 1; }
  if (name == "U1") { out = {1.0, 0.0, 0.0, std::polar(1.0, theta)}; return 1; }
  if (name == "SWAP") {
    out.assign(16, 0.0);
    out[0] = out[6] = out[9] = out[15] = 1.0;
    return 2;
  }
  return 0;
}

void default_tile(int n, bool dbl, const TuneOpts& o, int* m, int* L) {
  int mm = o.tile_bits > 0 ? o.tile_bits : 12;
  int ll = o.low_bits > 0 ? o.low_bits : (dbl ? 5 : 6);
  mm = std::min(mm, dbl ? 12 : 13);  // <= 64 KiB of LDS per workgroup
  mm = std::max(mm, 6);
  if (mm > n) mm = n;
  if (ll > mm) ll = mm;
  if (mm < n && mm - ll < 5) ll = std::max(1, mm - 5);  // room for a 5-qubit gate
  if (mm - ll > kMaxHighBits) ll = mm - kMaxHighBits;    // at most 2^7 rows per tile
  if (ll > 8) ll = 8;
  *m = mm;
  *L = ll;
}

namespace {

// (I - Pc) (x) I + Pc (x) G on (controls..., targets...): a controlled gate as
// one dense matrix, controls as the most significant index bits
std::vector<cd> expand_controls(const std::vector<cd>& G, int k, int nc) {
  const int dk = 1 << k, dt = 1 << (k + nc);
  std::vector<cd> M(size_t(dt) * dt, cd(0, 0));
  for (int i = 0; i < dt; ++i) M[size_t(i) * dt + i] = 1.0;
  const int c1 = ((1 << nc) - 1) << k;  // all controls 1
  for (int r = 0; r < dk; ++r)
    for (int c = 0; c < dk; ++c) M[size_t(c1 | r) * dt + (c1 | c)] = G[size_t(r) * dk + c];
  return M;
}

// Convert a user gate to index bits under the current relabelling.
BitGate to_bits(const Gate& g, int n, const std::vector<int>& phys, const TuneOpts& opts) {
  BitGate b;
  if (g.spoly) {  // diagonal on every bit of its polynomial (index bits already)
    b.kind = BK_SPHASE;
    b.spoly = g.spoly;
    b.scale_slot = g.scale_slot;
    b.dmask = g.spoly->support();
    if (!b.dmask) b.dmask = 1;  // a constant still orders against nothing but keeps a bit
    return b;
  }
  b.k = g.k;
  for (int i = 0; i < g.k; ++i) b.tb[i] = phys[g.tq[i]];
  for (int q : g.cq) b.cmask |= 1ull << phys[q];
  b.dmask = b.cmask;
  if (g.is_rot) {
    b.kind = BK_ROT;
    b.pauli = g.pauli;
    b.pidx = g.pidx;
    b.rsign = g.rsign;
    if (g.pauli == 'Z') b.dmask |= 1ull << b.tb[0];
    else b.nmask |= 1ull << b.tb[0];
    return b;
  }
  const int dim = 1 << g.k;
  b.mat = g.mat;
  const bool diag = is_diag(g.mat, dim);
  uint64_t tmask = 0;
  for (int i = 0; i < g.k; ++i) tmask |= 1ull << b.tb[i];
  if (!diag) {
    b.kind = BK_DENSE;
    b.nmask = tmask;
    const int kt = g.k + (int)g.cq.size();
    const int kmin = opts.use_mfma > 0 ? 3 : 4;
    if (opts.use_mfma != 0 && kt >= kmin && kt <= 5 && n >= std::max(kt, 4) + 7) {
      // the whole controlled gate becomes one dense block on matrix cores
      b.mfma = true;
      if (!g.cq.empty()) {
        b.mat = expand_controls(g.mat, g.k, (int)g.cq.size());
        int t = 0;
        for (int q : g.cq) b.tb[t++] = phys[q];
        for (int i = 0; i < g.k; ++i) b.tb[t++] = phys[g.tq[i]];
        b.k = kt;
        b.nmask = b.cmask | tmask;
        b.dmask = 0;
        b.cmask = 0;
      }
      if (b.k == 3) {
        // the matrix-core kernel takes 4- and 5-qubit blocks: widen to G (x) I
        // with the lowest free index bit as the new least significant target
        uint64_t used = 0;
        for (int t = 0; t < 3; ++t) used |= 1ull << b.tb[t];
        const int e = __builtin_ctzll(~used);
        std::vector<cd> M(256, cd(0, 0));
        for (int r = 0; r < 8; ++r)
          for (int c = 0; c < 8; ++c)
            for (int a = 0; a < 2; ++a) M[size_t((r << 1) | a) * 16 + ((c << 1) | a)] = b.mat[size_t(r) * 8 + c];
        b.mat = M;
        b.tb[3] = e;
        b.k = 4;
        b.nmask |= 1ull << e;
      }
    }
    return b;
  }
  b.dmask |= tmask;
  bool unit = true;
  for (int i = 0; i < dim; ++i)
    if (std::abs(std::abs(g.mat[size_t(i) * dim + i]) - 1.0) > 1e-12) unit = false;
  const int nc = (int)g.cq.size();
  if (!unit || g.k + nc > 2) {
    b.kind = BK_DENSE;  // diagonal but not a quadratic phase: applied as a tile op
    return b;
  }
  b.kind = BK_PHASE;
  auto arg = [&](int i) { return std::arg(g.mat[size_t(i) * dim + i]); };
  if (g.k == 1 && nc == 0) {
    int a = b.tb[0];
    b.cphase += arg(0);
    b.terms.push_back({a, a, arg(1) - arg(0)});
  } else if (g.k == 1 && nc == 1) {
    int a = b.tb[0], cb = __builtin_ctzll(b.cmask);
    b.terms.push_back({cb, cb, arg(0)});
    b.terms.push_back({std::min(a, cb), std::max(a, cb), arg(1) - arg(0)});
  } else {  // k == 2, no controls; matrix index = 2*x_a + x_b
    int a = b.tb[0], bb = b.tb[1];
    b.cphase += arg(0);
    b.terms.push_back({a, a, arg(2) - arg(0)});
    b.terms.push_back({bb, bb, arg(1) - arg(0)});
    b.terms.push_back({std::min(a, bb), std::max(a, bb), arg(3) - arg(2) - arg(1) + arg(0)});
  }
  return b;
}

void add_terms(PhasePoly& P, int n, const BitGate& g) {
  P.c += g.cphase;
  for (const Term& t : g.terms) {
    if (t.ang == 0.0) continue;
    if (t.p == t.q) P.mu[t.p] += t.ang;
    else {
      P.lam[size_t(t.p) * n + t.q] += t.ang;
      P.lam[size_t(t.q) * n + t.p] += t.ang;
    }
    P.empty = false;
  }
  if (g.cphase != 0.0) P.empty = false;
}

// Move the terms of P that touch any bit of mask into a new polynomial.
PhasePoly extract_terms(PhasePoly& P, int n, uint64_t mask, bool with_const) {
  PhasePoly Q;
  Q.init(n);
  if (P.empty) return Q;
  for (int p = 0; p < n; ++p) {
    if (!((mask >> p) & 1)) continue;
    if (P.mu[p] != 0.0) { Q.mu[p] = P.mu[p]; P.mu[p] = 0.0; Q.empty = false; }
    for (int q = 0; q < n; ++q) {
      double v = P.lam[size_t(p) * n + q];
      if (v != 0.0) {
        Q.lam[size_t(p) * n + q] = v;
        Q.lam[size_t(q) * n + p] = v;
        P.lam[size_t(p) * n + q] = 0.0;
        P.lam[size_t(q) * n + p] = 0.0;
        Q.empty = false;
      }
    }
  }
  if (with_const && P.c != 0.0) { Q.c = P.c; P.c = 0.0; Q.empty = false; }
  bool any = P.c != 0.0;
  for (double v : P.mu) any |= v != 0.0;
  if (!any)
    for (double v : P.lam) if (v != 0.0) { any = true; break; }
  P.empty = !any;
  return Q;
}

double wrap_angle(double a) { return a - kTwoPi * std::nearbyint(a / kTwoPi); }

}  // namespace

TileOp make_phase_op(Plan& plan, const PassGeom& g, const PhasePoly& P, int scale_idx) {
  const int n = g.n;
  int pos[kMaxTileBits];
  for (int b = 0; b < g.L; ++b) pos[b] = b;
  for (int j = 0; j < g.H; ++j) pos[g.L + j] = g.hbits[j];
  TileOp op;
  std::memset(&op, 0, sizeof(op));
  op.kind = OP_PHASE;
  op.mat = -1;
  op.pidx = -1;
  op.gslot = -1;
  op.sign = 1;
  PhaseRec rec;
  rec.dpool = (int)plan.dpool.size();
  plan.dpool.push_back(P.c);
  plan.dpool.insert(plan.dpool.end(), P.mu.begin(), P.mu.end());
  plan.dpool.insert(plan.dpool.end(), P.lam.begin(), P.lam.end());
  rec.qtab_off = (int)plan.qtab.size();
  rec.scale_idx = scale_idx;
  rec.wr_off = -1;
  rec.bt_off = -1;
  rec.wr_trivial = 0;
  rec.kt_off = -1;
  rec.wr_sign = 0;
  rec.ctab_off = -1;
  rec.ctab_n = 0;
  const int M = 1 << g.m;
  std::vector<double> ang(M, 0.0);
  for (int j = 1; j < M; ++j) {  // ang[j] = ang[j without its top bit] + the top bit's terms
    const int top = 31 - __builtin_clz((unsigned)j);
    const int rest = j & ~(1 << top);
    const int pt = pos[top];
    double a = ang[rest] + P.mu[pt];
    for (int r2 = rest; r2; r2 &= r2 - 1) a += P.lam[size_t(pt) * n + pos[__builtin_ctz((unsigned)r2)]];
    ang[j] = a;
  }
  for (int j = 0; j < M; ++j) {
    // unscaled tables are exact phases; scaled ones keep the raw angle
    const double a = scale_idx < 0 ? wrap_angle(ang[j]) : ang[j];
    plan.qtab.push_back(std::polar(1.0, a));
    plan.qang.push_back(a);
  }
  op.aux = (int)plan.phases.size();
  plan.phases.push_back(rec);
  return op;
}

PhasePoly ising_poly(int n, const double* J, const double* h) {
  // E(z) = sum_{i<j} J_ij z_i z_j + sum_i h_i z_i with z = 1 - 2 x, x the bit
  // of qubit q at index position n-1-q
  PhasePoly P;
  P.init(n);
  for (int i = 0; i < n; ++i) {
    const int a = n - 1 - i;
    P.c += h[i];
    P.mu[a] += -2.0 * h[i];
    for (int j = i + 1; j < n; ++j) {
      const double v = J[size_t(i) * n + j];
      if (v == 0.0) continue;
      const int b = n - 1 - j;
      P.c += v;
      P.mu[a] += -2.0 * v;
      P.mu[b] += -2.0 * v;
      P.lam[size_t(a) * n + b] += 4.0 * v;
      P.lam[size_t(b) * n + a] += 4.0 * v;
    }
  }
  P.empty = false;
  return P;
}

namespace {

int nphase_raw(const std::vector<RawOp>& raw) {
  int c = 0;
  for (const RawOp& r : raw) c += r.kind == OP_PHASE;
  return c;
}

int ngrad_raw(const std::vector<RawOp>& raw) {
  int c = 0;
  for (const RawOp& r : raw) c += r.kind == OP_ROT && r.g.pidx >= 0;
  return c;
}

bool has(const std::vector<int>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); }

// Register-blocked form of a pass (tiles of >= 2^12 amplitudes): split its op
// list into stages whose dense targets all lie in kRegBits tile bits (and,
// with lanes, one-qubit ops on the lane bits), and rewrite the ops in
// register-slot terms.
void stage_ops(Plan& plan, PassGeom& g, std::vector<TileOp>& pops, bool lanes, bool* used_lanes) {
  struct {
    std::vector<TileOp>& ops;
  } ps{pops};
  if (used_lanes) *used_lanes = false;
  g.kern = 1;
  g.st0 = g.nst = g.ph0 = g.nph = 0;
  g.ctrl = 0;
  if (g.m < (plan.force_stage ? kRegBits + 1 : 12)) return;
  int nph = 0;
  for (const TileOp& op : ps.ops) {
    if (op.kind == OP_DENSEK) return;  // k >= 3 matrices keep the one-sweep-per-op kernel
    if (op.kind == OP_PHASE) ++nph;
  }
  if (nph > kMaxPhasePerPass) return;
  const int n = g.n;
  auto pos = [&](int local) { return local < g.L ? local : g.hbits[local - g.L]; };
  auto targets = [](const TileOp& op) {
    std::vector<int> s;
    const int k = (op.kind == OP_DENSE1 || op.kind == OP_ROT) ? 1
                  : op.kind == OP_DENSE2                     ? 2
                  : op.kind == OP_DENSEK                     ? op.k
                                                             : 0;
    for (int t = 0; t < k; ++t) s.push_back(op.b[t]);
    return s;
  };
  struct St {
    std::vector<int> rb;
    std::vector<TileOp> ops;
  };
  // Ops that commute may run in any order: pack them into as few register
  // stages as the dependencies allow.  Per op: the tile bits it changes
  // non-diagonally, the bits it only reads or multiplies by a phase
  // (controls, diagonal targets, a phase polynomial's support) and the bits
  // it needs in register slots.  Two ops depend on each other when one
  // changes a bit non-diagonally that the other touches.
  const int N = (int)ps.ops.size();
  std::vector<uint32_t> nd(N, 0), dg(N, 0), tm(N, 0);
  for (int i = 0; i < N; ++i) {
    const TileOp& op = ps.ops[i];
    uint32_t t = 0;
    for (int b : targets(op)) t |= 1u << b;
    tm[i] = t;
    dg[i] = op.cin;
    bool diagonal = op.kind == OP_ROT && op.pauli == 3;
    if (op.kind == OP_DENSE1) {
      const cd* M = plan.matpool.data() + op.mat;
      diagonal = M[1] == 0.0 && M[2] == 0.0 && M[5] == 0.0 && M[6] == 0.0;
    }
    if (op.kind != OP_DENSE1 && op.kind != OP_DENSE2 && op.kind != OP_ROT && op.kind != OP_PHASE) {
      nd[i] = (1u << g.m) - 1u;  // not modelled: ordered against every op
    } else if (op.kind == OP_PHASE) {
      const double* P = plan.dpool.data() + plan.phases[op.aux].dpool;
      for (int b = 0; b < g.m; ++b) {
        const int q = pos(b);
        bool on = P[1 + q] != 0.0;
        for (int r = 0; r < n && !on; ++r) on = P[1 + n + size_t(q) * n + r] != 0.0 || P[1 + n + size_t(r) * n + q] != 0.0;
        if (on) dg[i] |= 1u << b;
      }
    } else if (diagonal) {
      dg[i] |= t;
    } else {
      nd[i] = t;
    }
  }
  std::vector<std::vector<int>> pred(N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < i; ++j)
      if ((nd[j] & (nd[i] | dg[i])) || (nd[i] & (nd[j] | dg[j]))) pred[i].push_back(j);
  std::vector<char> done(N, 0);
  auto ready = [&](int i) {
    if (done[i]) return false;
    for (int j : pred[i])
      if (!done[j]) return false;
    return true;
  };
  std::vector<St> sts;
  int left = N;
  while (left > 0) {
    St cur;
    uint32_t mask = 0;
    auto take = [&](int i) {
      for (int b : targets(ps.ops[i]))
        if (!has(cur.rb, b)) cur.rb.push_back(b);
      mask |= tm[i];
      cur.ops.push_back(ps.ops[i]);
      done[i] = 1;
      --left;
    };
    for (;;) {
      bool grew = false;
      for (int i = 0; i < N; ++i)  // every ready op that needs no new register bit, in order
        if (ready(i) && (tm[i] & ~mask) == 0) {
          take(i);
          grew = true;
        }
      if (grew) continue;
      int best = -1, bestnew = kRegBits + 1;  // else the ready op adding the fewest bits
      for (int i = 0; i < N; ++i)
        if (ready(i) && __builtin_popcount(mask | tm[i]) <= kRegBits) {
          const int nb = __builtin_popcount(tm[i] & ~mask);
          if (nb < bestnew) {
            bestnew = nb;
            best = i;
          }
        }
      if (best < 0) break;
      take(best);
    }
    // lane ops: with the register set fixed (padded with the lowest free
    // bits), uncontrolled one-qubit ops on the lowest non-register tile bits
    // run in the same stage across lanes of a row (the group index's bits
    // 0..3 are lane bits; a small tile has 2^(m-4) groups, so only bits whose
    // partner group exists qualify)
    {
      for (int b = 0; (int)cur.rb.size() < kRegBits; ++b)
        if (!has(cur.rb, b)) cur.rb.push_back(b);
      uint32_t rmask = 0;
      for (int b : cur.rb) rmask |= 1u << b;
      const int nlane = lanes ? std::min(4, g.m - kRegBits) : 0;
      uint32_t lmask = 0;
      for (int b = 0, j = 0; b < g.m && j < nlane; ++b)
        if (!((rmask >> b) & 1)) {
          lmask |= 1u << b;
          ++j;
        }
      for (bool grew = true; grew;) {
        grew = false;
        for (int i = 0; i < N; ++i) {
          if (!ready(i)) continue;
          const TileOp& op = ps.ops[i];
          const bool fits = (tm[i] & ~rmask) == 0;
          const bool lane = (op.kind == OP_DENSE1 || op.kind == OP_ROT) && op.cin == 0 && (tm[i] & ~lmask) == 0;
          if (fits || lane) {
            cur.ops.push_back(op);
            done[i] = 1;
            --left;
            grew = true;
          }
        }
      }
    }
    if (cur.ops.empty()) throw std::runtime_error("planner: no op fits a register stage");
    sts.push_back(cur);
  }

  std::vector<TileOp> out;
  g.st0 = (int)plan.stages.size();
  g.ph0 = (int)plan.phlist.size();
  g.nph = 0;
  for (St& s : sts) {
    for (int b = 0; (int)s.rb.size() < kRegBits; ++b)
      if (!has(s.rb, b)) s.rb.push_back(b);
    StageRec sr;
    std::memset(&sr, 0, sizeof(sr));
    int slot_of[kMaxTileBits];
    for (int b = 0; b < kMaxTileBits; ++b) slot_of[b] = -1;
    for (int k = 0; k < kRegBits; ++k) {
      sr.rb[k] = s.rb[k];
      sr.rbmask |= 1u << s.rb[k];
      slot_of[s.rb[k]] = k;
    }
    sr.op0 = (int)out.size();
    sr.nops = (int)s.ops.size();
    for (TileOp op : s.ops) {
      const uint32_t cin = op.cin;
      op.cin = 0;
      op.creg = 0;
      for (uint32_t c = cin; c; c &= c - 1) {
        const int b = __builtin_ctz(c);
        if (slot_of[b] >= 0) op.creg |= 1u << slot_of[b];
        else op.cin |= 1u << b;
      }
      const int dim = op.kind == OP_DENSE1 ? 2 : op.kind == OP_DENSE2 ? 4 : op.kind == OP_DENSEK ? (1 << op.k) : 0;
      int lane_j = -1;  // lane op: index of its bit among the non-register tile bits
      if ((op.kind == OP_DENSE1 || op.kind == OP_ROT) && slot_of[op.b[0]] < 0) {
        lane_j = 0;
        for (int b = 0; b < op.b[0]; ++b)
          if (!((sr.rbmask >> b) & 1)) ++lane_j;
        if (lane_j > 3 || cin != 0) throw std::runtime_error("planner: lane op outside the lane bits");
      }
      if (op.kind == OP_DENSE1 || op.kind == OP_ROT) {
        op.b[0] = lane_j >= 0 ? lane_j : slot_of[op.b[0]];
      } else if (op.kind == OP_DENSE2) {
        int s0 = slot_of[op.b[0]], s1 = slot_of[op.b[1]];
        if (s0 < s1) {  // make the higher slot the matrix MSB: swap the two index bits
          static const int pm[4] = {0, 2, 1, 3};
          for (int w = 0; w < 2; ++w) {
            cd* M = plan.matpool.data() + op.mat + w * 16;
            cd T[16];
            for (int r = 0; r < 4; ++r)
              for (int c = 0; c < 4; ++c) T[r * 4 + c] = M[pm[r] * 4 + pm[c]];
            std::copy(T, T + 16, M);
          }
          std::swap(s0, s1);
        }
        op.b[0] = s0;
        op.b[1] = s1;
      } else if (op.kind == OP_DENSEK) {
        for (int t = 0; t < op.k; ++t) op.b[t] = slot_of[op.b[t]];
      } else if (op.kind == OP_PHASE) {
        PhaseRec& rec = plan.phases[op.aux];
        op.pidx = g.nph++;
        plan.phlist.push_back(op.aux);
        rec.wr_off = (int)plan.qtab.size();
        const double* mu = plan.dpool.data() + rec.dpool + 1;
        const double* lam = mu + n;
        bool trivial = true;
        for (int e = 0; e < (1 << kRegBits); ++e) {
          double q = 0.0;
          for (int k = 0; k < kRegBits; ++k)
            for (int k2 = k + 1; k2 < kRegBits; ++k2)
              if (((e >> k) & 1) && ((e >> k2) & 1)) q += lam[size_t(pos(s.rb[k])) * n + pos(s.rb[k2])];
          trivial &= q == 0.0;
          plan.qtab.push_back(std::polar(1.0, rec.scale_idx < 0 ? wrap_angle(q) : q));
          plan.qang.push_back(rec.scale_idx < 0 ? wrap_angle(q) : q);
        }
        rec.wr_trivial = trivial ? 1 : 0;
        // a fixed phase whose coefficients are all multiples of pi (CZ, Z and
        // CZ-layer terms) only flips signs: keep the parity of Q_R(e)
        rec.wr_sign = 0;
        if (rec.scale_idx < 0) {
          auto pi_mult = [](double v) {
            const double r = v / kPi;
            return std::fabs(r - std::nearbyint(r)) < 1e-9;
          };
          bool sign = pi_mult(plan.dpool[rec.dpool]);
          for (int p2 = 0; p2 < n && sign; ++p2) {
            sign &= pi_mult(mu[p2]);
            for (int q2 = p2 + 1; q2 < n && sign; ++q2) sign &= pi_mult(lam[size_t(p2) * n + q2]);
          }
          if (sign) {
            op.flags |= 4u;
            for (int e = 0; e < (1 << kRegBits); ++e)
              if ((long long)std::llround(plan.qang[rec.wr_off + e] / kPi) & 1) rec.wr_sign |= 1 << e;
          }
        }
        // does every term of theta contain one register bit (a phase that is
        // 1 wherever that bit is 0)?
        for (int k = 0; k < kRegBits && !(op.flags & 2u); ++k) {
          const int qb = pos(s.rb[k]);
          bool one = plan.dpool[rec.dpool] == 0.0;
          for (int p2 = 0; p2 < n && one; ++p2) {
            if (p2 != qb && mu[p2] != 0.0) one = false;
            for (int q2 = 0; q2 < n && one; ++q2)
              if (p2 != qb && q2 != qb && lam[size_t(p2) * n + q2] != 0.0) one = false;
          }
          if (one) {
            op.flags |= 2u;
            op.b[0] = k;
          }
        }
        // per thread group jg (register bits zero): theta_T(jg) and, for each
        // register slot k, mu_k + sum_{a in jg} lam_{a,k}
        // a workgroup visits tiles t = t0 + kk * G (G = 2^gb workgroups); the
        // staged kernel places the gb grid bits of t at the highest non-tile
        // index positions and the k bits (kk) at the lowest ones, kp[j]
        {
          const int ntb = n - g.m;
          const int gb = std::min(ntb, plan.grid_bits);
          const int kb = ntb - gb;
          if (kb > kMaxKBits) throw std::runtime_error("planner: too many tile-index bits");
          std::vector<int> kp;
          int idx = 0;
          for (int q = 0; q < n; ++q) {
            bool tile = q < g.L;
            for (int h = 0; h < g.H; ++h) tile |= g.hbits[h] == q;
            if (tile) continue;
            if (idx < kb) kp.push_back(q);
            ++idx;
          }
          rec.kt_off = (int)plan.btab.size();
          for (int b = 0; b < g.m; ++b)
            for (int j = 0; j < kMaxKBits; ++j) plan.btab.push_back(j < kb ? lam[size_t(pos(b)) * n + kp[j]] : 0.0);
          for (int kk = 0; kk < (1 << kb); ++kk) {
            double q = 0.0;
            for (int j = 0; j < kb; ++j)
              for (int j2 = j + 1; j2 < kb; ++j2)
                if (((kk >> j) & 1) && ((kk >> j2) & 1)) q += lam[size_t(kp[j]) * n + kp[j2]];
            plan.btab.push_back(q);
          }
        }
        const int ngr = 1 << (g.m - kRegBits);
        std::vector<double> ang;  // per group: theta_T(jg), beta_0..beta_3
        ang.reserve(size_t(ngr) * (kRegBits + 1));
        for (int grp = 0; grp < ngr; ++grp) {
          uint32_t jg = (uint32_t)grp;
          for (int k2 = 0; k2 < g.m; ++k2)  // insert zeros at the register bits, ascending
            if ((sr.rbmask >> k2) & 1) jg = ((jg >> k2) << (k2 + 1)) | (jg & ((1u << k2) - 1u));
          ang.push_back(plan.qang[rec.qtab_off + jg]);
          for (int k = 0; k < kRegBits; ++k) {
            const int pk = pos(s.rb[k]);
            double b = mu[pk];
            for (uint32_t r = jg; r; r &= r - 1) b += lam[size_t(pos(__builtin_ctz(r))) * n + pk];
            ang.push_back(b);
          }
        }
        rec.bt_off = (int)plan.btab.size();
        rec.ctab_off = (int)plan.ctab.size();
        if (op.flags & 4u) {
          // sign op: only the parity of each angle / pi matters.  Bit-sliced,
          // slice s (theta_T, beta_0..beta_3) holds one bit per group, 64
          // groups a word, so a wave fetches its bits with scalar loads
          const int nw = (ngr + 63) / 64;
          std::vector<uint64_t> words(size_t(kRegBits + 1) * nw, 0);
          for (int grp = 0; grp < ngr; ++grp)
            for (int sl = 0; sl <= kRegBits; ++sl)
              if (std::llround(ang[size_t(grp) * (kRegBits + 1) + sl] / kPi) & 1)
                words[size_t(sl) * nw + grp / 64] |= 1ull << (grp % 64);
          for (uint64_t w : words) {
            double d;
            std::memcpy(&d, &w, sizeof d);  // raw bits in the double pool
            plan.btab.push_back(d);
          }
          rec.ctab_n = 0;
        } else {
          plan.btab.insert(plan.btab.end(), ang.begin(), ang.end());
          // the same angles as unit complex factors (left zero for a scaled
          // record: its scale is known per launch)
          rec.ctab_n = ngr * (kRegBits + 1) + (1 << kRegBits);
          for (int i = 0; i < ngr * (kRegBits + 1); ++i)
            plan.ctab.push_back(rec.scale_idx < 0 ? std::polar(1.0, ang[i]) : cd(0, 0));
          for (int e = 0; e < (1 << kRegBits); ++e)
            plan.ctab.push_back(rec.scale_idx < 0 ? plan.qtab[rec.wr_off + e] : cd(0, 0));
        }
      }
      if (op.kind != OP_PHASE) op.flags = 0;
      if (op.kind == OP_ROT && op.pauli == 2) op.flags |= 1u;
      if (op.kind == OP_ROT && op.pauli == 1) op.flags |= 8u;   // [[c, -is], [-is, c]]
      if (op.kind == OP_ROT && op.pauli == 3) op.flags |= 16u;  // diagonal
      if (dim) {
        bool real = true;
        for (int i = 0; i < dim * dim; ++i) real &= plan.matpool[op.mat + i].imag() == 0.0;
        if (real) op.flags |= 1u;
      }
      if (op.kind == OP_DENSE1 && !(op.flags & 1u)) {
        // forward and inverse both diagonal, or both of the form [[a, ib], [ib, a]], a and b real
        const cd* M = plan.matpool.data() + op.mat;
        bool diag = true, xf = true;
        for (int w2 = 0; w2 < 2; ++w2, M += 4) {
          diag &= M[1] == 0.0 && M[2] == 0.0;
          xf &= M[0] == M[3] && M[0].imag() == 0.0 && M[1] == M[2] && M[1].real() == 0.0;
        }
        if (diag) op.flags |= 16u;
        else if (xf) op.flags |= 8u;
      }
      if (lane_j >= 0) {
        op.flags |= 32u;
        if (used_lanes) *used_lanes = true;
      }
      if (op.cin != 0 || op.creg != 0) g.ctrl = 1;
      out.push_back(op);
    }
    plan.stages.push_back(sr);
  }
  g.nst = (int)sts.size();
  ps.ops = out;
  g.kern = 2;
}

// Stage a pass; when its forward stages use lane ops, stage the same ops
// again without them for the two-state kernel (its phase records are copies,
// since a record's tables depend on the stage it sits in).
void stage_pass(Plan& plan, Pass& ps) {
  std::vector<TileOp> orig = ps.ops;
  // staging may swap the two index bits of a two-qubit matrix (forward and
  // inverse, 2 x 16 entries) in place: the second staging gets its own copy
  // of the matrices as they are now
  std::vector<int> mat2;
  for (const TileOp& op : orig)
    if (op.kind == OP_DENSE2) {
      mat2.push_back((int)plan.matpool.size());
      for (int i = 0; i < 32; ++i) plan.matpool.push_back(plan.matpool[op.mat + i]);
    }
  bool used = false;
  stage_ops(plan, ps.geom, ps.ops, plan.lane_ops, &used);
  ps.has_adj = false;
  ps.ops_adj.clear();
  if (ps.geom.kern != 2 || !used) return;  // (the copies stay unused)
  size_t k2 = 0;
  for (TileOp& op : orig) {
    if (op.kind == OP_PHASE) {
      plan.phases.push_back(plan.phases[op.aux]);
      op.aux = (int)plan.phases.size() - 1;
    } else if (op.kind == OP_DENSE2) {
      op.mat = mat2[k2++];
    }
  }
  ps.geom_adj = ps.geom;
  stage_ops(plan, ps.geom_adj, orig, false, nullptr);
  ps.ops_adj = std::move(orig);
  ps.has_adj = true;
}

// Close an open pass: fix the tile bit set, convert ops to tile-local form,
// build the phase tables.
void close_pass(Plan& plan, const HostCircuit& C, int m, int L, std::set<int>& hsel,
                std::vector<RawOp>& raw) {
  const int n = C.n;
  // pad the high set with the lowest unused bits: longer contiguous runs
  for (int b = L; b < n && (int)hsel.size() < m - L; ++b) hsel.insert(b);
  Pass ps;
  ps.kind = PASS_TILE;
  PassGeom& g = ps.geom;
  g.n = n;
  g.L = L;
  g.H = (int)hsel.size();
  g.m = L + g.H;
  int i = 0;
  for (int b : hsel) g.hbits[i++] = b;
  for (; i < kMaxTileBits; ++i) g.hbits[i] = 0;
  int local[kMaxQubits];
  for (int b = 0; b < n; ++b) local[b] = -1;
  for (int b = 0; b < L; ++b) local[b] = b;
  for (int j = 0; j < g.H; ++j) local[g.hbits[j]] = L + j;

  int ngrad = 0;
  for (RawOp& r : raw) {
    TileOp op;
    std::memset(&op, 0, sizeof(op));
    op.mat = -1;
    op.pidx = -1;
    op.aux = -1;
    op.gslot = -1;
    op.sign = 1;
    op.kind = r.kind;
    if (r.kind == OP_PHASE) {
      op = make_phase_op(plan, g, r.poly, r.scale_idx);
    } else {
      const BitGate& bg = r.g;
      op.k = bg.k;
      for (int t = 0; t < bg.k; ++t) {
        if (local[bg.tb[t]] < 0) throw std::runtime_error("planner: target outside tile");
        op.b[t] = local[bg.tb[t]];
      }
      for (uint64_t cm = bg.cmask; cm; cm &= cm - 1) {
        int b = __builtin_ctzll(cm);
        if (local[b] >= 0) op.cin |= 1u << local[b];
        else op.cout |= 1ull << b;
      }
      if (r.kind == OP_ROT) {
        op.pidx = bg.pidx;
        op.sign = bg.rsign;
        op.pauli = bg.pauli == 'X' ? 1 : bg.pauli == 'Y' ? 2 : 3;
        if (bg.pidx >= 0) {
          if (ngrad >= kMaxGradPerPass) throw std::runtime_error("planner: too many parameters in one pass");
          op.gslot = plan.ngrad_slots++;
          op.aux = ngrad++;
        }
        // forward and inverse 2x2, then their three-shear parameters, written per run
        op.mat = (int)plan.matpool.size();
        plan.matpool.insert(plan.matpool.end(), 12, cd(0, 0));
      } else {
        const int dim = 1 << bg.k;
        op.mat = (int)plan.matpool.size();
        plan.matpool.insert(plan.matpool.end(), bg.mat.begin(), bg.mat.end());
        std::vector<cd> inv = dagger(bg.mat, dim);
        plan.matpool.insert(plan.matpool.end(), inv.begin(), inv.end());
      }
    }
    ps.ops.push_back(op);
  }
  if (!ps.ops.empty()) {
    stage_pass(plan, ps);
    plan.passes.push_back(ps);
  }
  raw.clear();
  hsel.clear();
}

// Matrix of gate g (targets then controls, all inside `sup`) on the qubit
// list sup (sup[0] = most significant matrix bit).
std::vector<cd> embed_gate(const Gate& g, const std::vector<int>& sup) {
  const int w = (int)sup.size(), dim = 1 << w, dk = 1 << g.k;
  auto bitpos = [&](int q) { return w - 1 - int(std::find(sup.begin(), sup.end(), q) - sup.begin()); };
  std::vector<int> tp(g.k), cp;
  for (int t = 0; t < g.k; ++t) tp[t] = bitpos(g.tq[t]);
  for (int q : g.cq) cp.push_back(bitpos(q));
  std::vector<cd> M(size_t(dim) * dim, cd(0, 0));
  for (int x = 0; x < dim; ++x) {
    bool on = true;
    for (int c : cp) on &= ((x >> c) & 1) != 0;
    if (!on) {
      M[size_t(x) * dim + x] = 1.0;
      continue;
    }
    int col = 0, rest = x;
    for (int t = 0; t < g.k; ++t) {
      col = (col << 1) | ((x >> tp[t]) & 1);
      rest &= ~(1 << tp[t]);
    }
    for (int r = 0; r < dk; ++r) {
      int y = rest;
      for (int t = 0; t < g.k; ++t)
        if ((r >> (g.k - 1 - t)) & 1) y |= 1 << tp[t];
      M[size_t(y) * dim + x] += g.mat[size_t(r) * dk + col];
    }
  }
  return M;
}

}  // namespace

// Greedy fusion (the paper's circuit.fuse() of Sec. 2.4.5, widened to K
// qubits): consecutive fixed gates are multiplied into one dense matrix while
// their joint support stays within K qubits; rotations with run-time angles
// end a block and pass through.
std::vector<StagedOp> staged_records(const std::vector<TileOp>& ops, const std::vector<PhaseRec>& phases) {
  std::vector<StagedOp> out(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    const TileOp& op = ops[i];
    StagedOp& r = out[i];
    r.opc = -1;
    r.ctl = (op.cin & 0xFFFFu) | (op.creg << 16);
    r.cout_lo = (uint32_t)op.cout;
    r.cout_hi = (uint32_t)(op.cout >> 32);
    r.mat = op.mat;
    r.grad = (op.kind == OP_ROT && op.gslot >= 0) ? (op.aux | (op.pauli << 8) | (op.b[0] << 12)) : -1;
    r.ph = 0;
    r.tab = 0;
    const bool one = op.kind == OP_DENSE1 || op.kind == OP_ROT;
    if (op.kind == OP_PHASE) {
      const PhaseRec& rec = phases[op.aux];
      const bool single = (op.flags & 2u) != 0;
      r.ph = (op.pidx & 0xFF) | ((single ? op.b[0] & 3 : 0) << 8) | ((rec.wr_trivial ? 1 : 0) << 10) |
             ((single ? 1 : 0) << 11) | (int32_t)((uint32_t)(rec.wr_sign & 0xFFFF) << 16);
      if (op.flags & 4u) {
        r.opc = 14;
        r.tab = rec.bt_off;
      } else {
        r.opc = single ? 20 + op.b[0] : 19;
        r.tab = rec.ctab_off;
        r.mat = rec.ctab_n;
      }
      continue;
    }
    if (op.cin != 0 || op.creg != 0) {  // controlled: predicated path
      const bool two = op.kind == OP_DENSE2;
      r.tab = (one || two) ? (op.b[0] & 15) | ((two ? op.b[1] & 15 : 0) << 4) | (((op.flags & 1u) ? 1 : 0) << 8) |
                                 ((two ? 1 : 0) << 9)
                           : -1;
      continue;
    }
    if (one && (op.flags & 32u)) {  // lane ops
      const int form = (op.flags & 16u) ? 2 : (op.flags & 8u) ? 3 : (op.flags & 1u) ? 1 : 0;
      r.opc = 40 + 4 * form + op.b[0];
    } else if (op.kind == OP_ROT && (op.pauli == 1 || op.pauli == 2)) {  // X / Y rotation: three shears
      r.opc = (op.pauli == 1 ? 36 : 32) + op.b[0];
    } else if (one) {
      r.opc = ((op.flags & 16u) ? 24 : (op.flags & 8u) ? 28 : (op.flags & 1u) ? 4 : 0) + op.b[0];
    } else if (op.kind == OP_DENSE2) {
      const int kh = op.b[0], kl = op.b[1];
      r.opc = 8 + (kh == 1 ? 0 : kh == 2 ? 1 + kl : 3 + kl);
    }
  }
  return out;
}

std::vector<Gate> fuse_gates(const std::vector<Gate>& in, int K) {
  std::vector<Gate> out;
  std::vector<int> sup;
  std::vector<cd> U;
  std::vector<const Gate*> members;
  auto flush = [&]() {
    if (members.size() == 1) out.push_back(*members[0]);
    else if (!members.empty()) {
      Gate f;
      f.k = (int)sup.size();
      for (int i = 0; i < f.k; ++i) f.tq[i] = sup[i];
      f.mat = U;
      out.push_back(f);
    }
    members.clear();
    sup.clear();
    U.clear();
  };
  for (const Gate& g : in) {
    if (g.is_rot || g.spoly) {
      flush();
      out.push_back(g);
      continue;
    }
    std::vector<int> gs(g.tq, g.tq + g.k);
    gs.insert(gs.end(), g.cq.begin(), g.cq.end());
    std::vector<int> u = sup;
    for (int q : gs)
      if (!has(u, q)) u.push_back(q);
    if ((int)u.size() > K) {
      flush();
      u = gs;
    }
    std::sort(u.begin(), u.end());
    const int dim = 1 << u.size();
    // re-express the block so far on the grown support, then apply g
    std::vector<cd> prev(size_t(dim) * dim, cd(0, 0));
    if (members.empty()) {
      for (int i = 0; i < dim; ++i) prev[size_t(i) * dim + i] = 1.0;
    } else {
      Gate blk;
      blk.k = (int)sup.size();
      for (int i = 0; i < blk.k; ++i) blk.tq[i] = sup[i];
      blk.mat = U;
      prev = embed_gate(blk, u);
    }
    U = matmul(embed_gate(g, u), prev, dim);
    sup = u;
    members.push_back(&g);
    if (sup.size() > 5) throw std::runtime_error("fusion support exceeds 5 qubits");
  }
  flush();
  return out;
}

namespace {

// A dense block on matrix cores: tile = targets + the 7 lowest other bits.
// Low bits of a matrix-core pass whose blocks of k qubits target the bit set
// tm: the tile is [0, L) and the targets above L, k + 7 bits in all, with the
// smallest such L.  -1 when that L is below 7 (rows shorter than 128
// amplitudes), which only happens when two blocks share a tile.
int mfma_low_bits(uint64_t tm, int k, int n) {
  for (int L = 0; L <= n && L < 64; ++L)
    if (L + __builtin_popcountll(tm >> L) == k + 7) return L >= 7 ? L : -1;
  return -1;
}

uint64_t target_mask(const BitGate& b) {
  uint64_t tm = 0;
  for (int t = 0; t < b.k; ++t) tm |= 1ull << b.tb[t];
  return tm;
}

// One matrix-core pass: block b, and with b2 a second block of the same size
// on other bits that shares the tile (each block's targets lie among the
// other's 128 columns).
void add_mfma_pass(Plan& plan, int n, const BitGate& b, const BitGate* b2 = nullptr) {
  Pass ps;
  ps.kind = PASS_MFMA;
  const uint64_t tm = target_mask(b) | (b2 ? target_mask(*b2) : 0);
  const int L = mfma_low_bits(tm, b.k, n);
  if (L < 0) throw std::runtime_error("planner: matrix-core blocks do not fit one tile");
  std::vector<int> hs;
  for (uint64_t h = L >= 64 ? 0 : (tm >> L) << L; h; h &= h - 1) hs.push_back(__builtin_ctzll(h));
  PassGeom& g = ps.geom;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.L = L;
  g.H = (int)hs.size();
  g.m = L + g.H;
  for (int i = 0; i < g.H; ++i) g.hbits[i] = hs[i];
  g.kern = 0;
  for (const BitGate* bp : {&b, b2}) {
    if (!bp) continue;
    TileOp op;
    std::memset(&op, 0, sizeof(op));
    op.kind = OP_MFMA;
    op.k = bp->k;
    op.gslot = -1;
    op.pidx = -1;
    op.aux = -1;
    for (int t = 0; t < bp->k; ++t) {
      const int bit = bp->tb[t];
      op.b[t] = bit < L ? bit : L + (int)(std::find(hs.begin(), hs.end(), bit) - hs.begin());
    }
    const int dim = 1 << bp->k;
    op.mat = (int)plan.matpool.size();
    plan.matpool.insert(plan.matpool.end(), bp->mat.begin(), bp->mat.end());
    std::vector<cd> inv = dagger(bp->mat, dim);
    plan.matpool.insert(plan.matpool.end(), inv.begin(), inv.end());
    ps.ops.push_back(op);
  }
  plan.passes.push_back(ps);
}

// Involutive bit-permutation pass: data at bit a moves to bit tau[a].
void add_perm_pass(Plan& plan, int n, int L, bool dbl, const std::vector<int>& tau) {
  bool ident = true;
  for (int a = 0; a < n; ++a) ident &= tau[a] == a;
  if (ident) return;
  // the tile holds the low bits and their images: at most 2L bits, and the
  // permutation kernel takes tiles of at most 2^12 (complex64) or 2^11
  // (complex128) amplitudes
  L = std::min(L, dbl ? 5 : 6);
  Pass ps;
  ps.kind = PASS_PERM;
  ps.sigma = tau;
  std::set<int> hs;
  for (int a = 0; a < L; ++a)
    if (tau[a] >= L) hs.insert(tau[a]);
  const int mt = std::min(n, dbl ? 10 : 11);
  for (int b = L; b < n && L + (int)hs.size() < mt; ++b)
    if (tau[b] == b) hs.insert(b);
  PassGeom& g = ps.geom;
  g.n = n;
  g.L = L;
  g.H = (int)hs.size();
  g.m = L + g.H;
  int i = 0;
  for (int b : hs) g.hbits[i++] = b;
  for (; i < kMaxTileBits; ++i) g.hbits[i] = 0;
  plan.passes.push_back(ps);
}

}  // namespace

namespace {

Plan plan_tiles(const HostCircuit& C, const TuneOpts& opts, bool dbl, int m, int L) {
  const int n = C.n;
  Plan proto;
  proto.n = n;
  proto.dbl = dbl;
  proto.nparams = C.nparams;
  proto.ngates = (int)C.gates.size();
  proto.grid_bits = opts.grid_bits;
  proto.force_stage = opts.force_stage;
  proto.lane_ops = opts.lane_ops;
  const int Hmax = m - L;

  // 0. optional fusion of consecutive fixed gates into <= fuse_k-qubit blocks
  const std::vector<Gate> fused = opts.fuse_k >= 2 ? fuse_gates(C.gates, opts.fuse_k) : std::vector<Gate>();
  const std::vector<Gate>& gates = opts.fuse_k >= 2 ? fused : C.gates;

  // 1. relabel SWAPs, convert to index bits
  std::vector<int> phys(n);
  for (int q = 0; q < n; ++q) phys[q] = n - 1 - q;
  std::vector<BitGate> bg;
  bg.reserve(gates.size());
  for (const Gate& g : gates) {
    if (!g.is_rot && g.k == 2 && g.cq.empty() && is_swap(g.mat)) {
      std::swap(phys[g.tq[0]], phys[g.tq[1]]);
      continue;
    }
    bg.push_back(to_bits(g, n, phys, opts));
  }
  const int G = (int)bg.size();

  // 2. dependency graph: two gates commute on a shared bit only when both act
  //    diagonally there (controls, diagonal gates, Z rotations)
  std::vector<std::vector<int>> succ(G);
  std::vector<int> indeg0(G, 0);
  {
    std::vector<int> lastN(n, -1);
    std::vector<std::vector<int>> dsince(n);
    std::vector<int> mark(G, -1);
    for (int g = 0; g < G; ++g) {
      auto edge = [&](int from) {
        if (from < 0 || mark[from] == g) return;
        mark[from] = g;
        succ[from].push_back(g);
        indeg0[g]++;
      };
      uint64_t all = bg[g].nmask | bg[g].dmask;
      for (uint64_t t = all; t; t &= t - 1) {
        int b = __builtin_ctzll(t);
        edge(lastN[b]);
        if ((bg[g].nmask >> b) & 1)
          for (int d : dsince[b]) edge(d);
      }
      for (uint64_t t = all; t; t &= t - 1) {
        int b = __builtin_ctzll(t);
        if ((bg[g].nmask >> b) & 1) {
          lastN[b] = g;
          dsince[b].clear();
        } else {
          dsince[b].push_back(g);
        }
      }
    }
  }

  // 3. greedy list scheduling into tiled passes.  With lookahead (mode 1),
  //    each pass first picks its high bits: starting from the low bits, it
  //    repeatedly adds the new bits of the blocked gate that unlock the most
  //    gates per added bit (the gates reachable in dependency order inside the
  //    tile); mode 2 also tries every first choice, each completed that way,
  //    and keeps the set that unlocks the most gates.  Gates are then placed
  //    in index order as without lookahead (mode 0).
  auto schedule = [&](int mode) -> Plan {
    Plan plan = proto;
    std::vector<int> indeg = indeg0;
    std::set<int> ready;
    for (int g = 0; g < G; ++g)
      if (indeg[g] == 0) ready.insert(g);
    PhasePoly P;
    P.init(n);
    std::set<int> hsel;
    std::vector<RawOp> raw;
    int scheduled = 0;
    const uint64_t lowmask = L >= 64 ? ~0ull : ((1ull << L) - 1);
    const bool fuse1 = opts.fuse_k != 1;

    auto finish = [&](int g, std::set<int>::iterator& it) {
      it = ready.erase(it);
      ++scheduled;
      for (int s : succ[g])
        if (--indeg[s] == 0) ready.insert(s);
    };

    std::vector<int> seen(G, 0), touched;
    // non-phase gates placeable with tile bits T from the current ready set; the
    // blocked gates that wait only for tile bits go to front
    auto closure = [&](uint64_t T, std::vector<int>* front) {
      std::vector<int> stack(ready.begin(), ready.end());
      int cnt = 0, ngr = 0;
      while (!stack.empty()) {
        const int g = stack.back();
        stack.pop_back();
        const BitGate& b = bg[g];
        const bool diag = b.kind == BK_PHASE || b.kind == BK_SPHASE;
        if (!diag) {
          if (b.mfma) continue;
          bool fits = true;
          for (int t = 0; t < b.k; ++t) fits = fits && ((T >> b.tb[t]) & 1);
          if (!fits) {
            if (front) front->push_back(g);
            continue;
          }
          if (b.kind == BK_ROT && b.pidx >= 0 && ngr++ >= kMaxGradPerPass) continue;
          ++cnt;
        }
        for (int s : succ[g]) {
          if (seen[s]++ == 0) touched.push_back(s);
          if (seen[s] == indeg[s]) stack.push_back(s);
        }
      }
      for (int s : touched) seen[s] = 0;
      touched.clear();
      return cnt;
    };
    // grow the bit set T (nh high bits) greedily by unlocked gates per added bit
    auto complete = [&](uint64_t T, int nh) {
      std::vector<int> front;
      std::vector<uint64_t> tried;
      while (nh < Hmax) {
        front.clear();
        tried.clear();
        const int base = closure(T, &front);
        std::sort(front.begin(), front.end());
        double best = 0.0;
        uint64_t pick = 0;
        if ((int)front.size() > kRolloutMaxFront) front.resize(kRolloutMaxFront);  // lowest gate indices first
        for (int g : front) {
          uint64_t need = 0;
          for (int t = 0; t < bg[g].k; ++t) need |= (1ull << bg[g].tb[t]) & ~T;
          const int c = __builtin_popcountll(need);
          if (nh + c > Hmax || std::find(tried.begin(), tried.end(), need) != tried.end()) continue;
          tried.push_back(need);
          const double score = (double)(closure(T | need, nullptr) - base) / c;
          if (score > best) {
            best = score;
            pick = need;
          }
        }
        if (!pick) break;
        T |= pick;
        nh += __builtin_popcountll(pick);
      }
      return T;
    };
    // mode 1: greedy growth; mode 2: every first choice completed greedily,
    // the set that unlocks the most gates kept
    auto pick_bits = [&]() {
      uint64_t T = complete(lowmask, 0);
      if (mode == 2) {
        std::vector<int> front;
        std::vector<uint64_t> tried;
        closure(lowmask, &front);
        std::sort(front.begin(), front.end());
        int best = closure(T, nullptr);
        if ((int)front.size() > kRolloutMaxFront) front.resize(kRolloutMaxFront);  // lowest gate indices first
        for (int g : front) {
          uint64_t need = 0;
          for (int t = 0; t < bg[g].k; ++t) need |= (1ull << bg[g].tb[t]) & ~lowmask;
          const int c = __builtin_popcountll(need);
          if (c > Hmax || std::find(tried.begin(), tried.end(), need) != tried.end()) continue;
          tried.push_back(need);
          const uint64_t T2 = complete(lowmask | need, c);
          const int cnt = closure(T2, nullptr);
          if (cnt > best) {
            best = cnt;
            T = T2;
          }
        }
      }
      for (uint64_t h = T & ~lowmask; h; h &= h - 1) hsel.insert(__builtin_ctzll(h));
    };

    while (scheduled < G) {
      if (mode && hsel.empty()) pick_bits();
      bool progress = true;
      int placed = 0;
      while (progress) {
        progress = false;
        for (auto it = ready.begin(); it != ready.end();) {
          const int g = *it;
          BitGate& b = bg[g];
          if (b.kind == BK_PHASE) {
            add_terms(P, n, b);
            finish(g, it);
            progress = true;
            ++placed;
            continue;
          }
          if (b.kind == BK_SPHASE) {  // its own phase op, scaled per launch
            if (nphase_raw(raw) >= kMaxPhasePerPass - 2) {
              ++it;
              continue;
            }
            RawOp ro;
            ro.kind = OP_PHASE;
            ro.poly = *b.spoly;
            ro.scale_idx = b.scale_slot;
            raw.push_back(std::move(ro));
            finish(g, it);
            progress = true;
            ++placed;
            continue;
          }
          if (b.mfma) {  // placed between tiled passes below
            ++it;
            continue;
          }
          std::vector<int> need;
          for (int t = 0; t < b.k; ++t) {
            int bit = b.tb[t];
            if (!((lowmask >> bit) & 1) && !hsel.count(bit)) need.push_back(bit);
          }
          if ((int)(hsel.size() + need.size()) > Hmax) {
            ++it;
            continue;
          }
          if (b.nmask && nphase_raw(raw) >= kMaxPhasePerPass - 2) {  // keep the pass staged
            ++it;
            continue;
          }
          if (b.kind == BK_ROT && b.pidx >= 0 && ngrad_raw(raw) >= kMaxGradPerPass) {
            ++it;
            continue;
          }
          for (int bit : need) hsel.insert(bit);
          if (b.nmask && (b.nmask & P.support())) {
            // every pending term comes from a diagonal gate whose predecessors
            // are all placed, so applying all of them here is exact and leaves
            // fewer, fuller phase ops than flushing only the gate's bits
            PhasePoly Q = extract_terms(P, n, ~0ull, false);
            if (!Q.empty) {
              RawOp ro;
              ro.kind = OP_PHASE;
              ro.poly = std::move(Q);
              raw.push_back(std::move(ro));
            }
          }
          const int kind = b.kind == BK_ROT ? OP_ROT : (b.k == 1 ? OP_DENSE1 : b.k == 2 ? OP_DENSE2 : OP_DENSEK);
          bool merged = false;
          if (fuse1 && kind == OP_DENSE1 && !raw.empty()) {
            RawOp& last = raw.back();
            if (last.kind == OP_DENSE1 && last.g.tb[0] == b.tb[0] && last.g.cmask == b.cmask) {
              last.g.mat = matmul(b.mat, last.g.mat, 2);
              merged = true;
            }
          }
          if (!merged) {
            RawOp ro;
            ro.kind = kind;
            ro.g = b;
            raw.push_back(std::move(ro));
          }
          finish(g, it);
          progress = true;
          ++placed;
        }
      }
      int mg = -1;  // a ready matrix-core block goes next, after this pass
      for (int g : ready)
        if (bg[g].mfma) {
          mg = g;
          break;
        }
      // with a second ready block of the same size on other bits when both fit
      // one tile (two complex128 blocks of 32 exceed the kernel's registers)
      int mg2 = -1;
      if (mg >= 0)
        for (int g : ready) {
          if (g == mg || !bg[g].mfma || bg[g].k != bg[mg].k || (dbl && bg[g].k > 4)) continue;
          if (target_mask(bg[g]) & target_mask(bg[mg])) continue;
          if (mfma_low_bits(target_mask(bg[g]) | target_mask(bg[mg]), bg[mg].k, n) < 0) continue;
          mg2 = g;
          break;
        }
      if (mg >= 0) {
        PhasePoly Q = extract_terms(P, n, bg[mg].nmask | (mg2 >= 0 ? bg[mg2].nmask : 0), false);
        if (!Q.empty) {
          RawOp ro;
          ro.kind = OP_PHASE;
          ro.poly = std::move(Q);
          raw.push_back(std::move(ro));
        }
      }
      if (scheduled == G && !P.empty) {
        PhasePoly Q = extract_terms(P, n, ~0ull, true);
        if (!Q.empty) {
          RawOp ro;
          ro.kind = OP_PHASE;
          ro.poly = std::move(Q);
          raw.push_back(std::move(ro));
        }
      }
      if (scheduled == G && C.tail_phase) {
        RawOp ro;
        ro.kind = OP_PHASE;
        ro.poly = *C.tail_phase;
        ro.scale_idx = 0;
        raw.push_back(std::move(ro));
      }
      if (placed == 0 && raw.empty() && mg < 0) throw std::runtime_error("planner: no gate fits a tile");
      close_pass(plan, C, m, L, hsel, raw);
      if (mg >= 0) {
        add_mfma_pass(plan, n, bg[mg], mg2 >= 0 ? &bg[mg2] : nullptr);
        auto it = ready.find(mg);
        finish(mg, it);
        if (mg2 >= 0) {
          it = ready.find(mg2);
          finish(mg2, it);
        }
      }
    }
    if (!P.empty) {  // only reachable for an all-diagonal remainder after the loop
      PhasePoly Q = extract_terms(P, n, ~0ull, true);
      if (!Q.empty) {
        RawOp ro;
        ro.kind = OP_PHASE;
        ro.poly = std::move(Q);
        raw.push_back(std::move(ro));
        close_pass(plan, C, m, L, hsel, raw);
      }
    }

    // 4. restore the qubit order: sigma[phys[q]] = n-1-q, as two involutions
    std::vector<int> sigma(n);
    bool ident = true;
    for (int q = 0; q < n; ++q) {
      sigma[phys[q]] = n - 1 - q;
      ident &= phys[q] == n - 1 - q;
    }
    if (!ident) {
      std::vector<int> t1(n), t2(n);
      for (int a = 0; a < n; ++a) t1[a] = t2[a] = a;
      std::vector<bool> seen(n, false);
      for (int a0 = 0; a0 < n; ++a0) {
        if (seen[a0]) continue;
        std::vector<int> cyc;
        for (int a = a0; !seen[a]; a = sigma[a]) {
          seen[a] = true;
          cyc.push_back(a);
        }
        const int len = (int)cyc.size();
        for (int i = 0; i < len; ++i) {
          t1[cyc[i]] = cyc[((-i) % len + len) % len];
          t2[cyc[i]] = cyc[((1 - i) % len + len) % len];
        }
      }
      int Lp = std::min(L, n);
      add_perm_pass(plan, n, Lp, dbl, t1);
      add_perm_pass(plan, n, Lp, dbl, t2);
    }
    return plan;
  };

  // the three schedules; a lookahead one is kept only when it is shorter.
  // The rollout costs about |front|^2 * Hmax closure walks per pass, so it
  // is skipped for very long gate lists
  Plan plan = schedule(0);
  plan.schedule = 0;
  if (Hmax > 0 && plan.passes.size() > 1)
    for (int mode = 1; mode <= 2; ++mode) {
      if (mode == 2 && G > kRolloutMaxGates) break;
      Plan alt = schedule(mode);
      if (alt.passes.size() < plan.passes.size()) {
        plan = std::move(alt);
        plan.schedule = mode;
      }
    }
  return plan;
}

}  // namespace

// With the row length left open (low_bits 0), rows one bit shorter than the
// default free a tile bit for the high positions.  A pass over such rows
// costs a few percent more (256 instead of 512 contiguous bytes for
// complex64), so that plan is kept only when it needs fewer passes: a ring of
// RY layers and CZ gates on 30 qubits takes 11 passes instead of 13.
Plan plan_circuit(const HostCircuit& C, const TuneOpts& opts, bool dbl) {
  int m, L;
  default_tile(C.n, dbl, opts, &m, &L);
  Plan plan = plan_tiles(C, opts, dbl, m, L);
  if (opts.low_bits == 0 && L > 1 && m - L < kMaxHighBits && m < C.n && plan.passes.size() > 1) {
    Plan alt = plan_tiles(C, opts, dbl, m, L - 1);
    if (alt.passes.size() < plan.passes.size()) plan = std::move(alt);
  }
  return plan;
}

Plan plan_trotter(int n, bool dbl, const TuneOpts& opts, const PhasePoly* poly, int steps, bool final_layer) {
  HostCircuit hc;
  hc.n = n;
  hc.nparams = steps + (final_layer ? 1 : 0);
  for (int s = 0; s < steps; ++s) {
    for (int q = 0; q < n; ++q) {
      Gate g;
      g.k = 1;
      g.tq[0] = q;
      g.is_rot = true;
      g.pauli = 'X';
      g.pidx = s;
      hc.gates.push_back(g);
    }
    Gate ph;
    ph.spoly = poly;
    ph.scale_slot = s;
    hc.gates.push_back(ph);
  }
  if (final_layer)  // the closing half rotation layer, angle slot `steps`, planned with the last steps
    for (int q = 0; q < n; ++q) {
      Gate g;
      g.k = 1;
      g.tq[0] = q;
      g.is_rot = true;
      g.pauli = 'X';
      g.pidx = steps;
      hc.gates.push_back(g);
    }
  return plan_circuit(hc, opts, dbl);
}

}  // namespace qs
