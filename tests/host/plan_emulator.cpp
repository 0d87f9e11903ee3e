// Host check of the pass planner (test infrastructure): a circuit is planned
// as for the GPU, then every planned op is applied to a full state vector in
// planned order -- stage order inside register-staged passes, with register
// slots and lane bits decoded back to tile bits, tile bits to index bits --
// and compared with the circuit's gates applied one by one in user order.
// Both the one-state form of each pass and its two-state (adjoint) form are
// checked.  Exit status 0 when both agree to 1e-9.
//
//   plan_emulator <n> <tile_bits> <seed> <mode> [lane_ops] [complex128]
//   mode 0: random 1-/2-qubit gates with 0..2 controls (dense and diagonal)
//   mode 1: layers of X/Y/Z rotations on every qubit and a CZ ring
//   mode 2: QFT with its closing SWAPs
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "planner.h"

using namespace qs;
using Z = std::complex<double>;

static void apply_k(std::vector<Z>& psi, int n, const std::vector<int>& tb, const Z* M, uint64_t cmask) {
  const int k = (int)tb.size(), d = 1 << k;
  std::vector<Z> in(d), out(d);
  std::vector<uint64_t> idx(d);
  for (uint64_t x = 0; x < (1ull << n); ++x) {
    bool base = (x & cmask) == cmask;
    for (int t = 0; t < k; ++t) base = base && !((x >> tb[t]) & 1);
    if (!base) continue;
    for (int r = 0; r < d; ++r) {
      uint64_t y = x;
      for (int t = 0; t < k; ++t)
        if ((r >> (k - 1 - t)) & 1) y |= 1ull << tb[t];
      idx[r] = y;
      in[r] = psi[y];
    }
    for (int r = 0; r < d; ++r) {
      Z s = 0;
      for (int c = 0; c < d; ++c) s += M[r * d + c] * in[c];
      out[r] = s;
    }
    for (int r = 0; r < d; ++r) psi[idx[r]] = out[r];
  }
}

static std::vector<Z> rot(char p, double th) {
  const double c = std::cos(th / 2), s = std::sin(th / 2);
  if (p == 'X') return {c, Z(0, -s), Z(0, -s), c};
  if (p == 'Y') return {c, -s, s, c};
  return {std::polar(1.0, -th / 2), 0, 0, std::polar(1.0, th / 2)};
}

int main(int argc, char** argv) {
  if (argc < 5) return 2;
  const int n = atoi(argv[1]), tile_bits = atoi(argv[2]), seed = atoi(argv[3]), mode = atoi(argv[4]);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> N01;
  auto haar = [&](int d) {  // Gram-Schmidt of a complex Gaussian matrix
    std::vector<cd> m(d * d);
    for (auto& v : m) v = cd(N01(rng), N01(rng));
    for (int r = 0; r < d; ++r) {
      for (int q = 0; q < r; ++q) {
        cd dot = 0;
        for (int c = 0; c < d; ++c) dot += std::conj(m[q * d + c]) * m[r * d + c];
        for (int c = 0; c < d; ++c) m[r * d + c] -= dot * m[q * d + c];
      }
      double nn = 0;
      for (int c = 0; c < d; ++c) nn += std::norm(m[r * d + c]);
      for (int c = 0; c < d; ++c) m[r * d + c] /= std::sqrt(nn);
    }
    return m;
  };
  HostCircuit C;
  C.n = n;
  std::vector<double> params;
  if (mode == 0) {
    for (int gi = 0; gi < 160; ++gi) {
      Gate g;
      const int k = 1 + (int)(rng() % 2), nc = (int)(rng() % 3);
      std::vector<int> q;
      while ((int)q.size() < k + nc) {
        const int x = (int)(rng() % n);
        bool dup = false;
        for (int y : q) dup |= y == x;
        if (!dup) q.push_back(x);
      }
      g.k = k;
      for (int t = 0; t < k; ++t) g.tq[t] = q[t];
      for (int c = 0; c < nc; ++c) g.cq.push_back(q[k + c]);
      if (k == 1 && rng() % 3 == 0) {
        const double th = N01(rng);
        g.mat = {std::polar(1.0, -th / 2), 0, 0, std::polar(1.0, th / 2)};
      } else {
        g.mat = haar(1 << k);
      }
      C.gates.push_back(g);
    }
  } else if (mode == 1) {
    std::uniform_real_distribution<double> U(0, 2 * M_PI);
    for (int l = 0; l < 6; ++l) {
      for (int q = 0; q < n; ++q) {
        Gate g;
        g.k = 1;
        g.tq[0] = q;
        g.is_rot = true;
        g.pauli = "XYZ"[(q + l) % 3];
        g.pidx = (int)params.size();
        params.push_back(U(rng));
        C.gates.push_back(g);
      }
      for (int q = 0; q < n; ++q) {
        Gate g;
        g.k = 1;
        g.tq[0] = (q + 1) % n;
        g.cq = {q};
        g.mat = {1, 0, 0, -1};
        C.gates.push_back(g);
      }
    }
    C.nparams = (int)params.size();
  } else if (mode == 3) {  // dense 5- and 4-qubit blocks on low, high and spread qubits (matrix cores)
    const std::vector<std::vector<int>> sets = {
        {n - 5, n - 4, n - 3, n - 2, n - 1}, {0, 1, 2, 3, 4}, {0, n / 4, n / 2, 3 * n / 4, n - 1},
        {n - 4, n - 3, n - 2, n - 1},       {0, 1, 2, 3},    {3, n / 3 + 1, 2 * n / 3, n - 3},
        {1, 2, 3, 4},                        {n - 2, n - 3, n - 4, n - 5}};
    for (const auto& t : sets) {
      Gate g;
      g.k = (int)t.size();
      for (int i = 0; i < g.k; ++i) g.tq[i] = t[i];
      g.mat = haar(1 << g.k);
      C.gates.push_back(g);
    }
  } else {
    const double r = 1 / std::sqrt(2.0);
    for (int j = 0; j < n; ++j) {
      Gate h;
      h.k = 1;
      h.tq[0] = j;
      h.mat = {r, r, r, -r};
      C.gates.push_back(h);
      for (int k = j + 1; k < n; ++k) {
        Gate c;
        c.k = 1;
        c.tq[0] = j;
        c.cq = {k};
        c.mat = {1, 0, 0, std::polar(1.0, 2 * M_PI / std::pow(2.0, k - j + 1))};
        C.gates.push_back(c);
      }
    }
    for (int j = 0; j < n / 2; ++j) {
      Gate sw;
      sw.k = 2;
      sw.tq[0] = j;
      sw.tq[1] = n - 1 - j;
      sw.mat = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};
      C.gates.push_back(sw);
    }
  }
  TuneOpts o;
  o.tile_bits = tile_bits;
  o.lane_ops = argc > 5 ? atoi(argv[5]) != 0 : true;
  const bool dbl = argc > 6 && atoi(argv[6]) != 0;  // plan for complex128
  if (mode == 3) o.use_mfma = 1;
  const Plan p = plan_circuit(C, o, dbl);
  int fused = 0;
  for (const Pass& ps : p.passes) fused += ps.kind == PASS_MFMA && ps.ops.size() == 2;

  std::vector<Z> psi0(1ull << n);
  for (auto& v : psi0) v = Z(N01(rng), N01(rng));
  std::vector<Z> ref = psi0;
  for (const Gate& g : C.gates) {
    std::vector<int> tb;
    for (int t = 0; t < g.k; ++t) tb.push_back(n - 1 - g.tq[t]);
    uint64_t cm = 0;
    for (int q : g.cq) cm |= 1ull << (n - 1 - q);
    const std::vector<Z> M = g.is_rot ? rot(g.pauli, g.rsign * params[g.pidx]) : std::vector<Z>(g.mat.begin(), g.mat.end());
    apply_k(ref, n, tb, M.data(), cm);
  }
  int lane_ops = 0;
  for (int form = 0; form < 2; ++form) {  // 0: one-state form, 1: two-state form
    std::vector<Z> psi = psi0;
    for (const Pass& ps : p.passes) {
      const PassGeom& g = form ? ps.adj_geom() : ps.geom;
      const std::vector<TileOp>& ops = form ? ps.adj_ops() : ps.ops;
      auto pos = [&](int t) { return t < g.L ? t : g.hbits[t - g.L]; };
      if (ps.kind == PASS_PERM) {
        std::vector<Z> out(psi.size());
        for (uint64_t x = 0; x < psi.size(); ++x) {
          uint64_t y = 0;
          for (int a = 0; a < n; ++a)
            if ((x >> a) & 1) y |= 1ull << ps.sigma[a];
          out[y] = psi[x];
        }
        psi = out;
        continue;
      }
      if (ps.kind != PASS_TILE && ps.kind != PASS_MFMA) {
        std::printf("pass kind %d is not emulated\n", ps.kind);
        return 2;
      }
      auto run_op = [&](const TileOp& op, const StageRec* sr) {
        uint64_t cm = op.cout;
        for (uint32_t c = op.cin; c; c &= c - 1) cm |= 1ull << pos(__builtin_ctz(c));
        if (sr)
          for (uint32_t c = op.creg; c; c &= c - 1) cm |= 1ull << pos(sr->rb[__builtin_ctz(c)]);
        if (op.kind == OP_PHASE) {
          const double* P = p.dpool.data() + p.phases[op.aux].dpool;
          for (uint64_t x = 0; x < psi.size(); ++x) {
            double th = P[0];
            for (int a = 0; a < n; ++a)
              if ((x >> a) & 1) {
                th += P[1 + a];
                for (int b = a + 1; b < n; ++b)
                  if ((x >> b) & 1) th += P[1 + n + a * n + b];
              }
            psi[x] *= std::polar(1.0, th);
          }
          return;
        }
        const int k = op.kind == OP_DENSE1 || op.kind == OP_ROT ? 1 : op.kind == OP_DENSE2 ? 2 : op.k;
        std::vector<int> tb;
        for (int t = 0; t < k; ++t) {
          int local = op.b[t];
          if (sr && (op.flags & 32u)) {  // lane j: the j-th tile bit outside the registers
            local = -1;
            for (int b = 0, cnt = 0; b < g.m && local < 0; ++b)
              if (!((sr->rbmask >> b) & 1) && cnt++ == op.b[t]) local = b;
            ++lane_ops;
          } else if (sr) {
            local = sr->rb[op.b[t]];
          }
          tb.push_back(pos(local));
        }
        const std::vector<Z> M = op.kind == OP_ROT ? rot("?XYZ"[op.pauli], op.sign * params[op.pidx])
                                                   : std::vector<Z>(p.matpool.begin() + op.mat,
                                                                    p.matpool.begin() + op.mat + (1 << (2 * k)));
        apply_k(psi, n, tb, M.data(), cm);
      };
      if (ps.kind == PASS_TILE && g.kern == 2) {
        for (int s = 0; s < g.nst; ++s) {
          const StageRec& sr = p.stages[g.st0 + s];
          for (int i = sr.op0; i < sr.op0 + sr.nops; ++i) run_op(ops[i], &sr);
        }
      } else {
        for (const TileOp& op : ops) run_op(op, nullptr);
      }
    }
    double err = 0;
    for (size_t i = 0; i < psi.size(); ++i) err = std::max(err, std::abs(psi[i] - ref[i]));
    std::printf("%s n=%d tile_bits=%d seed=%d mode=%d passes=%zu lane_ops=%d mfma_fused=%d max_err=%.3e\n",
                form ? "two-state" : "one-state", n, tile_bits, seed, mode, p.passes.size(), lane_ops, fused, err);
    if (!(err < 1e-9)) return 1;
  }
  return 0;
}
