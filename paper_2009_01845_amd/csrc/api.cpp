// C ABI of the simulator: handle management, validation, plan upload and
// the host side of every entry point declared in include/qsim.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qsim.h"
#include "kernels.h"
#include "linalg.h"
#include "planner.h"

using namespace qs;

namespace {

thread_local std::string g_err;

struct Fail {
  qs_status code;
  std::string msg;
};

[[noreturn]] void fail(qs_status c, const std::string& m) { throw Fail{c, m}; }

void hipck(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) fail(QS_E_NOMEM, std::string(what) + ": out of device memory");
  if (e != hipSuccess) fail(QS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F> qs_status guard(F&& f) {
  try {
    f();
    g_err.clear();
    return QS_OK;
  } catch (const Fail& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return QS_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return QS_E_INVALID;
  } catch (...) {
    g_err = "unknown error";
    return QS_E_DEVICE;
  }
}

// ------------------------------------------------------------------ profiling
struct ProfEv {
  int fam;
  hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfEv> g_prof_ev;
int64_t g_prof_cnt[10] = {0};
double g_prof_ms[10] = {0};

struct ProfScope {
  int fam;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int f, hipStream_t st) : fam(f), s(st) {
    if (!g_prof) return;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!g_prof || !a) return;
    (void)hipEventRecord(b, s);
    g_prof_ev.push_back({fam, a, b});
  }
};

void prof_collect() {
  for (auto& e : g_prof_ev) {
    (void)hipEventSynchronize(e.b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e.a, e.b);
    g_prof_cnt[e.fam]++;
    g_prof_ms[e.fam] += ms;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  g_prof_ev.clear();
}

// ---------------------------------------------------------------- buffers
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) {
      hipck(hipDeviceSynchronize(), "hipDeviceSynchronize");
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    if (b == 0) return;
    hipck(hipMalloc(&p, b), "hipMalloc");
    bytes = b;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
};

template <typename T> void upload(DBuf& d, const std::vector<T>& v, hipStream_t s) {
  d.ensure(std::max<size_t>(v.size() * sizeof(T), 16));
  if (!v.empty()) hipck(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
}

bool g_arch_checked = false;
void check_device() {
  if (g_arch_checked) return;
  int dev = 0;
  hipck(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t pr;
  hipck(hipGetDeviceProperties(&pr, dev), "hipGetDeviceProperties");
  if (std::strncmp(pr.gcnArchName, "gfx950", 6) != 0)
    fail(QS_E_UNSUPPORTED, std::string("this library is built for gfx950, device is ") + pr.gcnArchName);
  g_arch_checked = true;
}

// Device copy of a plan.
template <typename T> void upload_complex(DBuf& d, const std::vector<cd>& v, bool dbl, hipStream_t s) {
  std::vector<T> f(v.size() * 2);
  for (size_t i = 0; i < v.size(); ++i) {
    f[2 * i] = (T)v[i].real();
    f[2 * i + 1] = (T)v[i].imag();
  }
  upload(d, f, s);
  (void)dbl;
}

struct DevPlanBuf {
  DBuf ops, sops, mat, dpool, phases, qtab, qang, stages, phlist, btab, matc, ctab;
  bool has_rot = false;
  bool has_scaled = false;
  DevPlan view;
  bool dbl = false;
  std::vector<PassGeom> geoms;      // op0 filled in
  std::vector<PassGeom> geoms_adj;  // the two-state (adjoint) form of each pass
  void load(const Plan& p, hipStream_t s) {
    std::vector<TileOp> all;
    geoms.clear();
    geoms_adj.clear();
    for (const Pass& ps : p.passes) {
      PassGeom g = ps.geom;
      g.op0 = (int)all.size();
      g.nops = (int)ps.ops.size();
      all.insert(all.end(), ps.ops.begin(), ps.ops.end());
      geoms.push_back(g);
    }
    for (size_t i = 0; i < p.passes.size(); ++i) {
      const Pass& ps = p.passes[i];
      if (!ps.has_adj) {
        geoms_adj.push_back(geoms[i]);
        continue;
      }
      PassGeom g = ps.geom_adj;
      g.op0 = (int)all.size();
      g.nops = (int)ps.ops_adj.size();
      all.insert(all.end(), ps.ops_adj.begin(), ps.ops_adj.end());
      geoms_adj.push_back(g);
    }
    upload(ops, all, s);
    upload(sops, staged_records(all, p.phases), s);
    std::vector<double> m(p.matpool.size() * 2);
    for (size_t i = 0; i < p.matpool.size(); ++i) {
      m[2 * i] = p.matpool[i].real();
      m[2 * i + 1] = p.matpool[i].imag();
    }
    upload(mat, m, s);
    if (p.dbl) {
      upload(matc, m, s);
    } else {
      std::vector<float> mf(m.begin(), m.end());
      upload(matc, mf, s);
    }
    has_rot = false;
    for (const TileOp& op : all) has_rot |= op.kind == OP_ROT;
    upload(dpool, p.dpool, s);
    upload(phases, p.phases, s);
    upload(qang, p.qang, s);
    upload(stages, p.stages, s);
    upload(phlist, p.phlist, s);
    upload(btab, p.btab, s);
    dbl = p.dbl;
    if (dbl) upload_complex<double>(ctab, p.ctab, dbl, s);
    else upload_complex<float>(ctab, p.ctab, dbl, s);
    has_scaled = false;
    for (const PhaseRec& r : p.phases) has_scaled |= r.scale_idx >= 0 && r.ctab_off >= 0;
    if (dbl) {
      std::vector<double> q(p.qtab.size() * 2);
      for (size_t i = 0; i < p.qtab.size(); ++i) {
        q[2 * i] = p.qtab[i].real();
        q[2 * i + 1] = p.qtab[i].imag();
      }
      upload(qtab, q, s);
    } else {
      std::vector<float> q(p.qtab.size() * 2);
      for (size_t i = 0; i < p.qtab.size(); ++i) {
        q[2 * i] = (float)p.qtab[i].real();
        q[2 * i + 1] = (float)p.qtab[i].imag();
      }
      upload(qtab, q, s);
    }
    view.ops = ops.as<TileOp>();
    view.sops = sops.as<StagedOp>();
    view.mat = mat.as<double>();
    view.dpool = dpool.as<double>();
    view.phases = phases.as<PhaseRec>();
    view.qtab = qtab.p;
    view.qang = qang.as<double>();
    view.stages = stages.as<StageRec>();
    view.phlist = phlist.as<int32_t>();
    view.btab = btab.as<double>();
    view.matc = matc.p;
    view.ctab = ctab.p;
    view.nphases = (int)p.phases.size();
    view.nops_total = (int)all.size();
  }
};

}  // namespace

// ------------------------------------------------------------------ handles
struct qs_state {
  int n = 0;
  qs_dtype dt = QS_C64;
  void* ptr = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  DBuf scratch;         // reductions
  DBuf scratch2;        // sampling prefix / misc
  DevPlanBuf single;    // plan of the last qs_apply
  bool dbl() const { return dt == QS_C128; }
  size_t bytes() const { return (size_t(1) << n) * (dbl() ? 16 : 8); }
};

struct qs_circuit {
  HostCircuit hc;
  int dens = 0;  // density-matrix circuit on dens qubits (hc.n = 2 dens), 0 for state vectors
  bool planned = false;
  bool plan_dbl = false;
  TuneOpts plan_opts;
  bool dev_ok = false;
  DevPlanBuf dev;
  DBuf dparams;
  DBuf gpart;
  DBuf gout;
  DBuf eout;
  std::vector<int> slot_pidx;
};

// Trotter block plans of one Ising observable and precision, by block length
// and whether the closing rotation layer rides the block.
struct TrotterPlans {
  std::map<std::pair<int, bool>, std::pair<Plan, std::unique_ptr<DevPlanBuf>>> m;
  DBuf ang, scl;  // per-step rotation angles and phase scales of the current segment
};

struct qs_obs {
  int n = 0;
  bool ising = false;
  std::vector<double> J, h;  // ising form (n*n, n)
  // Pauli form grouped by flip mask
  std::vector<uint64_t> flips;
  std::vector<int> goff;
  std::vector<PauliTermDev> terms;
  // the all-diagonal group as a quadratic polynomial in the index bits, when
  // every term in it has at most two Z factors: [c, mu[n], lam[n*n]] and the
  // table of its low-12-bit part (empty when not applicable)
  std::vector<double> poly, elo;
  // every other group, packed into tile sets (one pass over the state each)
  std::vector<PauliSet> sets;
  std::vector<PauliGroupTile> tgroups;
  std::vector<PauliTermTile> tterms;
  std::vector<int> far;  // groups whose flip bits do not fit a tile
  bool dev_ok = false;
  DBuf dflips, dgoff, dterms, dpoly, delo, dtgroups, dtterms;
  // adiabatic runs with this observable as H1: their Trotter plans (complex64,
  // complex128), planned and uploaded at the first run and kept for later ones
  TrotterPlans trotter[2];
  void to_device(hipStream_t s) {
    if (dev_ok) return;
    upload(dflips, flips, s);
    upload(dgoff, goff, s);
    upload(dterms, terms, s);
    if (!poly.empty()) {
      upload(dpoly, poly, s);
      upload(delo, elo, s);
    }
    upload(dtgroups, tgroups, s);
    upload(dtterms, tterms, s);
    dev_ok = true;
  }
};

struct qs_batch {
  int count = 0;
  bool dbl = false;
  int nparams = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<const qs_circuit*> circs;  // borrowed: they must outlive the batch
  std::vector<const qs_obs*> obs;
  std::vector<TuneOpts> opts;            // per instance (the circuit's, or the batch tuner's choice)
  std::vector<BatchInst> insts;
  std::vector<PassGeom> geoms, geoms_adj;
  // launch lists: forward levels, adjoint levels (item offset, count, ctrl),
  // and the chunk items of initialisation and energy
  struct Level {
    int off, cnt;
    bool ctrl;
  };
  std::vector<Level> fwd, adj;
  int chunk_off = 0, nchunks = 0;
  DBuf d_insts, d_geoms, d_geoms_adj, d_ops, d_sops, d_stages, d_matc, d_phases, d_phlist, d_dpool, d_btab, d_qtab, d_qang, d_ctab;
  DBuf d_terms, d_slot_pidx, d_op_inst, d_items, d_states, d_params, d_gpart, d_slot_sum, d_epart, d_energies,
      d_grads;
  double* h_params = nullptr;
  double* h_energies = nullptr;
  double* h_grads = nullptr;
  BatchArgs args;
  hipGraph_t graph[2] = {nullptr, nullptr};  // [0] energies only, [1] energies and gradients
  hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

void check_state(const qs_state* s) {
  if (!s) fail(QS_E_INVALID, "null state");
}

int max_qubits(qs_dtype dt) { return dt == QS_C128 ? QS_MAX_QUBITS_C128 : QS_MAX_QUBITS_C64; }

void check_dtype(qs_dtype dt) {
  if (dt != QS_C64 && dt != QS_C128) fail(QS_E_INVALID, "dtype must be QS_C64 or QS_C128");
}

void check_mem(size_t bytes) {
  const char* cap = std::getenv("QS_MEM_LIMIT_BYTES");
  if (cap && *cap) {
    const unsigned long long c = std::strtoull(cap, nullptr, 10);
    if (bytes > c) fail(QS_E_NOMEM, "state exceeds QS_MEM_LIMIT_BYTES");
  }
}

void ensure_plan(qs_circuit* c, bool dbl, hipStream_t s) {
  if (!c->planned || c->plan_dbl != dbl) {
    c->hc.plan = plan_circuit(c->hc, c->hc.opts, dbl);
    c->planned = true;
    c->plan_dbl = dbl;
    c->dev_ok = false;
  }
  if (!c->dev_ok) {
    c->dev.load(c->hc.plan, s);
    c->slot_pidx.assign(c->hc.plan.ngrad_slots, -1);
    for (const Pass& p : c->hc.plan.passes)
      for (const TileOp& op : p.ops)
        if (op.kind == OP_ROT && op.gslot >= 0) c->slot_pidx[op.gslot] = op.pidx;
    c->dev_ok = true;
  }
}

// Run every pass of a device plan on a state (forward) or on two states
// (adjoint: reversed order, gradient partials).
void run_passes(const DevPlanBuf& dp, const Plan& plan, bool dbl, void* psi, void* lam, const double* params,
                const double* scales, double* gpart, hipStream_t s) {
  const int np = (int)plan.passes.size();
  if (dp.has_rot && params) hipck(launch_rot_mats(dbl, dp.view, params, s), "rotation matrices");
  if (dp.has_scaled && scales) hipck(launch_phase_tabs(dbl, dp.view, scales, s), "phase factors");
  for (int k = 0; k < np; ++k) {
    const int i = lam ? np - 1 - k : k;
    const Pass& ps = plan.passes[i];
    if (ps.kind == PASS_PERM) {
      ProfScope pr(2, s);
      hipck(launch_perm_pass(dbl, psi, ps.geom, ps.sigma.data(), s), "perm pass");
      if (lam) hipck(launch_perm_pass(dbl, lam, ps.geom, ps.sigma.data(), s), "perm pass");
    } else if (ps.kind == PASS_MFMA) {
      ProfScope pr(3, s);
      // a fused pass holds two blocks on disjoint bits; they commute, so the
      // adjoint un-applies both in the same launch
      const TileOp& op = ps.ops[0];
      const TileOp* op2 = ps.ops.size() > 1 ? &ps.ops[1] : nullptr;
      const int inv = lam ? (1 << (2 * op.k)) : 0;
      const double* m = dp.view.mat + 2 * (op.mat + inv);
      const double* m2 = op2 ? dp.view.mat + 2 * (op2->mat + inv) : nullptr;
      const int* tl2 = op2 ? op2->b : nullptr;
      hipck(launch_mfma_pass(dbl, psi, ps.geom, op.b, op.k, m, tl2, m2, s), "mfma pass");
      if (lam) hipck(launch_mfma_pass(dbl, lam, ps.geom, op.b, op.k, m, tl2, m2, s), "mfma pass");
    } else {
      ProfScope pr(lam ? 7 : 0, s);
      hipck(launch_tile_pass(dbl, psi, lam, lam ? dp.geoms_adj[i] : dp.geoms[i], dp.view, params, scales, gpart, s),
            "tile pass");
    }
  }
}

std::vector<cd> read_matrix(const double* mat, int k) {
  const int d = 1 << k;
  std::vector<cd> m(size_t(d) * d);
  for (int i = 0; i < d * d; ++i) m[i] = cd(mat[2 * i], mat[2 * i + 1]);
  return m;
}

Gate make_gate(int n, const double* mat, int k, const int* targets, int nctrl, const int* controls) {
  if (!mat) fail(QS_E_INVALID, "null matrix");
  std::string err = validate_gate(n, k, targets, nctrl, controls);
  if (!err.empty()) fail(QS_E_INVALID, err);
  Gate g;
  g.k = k;
  for (int i = 0; i < k; ++i) g.tq[i] = targets[i];
  for (int i = 0; i < nctrl; ++i) g.cq.push_back(controls[i]);
  g.mat = read_matrix(mat, k);
  for (const cd& v : g.mat)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) fail(QS_E_INVALID, "non-finite matrix entry");
  return g;
}

double* scratch_doubles(qs_state* s, size_t count) {
  s->scratch.ensure(count * sizeof(double));
  return s->scratch.as<double>();
}

double download_scalar(const double* dev, hipStream_t s) {
  double v = 0;
  hipck(hipMemcpyAsync(&v, dev, sizeof(double), hipMemcpyDeviceToHost, s), "download");
  hipck(hipStreamSynchronize(s), "hipStreamSynchronize");
  return v;
}

// Expectation into dev_out[0] (device), asynchronous.
// sum over the observable's parts (polynomial diagonal, tile sets), each
// leaving one partial per workgroup in its own kGridMax-long slot; with lam,
// also lambda = H psi.  Fixed-order sums: the result is deterministic.
// Partial-sum slots of an observable's passes: one for the diagonal
// polynomial, one per tile set, one per far group.
int obs_slots(const qs_obs* o) {
  return (o->poly.empty() ? 0 : 1) + (int)o->sets.size() + (int)o->far.size();
}
// doubles of scratch that pauli_pass needs: per slot kGridMax partials, then
// the slot sums
size_t pauli_scratch_doubles(const qs_obs* o) {
  const size_t nslot = (size_t)std::max(obs_slots(o), 1);
  return (nslot + 1) * kGridMax + nslot + 8;
}

void pauli_pass(qs_state* s, qs_obs* o, void* lam, double* dev_out, double* part) {
  o->to_device(s->stream);
  const bool poly = !o->poly.empty();
  const int nslot = obs_slots(o);
  double* slots = part + size_t(nslot) * kGridMax;
  hipck(launch_zero(part, int64_t(std::max(nslot, 1)) * kGridMax, s->stream), "zero");
  int k = 0;
  if (poly) {
    if (lam)
      hipck(launch_hpsi_poly(s->dbl(), s->ptr, lam, s->n, o->dpoly.as<double>(), o->delo.as<double>(), part,
                             s->stream),
            "H psi (diagonal)");
    else
      hipck(launch_expect_poly(s->dbl(), s->ptr, s->n, o->dpoly.as<double>(), o->delo.as<double>(), part, s->stream),
            "expectation (diagonal)");
    ++k;
  } else if (lam && o->sets.empty() && o->far.empty()) {
    // an observable with no terms: lambda = 0 (one double per complex64, two per complex128)
    hipck(launch_zero(static_cast<double*>(lam), int64_t(1) << (s->n + (s->dbl() ? 1 : 0)), s->stream), "zero");
  }
  bool written = poly;  // lambda holds a first part
  for (size_t si = 0; si < o->sets.size(); ++si, ++k) {
    PauliSet ps = o->sets[si];
    ps.first = (lam && !written) ? 1 : 0;
    written = true;
    hipck(launch_pauli_set(s->dbl(), s->ptr, lam, ps, o->dtgroups.as<PauliGroupTile>(),
                           o->dtterms.as<PauliTermTile>(), part + size_t(k) * kGridMax, s->stream),
          "Pauli tile set");
  }
  for (size_t fi = 0; fi < o->far.size(); ++fi, ++k) {
    const int g = o->far[fi];
    hipck(launch_pauli_far(s->dbl(), s->ptr, lam, s->n, o->flips[g], o->dterms.as<PauliTermDev>() + o->goff[g],
                           o->goff[g + 1] - o->goff[g], (lam && !written) ? 1 : 0, part + size_t(k) * kGridMax,
                           s->stream),
          "Pauli group");
    written = true;
  }
  hipck(launch_slot_sums(part, std::max(nslot, 1), kGridMax, kGridMax, slots, s->stream), "slot sums");
  hipck(launch_final_sum(slots, std::max(nslot, 1), dev_out, s->stream), "final sum");
}

void expectation_dev(qs_state* s, qs_obs* o, double* dev_out) {
  ProfScope pr(5, s->stream);
  pauli_pass(s, o, nullptr, dev_out, scratch_doubles(s, pauli_scratch_doubles(o)));
}

// A device double for a synchronous result, placed past the scratch that
// pauli_pass uses (the state's scratch is sized once for both, so the pass
// does not reallocate it under the result).
double* expect_result_slot(qs_state* s, const qs_obs* o) {
  const size_t need = pauli_scratch_doubles(o);
  return scratch_doubles(s, need + 8) + need;
}

// Z_p = 1 - 2 x_p on index bit p, so a diagonal group of terms with at most
// two Z factors is c + sum mu_p x_p + sum_{p<q} lam_pq x_p x_q.
void diag_poly(qs_obs* o) {
  const int n = o->n;
  if (o->flips.empty() || o->flips[0] != 0) return;  // groups are sorted: flip 0 first
  std::vector<double> P(size_t(1) + n + size_t(n) * n, 0.0);
  double* mu = P.data() + 1;
  double* lam = P.data() + 1 + n;
  for (int t = o->goff[0]; t < o->goff[1]; ++t) {
    const PauliTermDev& T = o->terms[t];
    const int w = __builtin_popcountll(T.zy);
    if (w > 2) return;
    const double c = T.coeff;
    P[0] += c;
    if (w >= 1) {
      const int p = __builtin_ctzll(T.zy);
      mu[p] -= 2 * c;
      if (w == 2) {
        const int q = 63 - __builtin_clzll(T.zy);
        mu[q] -= 2 * c;
        lam[p * n + q] += 4 * c;
        lam[q * n + p] += 4 * c;
      }
    }
  }
  const int lb = n < 12 ? n : 12;
  std::vector<double> E(size_t(1) << lb, 0.0);
  for (int j = 0; j < (1 << lb); ++j) {
    double e = 0.0;
    for (int p = 0; p < lb; ++p) {
      if (!((j >> p) & 1)) continue;
      e += mu[p];
      for (int q = p + 1; q < lb; ++q)
        if ((j >> q) & 1) e += lam[p * n + q];
    }
    E[j] = e;
  }
  o->poly = std::move(P);
  o->elo = std::move(E);
}

// Pack the groups not handled by the polynomial path into tile sets: each set
// has the low L = min(n, 6) bits and up to 6 high bits, enough to hold every
// flip bit of its groups; a pass over the state evaluates the whole set.
void pauli_sets(qs_obs* o) {
  const int n = o->n;
  const int L = std::min(n, 6);
  const int Hmax = std::min(n - L, kPauliMaxH);
  std::vector<int> todo;
  for (int g = 0; g < (int)o->flips.size(); ++g) {
    if (o->flips[g] == 0 && !o->poly.empty()) continue;
    if (__builtin_popcountll(o->flips[g] >> L) > Hmax) o->far.push_back(g);
    else todo.push_back(g);
  }
  // groups with the same high flip bits next to each other
  std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) { return (o->flips[a] >> L) < (o->flips[b] >> L); });
  size_t i = 0;
  while (i < todo.size()) {
    std::set<int> hsel;
    std::vector<int> members;
    for (; i < todo.size(); ++i) {
      std::set<int> u = hsel;
      for (uint64_t f = o->flips[todo[i]] >> L; f; f &= f - 1) u.insert(L + __builtin_ctzll(f));
      if ((int)u.size() > Hmax) break;
      hsel = u;
      members.push_back(todo[i]);
    }
    if (members.empty()) fail(QS_E_STATE, "internal: a Pauli flip mask does not fit a tile");
    for (int b = L; b < n && (int)hsel.size() < Hmax; ++b) hsel.insert(b);  // fill to a full tile
    PauliSet ps;
    std::memset(&ps, 0, sizeof ps);
    ps.n = n;
    ps.L = L;
    ps.H = (int)hsel.size();
    ps.first = 0;
    int k = 0;
    int local[64];
    for (int b = 0; b < 64; ++b) local[b] = b < L ? b : -1;
    for (int b : hsel) {
      local[b] = L + k;
      ps.hbits[k++] = b;
    }
    ps.g0 = (int)o->tgroups.size();
    ps.ng = (int)members.size();
    for (int g : members) {
      PauliGroupTile G;
      G.fl = 0;
      for (uint64_t f = o->flips[g]; f; f &= f - 1) G.fl |= 1u << local[__builtin_ctzll(f)];
      G.t0 = (int)o->tterms.size();
      G.nt = o->goff[g + 1] - o->goff[g];
      G.pad = 0;
      for (int t = o->goff[g]; t < o->goff[g + 1]; ++t) {
        const PauliTermDev& T = o->terms[t];
        PauliTermTile tt;
        tt.zo = 0;
        tt.zl = 0;
        for (uint64_t z = T.zy; z; z &= z - 1) {
          const int b = __builtin_ctzll(z);
          if (local[b] >= 0) tt.zl |= 1u << local[b];
          else tt.zo |= 1ull << b;
        }
        tt.ny4 = T.ny4;
        tt.coeff = T.coeff;
        o->tterms.push_back(tt);
      }
      o->tgroups.push_back(G);
    }
    o->sets.push_back(ps);
  }
}

qs_obs* make_pauli_obs(int n, int nterms, const double* coeffs, const char* const* strings) {
  std::map<uint64_t, std::vector<PauliTermDev>> groups;
  for (int t = 0; t < nterms; ++t) {
    const char* w = strings[t];
    if (!w) fail(QS_E_INVALID, "null Pauli string");
    if ((int)std::strlen(w) != n) fail(QS_E_INVALID, "Pauli string length must equal n");
    if (!std::isfinite(coeffs[t])) fail(QS_E_INVALID, "non-finite coefficient");
    uint64_t flip = 0, zy = 0;
    int ny = 0;
    for (int q = 0; q < n; ++q) {
      const uint64_t bit = 1ull << (n - 1 - q);
      switch (w[q]) {
        case 'I': break;
        case 'X': flip |= bit; break;
        case 'Y': flip |= bit; zy |= bit; ++ny; break;
        case 'Z': zy |= bit; break;
        default: fail(QS_E_INVALID, std::string("bad Pauli character '") + w[q] + "'");
      }
    }
    PauliTermDev d;
    d.zy = zy;
    d.ny4 = ny & 3;
    d.pad = 0;
    d.coeff = coeffs[t];
    groups[flip].push_back(d);
  }
  auto* o = new qs_obs;
  o->n = n;
  o->goff.push_back(0);
  for (auto& kv : groups) {
    o->flips.push_back(kv.first);
    o->terms.insert(o->terms.end(), kv.second.begin(), kv.second.end());
    o->goff.push_back((int)o->terms.size());
  }
  diag_poly(o);
  pauli_sets(o);
  return o;
}

}  // namespace

// =========================================================================
extern "C" {

const char* qs_version(void) { return "qsim-mi355x 0.1.0 (gfx950)"; }
const char* qs_last_error(void) { return g_err.c_str(); }

qs_status qs_state_create(int32_t n, qs_dtype dt, void* stream, qs_state** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    check_dtype(dt);
    if (n < 1 || n > max_qubits(dt)) fail(QS_E_INVALID, "n out of range");
    auto s = std::make_unique<qs_state>();
    s->n = n;
    s->dt = dt;
    s->stream = (hipStream_t)stream;
    check_mem(s->bytes());
    check_device();
    size_t fr = 0, tot = 0;
    hipck(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    if (s->bytes() > fr) fail(QS_E_NOMEM, "state larger than free device memory");
    hipck(hipMalloc(&s->ptr, s->bytes()), "hipMalloc(state)");
    s->owned = true;
    hipck(launch_set_basis(s->dbl(), s->ptr, n, 0, s->stream), "init");
    *out = s.release();
  });
}

qs_status qs_state_wrap(void* dev_ptr, int32_t n, qs_dtype dt, void* stream, qs_state** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    check_dtype(dt);
    if (!dev_ptr) fail(QS_E_INVALID, "null device pointer");
    if (n < 1 || n > max_qubits(dt)) fail(QS_E_INVALID, "n out of range");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 16) fail(QS_E_INVALID, "device pointer not 16-byte aligned");
    check_device();
    auto s = std::make_unique<qs_state>();
    s->n = n;
    s->dt = dt;
    s->ptr = dev_ptr;
    s->owned = false;
    s->stream = (hipStream_t)stream;
    *out = s.release();
  });
}

qs_status qs_state_destroy(qs_state* s) {
  return guard([&] {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    if (s->owned && s->ptr) (void)hipFree(s->ptr);
    delete s;
  });
}

qs_status qs_state_info(const qs_state* s, int32_t* n, qs_dtype* dt, void** dev_ptr) {
  return guard([&] {
    check_state(s);
    if (n) *n = s->n;
    if (dt) *dt = s->dt;
    if (dev_ptr) *dev_ptr = s->ptr;
  });
}

qs_status qs_state_set_basis(qs_state* s, uint64_t x) {
  return guard([&] {
    check_state(s);
    if (x >> s->n) fail(QS_E_INVALID, "basis index out of range");
    hipck(launch_set_basis(s->dbl(), s->ptr, s->n, x, s->stream), "set_basis");
  });
}

qs_status qs_state_set_plus(qs_state* s) {
  return guard([&] {
    check_state(s);
    hipck(launch_set_plus(s->dbl(), s->ptr, s->n, s->stream), "set_plus");
  });
}

qs_status qs_state_upload(qs_state* s, const void* host_src) {
  return guard([&] {
    check_state(s);
    if (!host_src) fail(QS_E_INVALID, "null host pointer");
    hipck(hipMemcpyAsync(s->ptr, host_src, s->bytes(), hipMemcpyHostToDevice, s->stream), "upload");
    hipck(hipStreamSynchronize(s->stream), "sync");
  });
}

qs_status qs_state_download(const qs_state* s, void* host_dst) {
  return guard([&] {
    check_state(s);
    if (!host_dst) fail(QS_E_INVALID, "null host pointer");
    hipck(hipMemcpyAsync(host_dst, s->ptr, s->bytes(), hipMemcpyDeviceToHost, s->stream), "download");
    hipck(hipStreamSynchronize(s->stream), "sync");
  });
}

qs_status qs_state_copy(qs_state* dst, const qs_state* src) {
  return guard([&] {
    check_state(dst);
    check_state(src);
    if (dst->n != src->n || dst->dt != src->dt) fail(QS_E_STATE, "state shapes differ");
    hipck(launch_copy(dst->ptr, src->ptr, (int64_t)dst->bytes(), dst->stream), "copy");
  });
}

qs_status qs_state_sync(const qs_state* s) {
  return guard([&] {
    check_state(s);
    hipck(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  });
}

qs_status qs_gate_matrix(const char* name, double theta, double* out, int32_t* k_out) {
  return guard([&] {
    if (!name || !out) fail(QS_E_INVALID, "null argument");
    std::vector<cd> m;
    const int k = named_gate(name, theta, m);
    if (!k) fail(QS_E_INVALID, std::string("unknown gate ") + name);
    for (size_t i = 0; i < m.size(); ++i) {
      out[2 * i] = m[i].real();
      out[2 * i + 1] = m[i].imag();
    }
    if (k_out) *k_out = k;
  });
}

// Kraus operators of the textbook one-qubit channels (Nielsen & Chuang,
// Sec. 8.3): depolarising rho -> (1 - p) rho + p I/2, amplitude damping with
// decay probability p, phase damping with parameter p, bit and phase flip
// with probability p.
qs_status qs_channel_kraus(const char* name, double p, double* out, int32_t* nkraus_out, int32_t* k_out) {
  return guard([&] {
    if (!name || !out || !nkraus_out) fail(QS_E_INVALID, "null argument");
    if (!(p >= 0.0 && p <= 1.0)) fail(QS_E_INVALID, "channel parameter must be in [0, 1]");
    const std::string nm(name);
    std::vector<std::array<cd, 4>> ks;
    const cd z(0, 0), one(1, 0), im(0, 1);
    if (nm == "depolarizing") {
      const double a = std::sqrt(1.0 - 0.75 * p), b = std::sqrt(0.25 * p);
      ks = {{a * one, z, z, a * one}, {z, b * one, b * one, z}, {z, -b * im, b * im, z}, {b * one, z, z, -b * one}};
    } else if (nm == "amplitude_damping") {
      ks = {{one, z, z, std::sqrt(1.0 - p) * one}, {z, std::sqrt(p) * one, z, z}};
    } else if (nm == "phase_damping") {
      ks = {{one, z, z, std::sqrt(1.0 - p) * one}, {z, z, z, std::sqrt(p) * one}};
    } else if (nm == "bit_flip") {
      const double a = std::sqrt(1.0 - p), b = std::sqrt(p);
      ks = {{a * one, z, z, a * one}, {z, b * one, b * one, z}};
    } else if (nm == "phase_flip") {
      const double a = std::sqrt(1.0 - p), b = std::sqrt(p);
      ks = {{a * one, z, z, a * one}, {b * one, z, z, -b * one}};
    } else {
      fail(QS_E_INVALID, "unknown channel " + nm);
    }
    for (size_t t = 0; t < ks.size(); ++t)
      for (int i = 0; i < 4; ++i) {
        out[8 * t + 2 * i] = ks[t][i].real();
        out[8 * t + 2 * i + 1] = ks[t][i].imag();
      }
    *nkraus_out = (int32_t)ks.size();
    if (k_out) *k_out = 1;
  });
}

qs_status qs_apply(qs_state* s, const double* mat, int32_t k, const int32_t* targets, int32_t nctrl,
                   const int32_t* controls) {
  return guard([&] {
    check_state(s);
    HostCircuit hc;
    hc.n = s->n;
    hc.gates.push_back(make_gate(s->n, mat, k, targets, nctrl, controls));
    Plan p = plan_circuit(hc, TuneOpts{}, s->dbl());
    s->single.load(p, s->stream);
    run_passes(s->single, p, s->dbl(), s->ptr, nullptr, nullptr, nullptr, nullptr, s->stream);
  });
}

// ---------------------------------------------------------------- circuits
qs_status qs_circuit_create(int32_t n, qs_circuit** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS_C64) fail(QS_E_INVALID, "n out of range");
    auto c = new qs_circuit;
    c->hc.n = n;
    *out = c;
  });
}

qs_status qs_circuit_create_density(int32_t n, qs_circuit** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    if (n < 1 || 2 * n > QS_MAX_QUBITS_C64) fail(QS_E_INVALID, "n out of range (a density matrix needs 2n <= 35)");
    auto c = new qs_circuit;
    c->hc.n = 2 * n;
    c->dens = n;
    *out = c;
  });
}

qs_status qs_circuit_add_gate(qs_circuit* c, const double* mat, int32_t k, const int32_t* targets, int32_t nctrl,
                              const int32_t* controls) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    Gate g = make_gate(c->dens ? c->dens : c->hc.n, mat, k, targets, nctrl, controls);
    if (c->dens) {
      // U rho U^dagger: U on the row qubits, conj(U) on the column qubits
      Gate gc = g;
      for (int i = 0; i < gc.k; ++i) gc.tq[i] += c->dens;
      for (int& q : gc.cq) q += c->dens;
      for (cd& v : gc.mat) v = std::conj(v);
      c->hc.gates.push_back(std::move(g));
      c->hc.gates.push_back(std::move(gc));
    } else {
      c->hc.gates.push_back(std::move(g));
    }
    c->planned = false;
  });
}

qs_status qs_circuit_add_channel(qs_circuit* c, int32_t nkraus, const double* kraus, int32_t k,
                                 const int32_t* targets) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    if (!c->dens) fail(QS_E_STATE, "channels need a density-matrix circuit (qs_circuit_create_density)");
    if (k < 1 || k > 2) fail(QS_E_INVALID, "a channel acts on 1 or 2 qubits");
    if (nkraus < 1 || nkraus > 16) fail(QS_E_INVALID, "nkraus must be in [1, 16]");
    if (!kraus || !targets) fail(QS_E_INVALID, "null Kraus operators or targets");
    std::string err = validate_gate(c->dens, k, targets, 0, nullptr);
    if (!err.empty()) fail(QS_E_INVALID, err);
    const int d = 1 << k, dd = d * d;
    // superoperator S = sum_i K_i (x) conj(K_i) on (row targets, column targets):
    // S[(r, c), (r', c')] = sum_i K_i[r][r'] conj(K_i[c][c'])
    Gate g;
    g.k = 2 * k;
    for (int i = 0; i < k; ++i) {
      g.tq[i] = targets[i];
      g.tq[k + i] = targets[i] + c->dens;
    }
    g.mat.assign(size_t(dd) * dd, cd(0, 0));
    for (int t = 0; t < nkraus; ++t) {
      const std::vector<cd> K = read_matrix(kraus + size_t(t) * 2 * dd, k);
      for (const cd& v : K)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) fail(QS_E_INVALID, "non-finite Kraus entry");
      for (int r = 0; r < d; ++r)
        for (int cc = 0; cc < d; ++cc)
          for (int r2 = 0; r2 < d; ++r2)
            for (int c2 = 0; c2 < d; ++c2)
              g.mat[size_t(r * d + cc) * dd + (r2 * d + c2)] += K[r * d + r2] * std::conj(K[cc * d + c2]);
    }
    c->hc.gates.push_back(std::move(g));
    c->planned = false;
  });
}

qs_status qs_circuit_add_rot(qs_circuit* c, char pauli, int32_t target, int32_t param_index, int32_t nctrl,
                             const int32_t* controls) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    if (pauli != 'X' && pauli != 'Y' && pauli != 'Z') fail(QS_E_INVALID, "pauli must be X, Y or Z");
    if (param_index < 0) fail(QS_E_INVALID, "negative parameter index");
    std::string err = validate_gate(c->dens ? c->dens : c->hc.n, 1, &target, nctrl, controls);
    if (!err.empty()) fail(QS_E_INVALID, err);
    Gate g;
    g.k = 1;
    g.tq[0] = target;
    for (int i = 0; i < nctrl; ++i) g.cq.push_back(controls[i]);
    g.is_rot = true;
    g.pauli = pauli;
    g.pidx = param_index;
    c->hc.gates.push_back(g);
    if (c->dens) {
      // conj(exp(-i theta P/2)) = exp(-i (-theta) P/2) for X and Z (real P),
      // exp(-i theta Y/2) for Y (Y* = -Y)
      g.tq[0] += c->dens;
      for (int& q : g.cq) q += c->dens;
      g.rsign = pauli == 'Y' ? 1 : -1;
      c->hc.gates.push_back(g);
    }
    c->hc.nparams = std::max(c->hc.nparams, param_index + 1);
    c->planned = false;
  });
}

qs_status qs_circuit_compile(qs_circuit* c, const qs_tune* opts) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    TuneOpts o;
    if (opts) {
      if (opts->tile_bits != 0 && (opts->tile_bits < 6 || opts->tile_bits > kMaxTileBits))
        fail(QS_E_INVALID, "tile_bits must be 0 or in [6, 13]");
      if (opts->fuse_k < 0 || opts->fuse_k > 5) fail(QS_E_INVALID, "fuse_k must be in [0, 5]");
      if (opts->low_bits < 0 || opts->low_bits > 8) fail(QS_E_INVALID, "low_bits must be in [0, 8]");
      if (opts->lane_ops != 0 && opts->lane_ops != 1) fail(QS_E_INVALID, "lane_ops must be 0 or 1");
      o.tile_bits = opts->tile_bits;
      o.fuse_k = opts->fuse_k;
      o.use_mfma = opts->use_mfma;
      o.low_bits = opts->low_bits;
      o.lane_ops = opts->lane_ops != 0;
    }
    c->hc.opts = o;
    // plan for complex64 now (host only); a complex128 run replans
    c->hc.plan = plan_circuit(c->hc, o, false);
    c->planned = true;
    c->plan_dbl = false;
    c->dev_ok = false;
  });
}

qs_status qs_circuit_run(qs_circuit* c, qs_state* s, const double* params, int32_t params_on_device) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    check_state(s);
    if (c->hc.n != s->n) fail(QS_E_STATE, "circuit and state sizes differ");
    if (c->hc.nparams > 0 && !params) fail(QS_E_INVALID, "circuit has parameters but params is null");
    ensure_plan(c, s->dbl(), s->stream);
    const double* dpar = nullptr;
    if (c->hc.nparams > 0) {
      if (params_on_device) {
        dpar = params;
      } else {
        c->dparams.ensure(sizeof(double) * c->hc.nparams);
        hipck(hipMemcpyAsync(c->dparams.p, params, sizeof(double) * c->hc.nparams, hipMemcpyHostToDevice,
                             s->stream),
              "params upload");
        dpar = c->dparams.as<double>();
      }
    }
    run_passes(c->dev, c->hc.plan, s->dbl(), s->ptr, nullptr, dpar, nullptr, nullptr, s->stream);
  });
}

qs_status qs_circuit_info(const qs_circuit* c, int32_t* ngates, int32_t* npasses, int32_t* nparams) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    if (ngates) *ngates = (int)c->hc.gates.size();
    if (npasses) *npasses = c->planned ? (int)c->hc.plan.passes.size() : -1;
    if (nparams) *nparams = c->hc.nparams;
  });
}

qs_status qs_circuit_pass_info(const qs_circuit* c, int32_t i, int32_t* kind, int32_t* tile_bits, int32_t* nops) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    if (!c->planned) fail(QS_E_STATE, "circuit not compiled");
    if (i < 0 || i >= (int)c->hc.plan.passes.size()) fail(QS_E_INVALID, "pass index out of range");
    const Pass& p = c->hc.plan.passes[i];
    if (kind) *kind = p.kind;
    if (tile_bits) *tile_bits = p.geom.m;
    if (nops) *nops = (int)p.ops.size();
  });
}

qs_status qs_circuit_schedule(const qs_circuit* c, int32_t* schedule) {
  return guard([&] {
    if (!c || !schedule) fail(QS_E_INVALID, "null argument");
    if (!c->planned) fail(QS_E_STATE, "circuit not compiled");
    *schedule = c->hc.plan.schedule;
  });
}

qs_status qs_circuit_destroy(qs_circuit* c) {
  return guard([&] {
    if (!c) return;
    (void)hipDeviceSynchronize();
    delete c;
  });
}

// ------------------------------------------------------------- observables
qs_status qs_pauli_sum_create(int32_t n, int32_t nterms, const double* coeffs, const char* const* strings,
                              qs_obs** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS_C64) fail(QS_E_INVALID, "n out of range");
    if (nterms < 0) fail(QS_E_INVALID, "negative term count");
    if (nterms > 0 && (!coeffs || !strings)) fail(QS_E_INVALID, "null terms");
    *out = make_pauli_obs(n, nterms, coeffs, strings);
  });
}

qs_status qs_ising_create(int32_t n, const double* J, const double* h, qs_obs** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS_C64) fail(QS_E_INVALID, "n out of range");
    if (!J || !h) fail(QS_E_INVALID, "null J or h");
    std::vector<double> co;
    std::vector<std::string> ws;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        const double v = J[size_t(i) * n + j];
        if (!std::isfinite(v)) fail(QS_E_INVALID, "non-finite J");
        if (v == 0.0) continue;
        std::string w(n, 'I');
        w[i] = w[j] = 'Z';
        co.push_back(v);
        ws.push_back(w);
      }
    for (int i = 0; i < n; ++i) {
      if (!std::isfinite(h[i])) fail(QS_E_INVALID, "non-finite h");
      std::string w(n, 'I');
      w[i] = 'Z';
      co.push_back(h[i]);
      ws.push_back(w);
    }
    std::vector<const char*> pw;
    for (auto& w : ws) pw.push_back(w.c_str());
    qs_obs* o = make_pauli_obs(n, (int)co.size(), co.data(), pw.data());
    o->ising = true;
    o->J.assign(J, J + size_t(n) * n);
    o->h.assign(h, h + n);
    *out = o;
  });
}

qs_status qs_obs_destroy(qs_obs* o) {
  return guard([&] {
    if (!o) return;
    (void)hipDeviceSynchronize();
    delete o;
  });
}

qs_status qs_expectation(const qs_state* cs, const qs_obs* co, double* out) {
  return guard([&] {
    check_state(cs);
    if (!co || !out) fail(QS_E_INVALID, "null argument");
    auto* s = const_cast<qs_state*>(cs);
    auto* o = const_cast<qs_obs*>(co);
    if (o->n != s->n) fail(QS_E_STATE, "observable and state sizes differ");
    const int ng = (int)o->flips.size();
    if (ng == 0) {
      *out = 0.0;
      return;
    }
    double* res = expect_result_slot(s, o);
    expectation_dev(s, o, res);
    *out = download_scalar(res, s->stream);
  });
}

qs_status qs_expectation_async(const qs_state* cs, const qs_obs* co, double* dev_out) {
  return guard([&] {
    check_state(cs);
    if (!co || !dev_out) fail(QS_E_INVALID, "null argument");
    auto* s = const_cast<qs_state*>(cs);
    auto* o = const_cast<qs_obs*>(co);
    if (o->n != s->n) fail(QS_E_STATE, "observable and state sizes differ");
    if (o->flips.empty()) {
      hipck(launch_zero(dev_out, 1, s->stream), "zero");
      return;
    }
    expectation_dev(s, o, dev_out);
  });
}

qs_status qs_expectation_noalloc(const qs_state* cs, const qs_obs* co, double* dev_out) {
  return guard([&] {
    check_state(cs);
    if (!co || !dev_out) fail(QS_E_INVALID, "null argument");
    auto* s = const_cast<qs_state*>(cs);
    auto* o = const_cast<qs_obs*>(co);
    if (o->n != s->n) fail(QS_E_STATE, "observable and state sizes differ");
    if (o->flips.empty()) {
      hipck(launch_zero(dev_out, 1, s->stream), "zero");
      return;
    }
    if (!o->dev_ok)
      fail(QS_E_STATE,
           "the observable's tables are not on the device: one qs_expectation or qs_expectation_async call with it "
           "uploads them");
    const int nslot = obs_slots(o);
    if (nslot > kNoAllocMaxSlots || (int64_t)pauli_scratch_doubles(o) > kNoAllocScratchDoubles)
      fail(QS_E_INVALID, "observable needs " + std::to_string(nslot) + " reduction slots; the fixed workspace holds " +
                             std::to_string(kNoAllocMaxSlots));
    double* ws = nullptr;
    hipck(noalloc_scratch(&ws), "hipGetSymbolAddress(scratch)");
    pauli_pass(s, o, nullptr, dev_out, ws);
  });
}

qs_status qs_norm2(const qs_state* cs, double* out) {
  return guard([&] {
    check_state(cs);
    if (!out) fail(QS_E_INVALID, "null output");
    auto* s = const_cast<qs_state*>(cs);
    double* part = scratch_doubles(s, kGridMax + 8);
    ProfScope pr(5, s->stream);
    hipck(launch_sumsq(s->dbl(), s->ptr, s->n, part, s->stream), "norm");
    *out = download_scalar(part + kGridMax, s->stream);
  });
}

// ------------------------------------------------------- density matrices
qs_status qs_density_set_pure(qs_state* rho, const qs_state* psi) {
  return guard([&] {
    check_state(rho);
    check_state(psi);
    if (rho->n != 2 * psi->n || rho->dt != psi->dt)
      fail(QS_E_STATE, "rho must have 2n qubits of psi's n and the same dtype");
    ProfScope pr(9, rho->stream);
    if (psi->stream != rho->stream) hipck(hipStreamSynchronize(psi->stream), "hipStreamSynchronize");
    hipck(launch_outer(rho->dbl(), rho->ptr, psi->ptr, psi->n, rho->stream), "outer product");
  });
}

qs_status qs_density_expectation(const qs_state* crho, const qs_obs* co, double* out) {
  return guard([&] {
    check_state(crho);
    if (!co || !out) fail(QS_E_INVALID, "null argument");
    if (crho->n % 2 != 0 || co->n * 2 != crho->n) fail(QS_E_STATE, "rho must have twice the observable's qubits");
    auto* s = const_cast<qs_state*>(crho);
    auto* o = const_cast<qs_obs*>(co);
    o->to_device(s->stream);
    double* part = scratch_doubles(s, kGridMax + 8);
    ProfScope pr(5, s->stream);
    hipck(launch_dens_pauli(s->dbl(), s->ptr, o->n, o->dflips.as<uint64_t>(), o->dgoff.as<int32_t>(),
                            o->dterms.as<PauliTermDev>(), (int)o->flips.size(), part, part + kGridMax, s->stream),
          "Tr(H rho)");
    *out = download_scalar(part + kGridMax, s->stream);
  });
}

qs_status qs_density_trace(const qs_state* crho, double* out) {
  return guard([&] {
    check_state(crho);
    if (!out) fail(QS_E_INVALID, "null output");
    if (crho->n % 2 != 0) fail(QS_E_STATE, "a density matrix has an even number of vector qubits");
    auto* s = const_cast<qs_state*>(crho);
    double* part = scratch_doubles(s, kGridMax + 8);
    ProfScope pr(5, s->stream);
    hipck(launch_dens_pauli(s->dbl(), s->ptr, s->n / 2, nullptr, nullptr, nullptr, 0, part, part + kGridMax,
                            s->stream),
          "Tr(rho)");
    *out = download_scalar(part + kGridMax, s->stream);
  });
}

// ---------------------------------------------------------------- sampling
qs_status qs_sample(const qs_state* cs, int32_t m, const int32_t* qubits, int64_t shots, uint64_t seed,
                    const double* uniforms, int64_t* out) {
  return guard([&] {
    check_state(cs);
    auto* s = const_cast<qs_state*>(cs);
    if (m < 1 || m > s->n || m > 63) fail(QS_E_INVALID, "m must be in [1, min(n, 63)]");
    if (!qubits) fail(QS_E_INVALID, "null qubits");
    if (shots < 0) fail(QS_E_INVALID, "negative shots");
    if (shots > 0 && !out) fail(QS_E_INVALID, "null output");
    uint64_t seen = 0;
    std::vector<int> pos(m);
    for (int i = 0; i < m; ++i) {
      const int q = qubits[i];
      if (q < 0 || q >= s->n) fail(QS_E_INVALID, "qubit index out of range");
      if ((seen >> q) & 1) fail(QS_E_INVALID, "duplicate measured qubit");
      seen |= 1ull << q;
      pos[i] = s->n - 1 - q;
    }
    if (uniforms)
      for (int64_t j = 0; j < shots; ++j)
        if (!(uniforms[j] >= 0.0 && uniforms[j] < 1.0)) fail(QS_E_INVALID, "uniforms must lie in [0, 1)");
    if (shots == 0) return;
    const int64_t nb = sample_nblocks(s->n);
    const int64_t nc = sample_nchunks(s->n);
    // layout of scratch2: blocksums[nb] | prefix[nb+1] | chunks[2 nc + 1] | uniforms[shots] | out[shots]
    const size_t need =
        sizeof(double) * (2 * nb + 1 + 2 * nc + 1 + (uniforms ? shots : 0)) + sizeof(int64_t) * shots + 64;
    s->scratch2.ensure(need);
    double* bs = s->scratch2.as<double>();
    double* pre = bs + nb;
    double* chunks = pre + nb + 1;
    double* du = chunks + 2 * nc + 1;
    int64_t* dout = reinterpret_cast<int64_t*>(du + (uniforms ? shots : 0));
    if (uniforms)
      hipck(hipMemcpyAsync(du, uniforms, sizeof(double) * shots, hipMemcpyHostToDevice, s->stream), "uniforms");
    {
      ProfScope pr(6, s->stream);
      hipck(launch_sample(s->dbl(), s->ptr, s->n, bs, pre, chunks, shots, seed, uniforms ? du : nullptr, pos.data(), m,
                          dout, s->stream),
            "sample");
    }
    hipck(hipMemcpyAsync(out, dout, sizeof(int64_t) * shots, hipMemcpyDeviceToHost, s->stream), "download");
    hipck(hipStreamSynchronize(s->stream), "sync");
  });
}

// ---------------------------------------------------------------- adiabatic
}  // extern "C"

namespace {

int64_t step_count(double T, double dt) {
  if (!(T > 0) || !(dt > 0) || !std::isfinite(T) || !std::isfinite(dt)) fail(QS_E_INVALID, "T and dt must be > 0");
  const double kf = T / dt;
  const int64_t K = (int64_t)std::llround(kf);
  if (K < 1 || std::fabs(kf - (double)K) > 1e-9 * std::max(1.0, kf)) fail(QS_E_INVALID, "T/dt must be an integer");
  return K;
}

// Trotter steps k0 .. k1-1 of the schedule s_k = (k + 1/2) dt / T, each with
// its half rotation layers: the segment opens with the first half layer of
// step k0 and closes with the second half layer of step k1 - 1.  Blocks of S
// steps share passes (the last pass of a step carries the next step's
// rotations on its tile bits): up to 16 steps form one block, longer segments
// replay blocks of 8, and the last block also carries the closing layer.
// Plans depend only on the block length for a given H1 and precision; they
// are cached on the observable.

void trotter_segment(qs_state* s, const PhasePoly& E, double T, double dt, int64_t k0, int64_t k1, TrotterPlans& tp) {
  const int n = s->n;
  const bool dbl = s->dbl();
  const int64_t K = k1 - k0;
  const int S = (int)(K <= 16 ? K : 8);
  const int64_t rem = K % S;
  const int64_t nfull = K / S - (rem ? 0 : 1);  // blocks before the last segment
  const int L = (int)(rem ? rem : S);           // steps of the last segment
  auto get = [&](int steps, bool final) -> std::pair<Plan, std::unique_ptr<DevPlanBuf>>& {
    auto key = std::make_pair(steps, final);
    auto it = tp.m.find(key);
    if (it == tp.m.end()) {
      Plan p = plan_trotter(n, dbl, TuneOpts{}, &E, steps, final);
      auto d = std::make_unique<DevPlanBuf>();
      d->load(p, s->stream);
      it = tp.m.emplace(key, std::make_pair(std::move(p), std::move(d))).first;
    }
    return it->second;
  };
  std::vector<double> ang(K + 1), scl(K);
  auto sk = [&](int64_t k) { return (double(k) + 0.5) * dt / T; };
  for (int64_t j = 0; j <= K; ++j) {
    double a = 0.0;
    if (j < K) a += -(1.0 - sk(k0 + j)) * dt;
    if (j > 0) a += -(1.0 - sk(k0 + j - 1)) * dt;
    ang[j] = a;
  }
  for (int64_t j = 0; j < K; ++j) scl[j] = -sk(k0 + j) * dt;
  DBuf& dang = tp.ang;
  DBuf& dscl = tp.scl;
  upload(dang, ang, s->stream);
  upload(dscl, scl, s->stream);
  if (nfull > 0) {
    auto& blk = get(S, false);
    for (int64_t b = 0; b < nfull; ++b)
      run_passes(*blk.second, blk.first, dbl, s->ptr, nullptr, dang.as<double>() + b * S, dscl.as<double>() + b * S,
                 nullptr, s->stream);
  }
  // the last segment: angle slots K - L .. K (the closing layer is slot L), scales K - L .. K - 1
  auto& last = get(L, true);
  run_passes(*last.second, last.first, dbl, s->ptr, nullptr, dang.as<double>() + (K - L), dscl.as<double>() + (K - L),
             nullptr, s->stream);
  // the host angle and scale arrays end with this call, and the next segment
  // rewrites dang / dscl: the copies and the passes that read them must be done
  hipck(hipStreamSynchronize(s->stream), "sync");
}

// Reduced density matrix of qubits 0..a-1 (or of the rest, the smaller side)
// as a Gram matrix on the GPU, its eigenvalues on the host.
double entropy_dev(qs_state* s, int a) {
  const int n = s->n, b = n - a;
  const int small = std::min(a, b), big = std::max(a, b);
  if (small > 10) fail(QS_E_UNSUPPORTED, "entropy needs min(a, n - a) <= 10");
  const int d = 1 << small;
  const int64_t K = int64_t(1) << big;
  const int64_t cols = int64_t(1) << b;  // psi[i * 2^b + j]: i the first a qubits, j the rest
  // rho_A = M M^dagger (a <= b) or rho_B = M^T conj(M) (a > b): same nonzero spectrum
  int64_t ars, acs, brs, bcs;
  if (a <= b) {
    ars = cols; acs = 1; brs = 1; bcs = cols;
  } else {
    ars = 1; acs = cols; brs = cols; bcs = 1;
  }
  const int tiles = ((d + 63) / 64) * ((d + 63) / 64);
  int want = std::max(1, 1024 / tiles);
  want = (int)std::min<int64_t>(want, std::max<int64_t>(1, K / 64));
  const int splits = zgemm_splits(K, want);
  const size_t dd = size_t(d) * d;
  s->scratch2.ensure((splits + 1) * dd * 16);
  double* part = s->scratch2.as<double>();
  double* G = part + 2 * splits * dd;
  hipck(launch_zgemm(s->dbl(), s->ptr, ars, acs, 0, s->ptr, brs, bcs, 1, d, d, K, want, part, 1.0, 0.0, 0,
                     s->stream),
        "Gram matrix");
  hipck(launch_split_sum(part, splits, (int64_t)dd, G, s->stream), "Gram sum");
  std::vector<cd> h(dd);
  hipck(hipMemcpyAsync(h.data(), G, dd * 16, hipMemcpyDeviceToHost, s->stream), "download");
  hipck(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  return entropy_of_eigenvalues(hermitian_eigenvalues(d, std::move(h)));
}

void check_callbacks(const qs_callbacks* cb, const qs_state* s) {
  if (!cb || cb->every <= 0) return;
  if (cb->energy && (!cb->energies || cb->energy->n != s->n)) fail(QS_E_INVALID, "energy callback: bad observable or null output");
  if (cb->entropy_qubits > 0) {
    if (!cb->entropies) fail(QS_E_INVALID, "entropy callback: null output");
    if (cb->entropy_qubits >= s->n) fail(QS_E_INVALID, "entropy callback: entropy_qubits must be in [1, n-1]");
    if (std::min(cb->entropy_qubits, s->n - cb->entropy_qubits) > 10)
      fail(QS_E_UNSUPPORTED, "entropy needs min(a, n - a) <= 10");
  }
  if (cb->entropy_qubits < 0) fail(QS_E_INVALID, "negative entropy_qubits");
}

void run_callbacks(qs_state* s, const qs_callbacks* cb, int64_t idx) {
  if (cb->energy) {
    auto* o = const_cast<qs_obs*>(cb->energy);
    double* res = expect_result_slot(s, o);
    expectation_dev(s, o, res);
    cb->energies[idx] = download_scalar(res, s->stream);
  }
  if (cb->entropy_qubits > 0) cb->entropies[idx] = entropy_dev(s, cb->entropy_qubits);
}

double coeff_norm(const qs_obs* o) {
  double t = 0.0;
  for (const PauliTermDev& d : o->terms) t += std::fabs(d.coeff);
  return t;
}

// One state-sized device vector viewed as a state (same n, dtype, stream).
struct VecView {
  qs_state v;
  VecView(const qs_state* s, void* p) {
    v.n = s->n;
    v.dt = s->dt;
    v.ptr = p;
    v.owned = false;
    v.stream = s->stream;
  }
};

// lambda = H(u) y = (1 - u) h0 y + u h1 y, then k = -i lambda (in place)
void rk_rhs(qs_state* s, qs_obs* h0, qs_obs* h1, void* y, void* k, void* tmp, double u, double* part, double* res) {
  VecView yv(s, y);
  pauli_pass(&yv.v, h0, k, res, part);
  pauli_pass(&yv.v, h1, tmp, res, part);
  LinComb lc{};
  lc.nin = 2;
  lc.in[0] = k;
  lc.cre[0] = 0.0;
  lc.cim[0] = -(1.0 - u);
  lc.in[1] = tmp;
  lc.cre[1] = 0.0;
  lc.cim[1] = -u;
  hipck(launch_lincomb(s->dbl(), k, s->n, lc, s->stream), "lincomb");
}

}  // namespace

extern "C" {

qs_status qs_adiabatic_run(qs_state* s, const qs_obs* h1, double T, double dt, int32_t order,
                           double* energy_out) {
  return qs_adiabatic_run_callbacks(s, h1, T, dt, order, nullptr, energy_out);
}

qs_status qs_adiabatic_run_callbacks(qs_state* s, const qs_obs* h1, double T, double dt, int32_t order,
                                     const qs_callbacks* cb, double* energy_out) {
  return guard([&] {
    check_state(s);
    if (!h1 || !h1->ising) fail(QS_E_INVALID, "h1 must be an Ising observable");
    if (h1->n != s->n) fail(QS_E_STATE, "observable and state sizes differ");
    if (order != 2) fail(QS_E_UNSUPPORTED, "only the second-order split is implemented");
    const int64_t K = step_count(T, dt);
    check_callbacks(cb, s);
    const PhasePoly E = ising_poly(s->n, h1->J.data(), h1->h.data());
    TrotterPlans& tp = const_cast<qs_obs*>(h1)->trotter[s->dbl() ? 1 : 0];
    const int64_t every = (cb && cb->every > 0) ? cb->every : K;
    int64_t idx = 0;
    for (int64_t k0 = 0; k0 < K; k0 += every) {
      const int64_t k1 = std::min(K, k0 + every);
      trotter_segment(s, E, T, dt, k0, k1, tp);
      if (cb && cb->every > 0 && k1 - k0 == every) run_callbacks(s, cb, idx++);
    }
    if (energy_out) {
      auto* o = const_cast<qs_obs*>(h1);
      double* res = expect_result_slot(s, o);
      expectation_dev(s, o, res);
      *energy_out = download_scalar(res, s->stream);
    } else {
      hipck(hipStreamSynchronize(s->stream), "sync");
    }
  });
}

qs_status qs_entanglement_entropy(const qs_state* cs, int32_t a, double* out) {
  return guard([&] {
    check_state(cs);
    if (!out) fail(QS_E_INVALID, "null output");
    if (a < 1 || a >= cs->n) fail(QS_E_INVALID, "a must be in [1, n-1]");
    *out = entropy_dev(const_cast<qs_state*>(cs), a);
  });
}

qs_status qs_evolve(qs_state* s, const qs_obs* ch0, const qs_obs* ch1, double T, double dt, int32_t solver,
                    const qs_callbacks* cb) {
  return guard([&] {
    check_state(s);
    if (!ch0 || !ch1) fail(QS_E_INVALID, "null observable");
    if (ch0->n != s->n || ch1->n != s->n) fail(QS_E_STATE, "observables and state sizes differ");
    if (solver != QS_SOLVER_EXP && solver != QS_SOLVER_RK4 && solver != QS_SOLVER_RK45)
      fail(QS_E_INVALID, "unknown solver");
    const int64_t K = step_count(T, dt);
    check_callbacks(cb, s);
    auto* h0 = const_cast<qs_obs*>(ch0);
    auto* h1 = const_cast<qs_obs*>(ch1);
    h0->to_device(s->stream);
    h1->to_device(s->stream);
    const int n = s->n;
    const bool dbl = s->dbl();
    const int64_t every = (cb && cb->every > 0) ? cb->every : 0;
    int64_t idx = 0;
    auto after_step = [&](int64_t k) {
      if (every && (k + 1) % every == 0) run_callbacks(s, cb, idx++);
    };
    if (solver == QS_SOLVER_EXP) {
      if (n > 12) fail(QS_E_UNSUPPORTED, "the exp solver builds a dense 2^n x 2^n matrix: n <= 12");
      const int64_t D = int64_t(1) << n;
      const size_t mat = size_t(D) * D * 2;  // doubles
      DBuf bH, bP, bQ, bT;
      bH.ensure(mat * 8);
      bP.ensure(mat * 8);
      bQ.ensure(mat * 8);
      bT.ensure(size_t(D) * (dbl ? 16 : 8));
      double* H = bH.as<double>();
      const double c0 = coeff_norm(h0), c1 = coeff_norm(h1);
      for (int64_t k = 0; k < K; ++k) {
        const double u = (double(k) + 0.5) * dt / T;
        hipck(launch_zero(H, (int64_t)mat, s->stream), "zero");
        hipck(launch_dense_h_add(H, n, h0->dflips.as<uint64_t>(), h0->dgoff.as<int32_t>(), h0->dterms.as<PauliTermDev>(),
                                 (int)h0->flips.size(), 1.0 - u, s->stream),
              "dense H0");
        hipck(launch_dense_h_add(H, n, h1->dflips.as<uint64_t>(), h1->dgoff.as<int32_t>(), h1->dterms.as<PauliTermDev>(),
                                 (int)h1->flips.size(), u, s->stream),
              "dense H1");
        // exp(-i dt H) = (T_m(X))^(2^q), X = -i dt H / 2^q with ||X|| <= 1/2
        // (||H|| <= sum |c_t| of the Pauli terms), T_m the Taylor polynomial
        // of degree m with ||X||^(m+1) / (m+1)! <= 1e-18, in Horner form
        const double th = dt * ((1.0 - u) * c0 + u * c1);
        int q = 0;
        while (std::ldexp(th, -q) > 0.5) ++q;
        const double x = std::ldexp(th, -q);
        int m = 1;
        double rem = x * x / 2.0;  // x^(m+1) / (m+1)!
        while (rem > 1e-18 && m < 40) {
          ++m;
          rem *= x / (m + 1);
        }
        double* P = bP.as<double>();
        double* Q = bQ.as<double>();
        hipck(launch_identity(P, n, s->stream), "identity");
        const double sc = -dt * std::ldexp(1.0, -q);
        for (int j = m; j >= 1; --j) {  // P <- I + X P / j
          hipck(launch_zgemm(true, H, D, 1, 0, P, D, 1, 0, (int)D, (int)D, D, 1, Q, 0.0, sc / j, 1, s->stream),
                "Taylor step");
          std::swap(P, Q);
        }
        for (int r = 0; r < q; ++r) {  // squaring
          hipck(launch_zgemm(true, P, D, 1, 0, P, D, 1, 0, (int)D, (int)D, D, 1, Q, 1.0, 0.0, 0, s->stream), "square");
          std::swap(P, Q);
        }
        hipck(launch_matvec(dbl, P, s->ptr, bT.p, n, s->stream), "U psi");
        hipck(hipMemcpyAsync(s->ptr, bT.p, size_t(D) * (dbl ? 16 : 8), hipMemcpyDeviceToDevice, s->stream), "copy");
        after_step(k);
      }
      hipck(hipStreamSynchronize(s->stream), "sync");
      return;
    }
    // Runge-Kutta: tableau (c, a, b) of the classical RK4 or of Dormand-Prince 5(4)
    static const double rk4_c[4] = {0.0, 0.5, 0.5, 1.0};
    static const double rk4_a[4][6] = {{0}, {0.5}, {0.0, 0.5}, {0.0, 0.0, 1.0}};
    static const double rk4_b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    static const double dp_c[6] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0};
    static const double dp_a[6][6] = {{0},
                                      {1.0 / 5},
                                      {3.0 / 40, 9.0 / 40},
                                      {44.0 / 45, -56.0 / 15, 32.0 / 9},
                                      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
                                      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656}};
    static const double dp_b[6] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84};
    const bool rk4 = solver == QS_SOLVER_RK4;
    const int S = rk4 ? 4 : 6;
    const double* cc = rk4 ? rk4_c : dp_c;
    const double* bb = rk4 ? rk4_b : dp_b;
    auto aa = [&](int j, int l) { return rk4 ? rk4_a[j][l] : dp_a[j][l]; };
    const size_t vb = s->bytes();
    std::vector<std::unique_ptr<DBuf>> kv(S);
    for (auto& b : kv) {
      b = std::make_unique<DBuf>();
      b->ensure(vb);
    }
    DBuf by, btmp, bpart;
    by.ensure(vb);
    btmp.ensure(vb);
    const size_t pd = std::max(pauli_scratch_doubles(h0), pauli_scratch_doubles(h1)) + 8;
    bpart.ensure(pd * 8);
    double* part = bpart.as<double>();
    double* res = part + pd - 8;
    for (int64_t k = 0; k < K; ++k) {
      const double t = double(k) * dt;
      for (int j = 0; j < S; ++j) {
        void* y = s->ptr;
        if (j > 0) {  // y = psi + dt sum_l a_jl k_l
          LinComb lc{};
          lc.in[lc.nin] = s->ptr;
          lc.cre[lc.nin++] = 1.0;
          for (int l = 0; l < j; ++l)
            if (aa(j, l) != 0.0) {
              lc.in[lc.nin] = kv[l]->p;
              lc.cre[lc.nin++] = dt * aa(j, l);
            }
          hipck(launch_lincomb(dbl, by.p, n, lc, s->stream), "stage input");
          y = by.p;
        }
        rk_rhs(s, h0, h1, y, kv[j]->p, btmp.p, (t + cc[j] * dt) / T, part, res);
      }
      LinComb lc{};  // psi <- psi + dt sum_l b_l k_l
      lc.in[lc.nin] = s->ptr;
      lc.cre[lc.nin++] = 1.0;
      for (int l = 0; l < S; ++l)
        if (bb[l] != 0.0) {
          lc.in[lc.nin] = kv[l]->p;
          lc.cre[lc.nin++] = dt * bb[l];
        }
      hipck(launch_lincomb(dbl, s->ptr, n, lc, s->stream), "step");
      after_step(k);
    }
    hipck(hipStreamSynchronize(s->stream), "sync");
  });
}

// ---------------------------------------------------------------- adjoint
qs_status qs_adjoint(qs_circuit* c, const double* params, const qs_obs* H, qs_state* psi, qs_state* lam,
                     double* grad_out, double* energy_out) {
  return guard([&] {
    if (!c || !H) fail(QS_E_INVALID, "null argument");
    check_state(psi);
    check_state(lam);
    if (c->dens) fail(QS_E_UNSUPPORTED, "the adjoint needs a state-vector circuit, not a density-matrix one");
    if (psi == lam || psi->ptr == lam->ptr) fail(QS_E_INVALID, "psi and lambda must be distinct states");
    if (c->hc.n != psi->n || lam->n != psi->n || lam->dt != psi->dt || H->n != psi->n)
      fail(QS_E_STATE, "circuit, observable and states must have the same n and dtype");
    if (c->hc.nparams > 0 && (!params || !grad_out)) fail(QS_E_INVALID, "null params or grad_out");
    for (const Gate& g : c->hc.gates)
      if (!g.is_rot) {
        const int d = 1 << g.k;
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j) {
            cd acc = 0;
            for (int r = 0; r < d; ++r) acc += std::conj(g.mat[size_t(r) * d + i]) * g.mat[size_t(r) * d + j];
            if (std::abs(acc - (i == j ? 1.0 : 0.0)) > 1e-9) fail(QS_E_UNSUPPORTED, "adjoint needs unitary gates");
          }
      }
    hipStream_t st = psi->stream;
    ensure_plan(c, psi->dbl(), st);
    auto* o = const_cast<qs_obs*>(H);
    o->to_device(st);
    const int np = c->hc.nparams;
    const double* dpar = nullptr;
    if (np > 0) {
      c->dparams.ensure(sizeof(double) * np);
      hipck(hipMemcpyAsync(c->dparams.p, params, sizeof(double) * np, hipMemcpyHostToDevice, st), "params");
      dpar = c->dparams.as<double>();
    }
    // lambda = H psi and E = Re <psi|lambda> in the same passes
    double E = 0.0;
    {
      ProfScope pr(7, st);
      c->eout.ensure(sizeof(double));
      pauli_pass(psi, o, lam->ptr, c->eout.as<double>(), scratch_doubles(psi, pauli_scratch_doubles(o)));
      hipck(hipMemcpyAsync(&E, c->eout.p, sizeof(double), hipMemcpyDeviceToHost, st), "energy");
    }
    const int ns = c->hc.plan.ngrad_slots;
    c->gpart.ensure(sizeof(double) * (size_t(std::max(ns, 1)) * kGradStride));
    c->gout.ensure(sizeof(double) * std::max(ns, 1));
    if (ns > 0) hipck(launch_zero(c->gpart.as<double>(), int64_t(ns) * kGradStride, st), "zero");
    run_passes(c->dev, c->hc.plan, psi->dbl(), psi->ptr, lam->ptr, dpar, nullptr, c->gpart.as<double>(), st);
    std::vector<double> slots(ns);
    if (ns > 0) {
      hipck(launch_slot_sums(c->gpart.as<double>(), ns, kGradStride, kGradStride, c->gout.as<double>(), st),
            "slot sums");
      hipck(hipMemcpyAsync(slots.data(), c->gout.p, sizeof(double) * ns, hipMemcpyDeviceToHost, st), "grad");
    }
    hipck(hipStreamSynchronize(st), "sync");
    if (np > 0) {
      std::fill(grad_out, grad_out + np, 0.0);
      for (int i = 0; i < ns; ++i)
        if (c->slot_pidx[i] >= 0) grad_out[c->slot_pidx[i]] += slots[i];
    }
    if (energy_out) *energy_out = E;
  });
}

// ------------------------------------------------------------------- batch
namespace {
// (Re)build a batch's plans, level lists and device tables from its circuits,
// observables and per-instance options; any captured graphs are dropped.
void batch_build(qs_batch* b) {
  const int count = b->count;
  for (int w = 0; w < 2; ++w) {
    if (b->exec[w]) (void)hipGraphExecDestroy(b->exec[w]);
    if (b->graph[w]) (void)hipGraphDestroy(b->graph[w]);
    b->exec[w] = nullptr;
    b->graph[w] = nullptr;
  }
  b->insts.clear();
  b->geoms.clear();
  b->geoms_adj.clear();
  b->fwd.clear();
  b->adj.clear();
  hipck(hipStreamSynchronize(b->stream), "sync");
  if (b->h_params) (void)hipHostFree(b->h_params);
  if (b->h_energies) (void)hipHostFree(b->h_energies);
  if (b->h_grads) (void)hipHostFree(b->h_grads);
  b->h_params = b->h_energies = b->h_grads = nullptr;
  std::vector<TileOp> ops;
  std::vector<StagedOp> sops;
  std::vector<StageRec> stages;
  std::vector<cd> mats;
  std::vector<PhaseRec> phases;
  std::vector<int32_t> phlist, op_inst;
  std::vector<double> dpool, btab, qang;
  std::vector<cd> qtab, ctab;
  std::vector<PauliTermDev> terms;
  std::vector<int32_t> slot_pidx;
  std::vector<std::vector<bool>> pass_ctrl(count);
  int64_t state_elems = 0, gp_elems = 0;
  int params = 0, slots = 0, chunks = 0;
  for (int i = 0; i < count; ++i) {
    const qs_circuit* c = b->circs[i];
    const qs_obs* o = b->obs[i];
    TuneOpts opt = b->opts[i];
    opt.grid_bits = kGridBits;  // one workgroup per tile: every tile-index bit is a grid bit
    opt.force_stage = true;
    Plan p = plan_circuit(c->hc, opt, b->dbl);
    BatchInst in;
    std::memset(&in, 0, sizeof(in));
    in.n = c->hc.n;
    in.npass = (int)p.passes.size();
    in.pass0 = (int)b->geoms.size();
    in.ops_base = (int)ops.size();
    in.st_base = (int)stages.size();
    in.mat_base = (int)mats.size();
    in.ph_base = (int)phases.size();
    in.phl_base = (int)phlist.size();
    in.dp_base = (int)dpool.size();
    in.bt_base = (int)btab.size();
    in.qt_base = (int)qtab.size();
    in.ct_base = (int)ctab.size();
    for (const PhaseRec& r : p.phases)
      if (r.scale_idx >= 0) fail(QS_E_UNSUPPORTED, "batch circuits cannot hold run-time scaled phases");
    int nops = 0, tbits = -1;
    for (const Pass& ps : p.passes) {
      if (ps.kind != PASS_TILE || ps.geom.kern != 2)
        fail(QS_E_UNSUPPORTED, "batch circuits must plan into register-blocked tiled passes (no SWAP or k>=3 gates)");
      PassGeom g = ps.geom;
      if (tbits >= 0 && g.n - g.m != tbits) fail(QS_E_STATE, "internal: batch passes with different tile sizes");
      tbits = g.n - g.m;
      g.op0 = nops;
      g.nops = (int)ps.ops.size();
      nops += g.nops;
      ops.insert(ops.end(), ps.ops.begin(), ps.ops.end());
      op_inst.insert(op_inst.end(), ps.ops.size(), i);
      b->geoms.push_back(g);
      pass_ctrl[i].push_back(g.ctrl != 0);
    }
    for (size_t k = 0; k < p.passes.size(); ++k) {  // the two-state form of each pass
      const Pass& ps = p.passes[k];
      if (!ps.has_adj) {
        b->geoms_adj.push_back(b->geoms[in.pass0 + k]);
        continue;
      }
      PassGeom g = ps.geom_adj;
      g.op0 = nops;
      g.nops = (int)ps.ops_adj.size();
      nops += g.nops;
      ops.insert(ops.end(), ps.ops_adj.begin(), ps.ops_adj.end());
      op_inst.insert(op_inst.end(), ps.ops_adj.size(), i);
      b->geoms_adj.push_back(g);
      pass_ctrl[i][k] = pass_ctrl[i][k] || g.ctrl != 0;
    }
    in.nops = nops;
    in.tbits = std::max(tbits, 0);
    {  // this instance's op records, against its own phase records
      const std::vector<TileOp> mine(ops.begin() + in.ops_base, ops.end());
      const std::vector<StagedOp> r = staged_records(mine, p.phases);
      sops.insert(sops.end(), r.begin(), r.end());
    }
    stages.insert(stages.end(), p.stages.begin(), p.stages.end());
    mats.insert(mats.end(), p.matpool.begin(), p.matpool.end());
    phases.insert(phases.end(), p.phases.begin(), p.phases.end());
    phlist.insert(phlist.end(), p.phlist.begin(), p.phlist.end());
    dpool.insert(dpool.end(), p.dpool.begin(), p.dpool.end());
    btab.insert(btab.end(), p.btab.begin(), p.btab.end());
    qtab.insert(qtab.end(), p.qtab.begin(), p.qtab.end());
    qang.insert(qang.end(), p.qang.begin(), p.qang.end());
    ctab.insert(ctab.end(), p.ctab.begin(), p.ctab.end());
    in.param_base = params;
    in.nparams = c->hc.nparams;
    params += c->hc.nparams;
    in.slot_base = slots;
    in.nslots = p.ngrad_slots;
    slots += p.ngrad_slots;
    in.gp_off = gp_elems;
    gp_elems += int64_t(p.ngrad_slots) * (4ll << in.tbits);
    std::vector<int32_t> sp(p.ngrad_slots, -1);
    for (const Pass& ps : p.passes)
      for (const TileOp& op : ps.ops)
        if (op.kind == OP_ROT && op.gslot >= 0) sp[op.gslot] = op.pidx;
    slot_pidx.insert(slot_pidx.end(), sp.begin(), sp.end());
    in.obs_off = (int)terms.size();
    in.obs_nterms = (int)o->terms.size();
    terms.insert(terms.end(), o->terms.begin(), o->terms.end());
    in.state_off = state_elems;
    in.lam_off = state_elems + (1ll << in.n);
    state_elems += 2 * (1ll << in.n);
    in.e0 = chunks;
    in.ne = (int)std::max<int64_t>(1, (1ll << in.n) >> kBatchChunkBits);
    chunks += in.ne;
    b->insts.push_back(in);
  }
  b->nparams = params;
  // work items: the chunks, then forward level k = pass k of every instance
  // that has it, then adjoint level k = pass npass-1-k; the largest
  // instances first within a launch
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->insts[x].n > b->insts[y].n; });
  std::vector<BatchItem> items;
  b->chunk_off = 0;
  for (int i : order)
    for (int cidx = 0; cidx < b->insts[i].ne; ++cidx) items.push_back(BatchItem{i, 0, cidx, 0});
  b->nchunks = (int)items.size();
  int maxp = 0;
  for (const BatchInst& in : b->insts) maxp = std::max(maxp, in.npass);
  for (int dir = 0; dir < 2; ++dir)
    for (int k = 0; k < maxp; ++k) {
      qs_batch::Level lv{(int)items.size(), 0, false};
      for (int i : order) {
        const BatchInst& in = b->insts[i];
        if (k >= in.npass) continue;
        const int pass = dir ? in.npass - 1 - k : k;
        lv.ctrl = lv.ctrl || pass_ctrl[i][pass];
        for (int t = 0; t < (1 << in.tbits); ++t) items.push_back(BatchItem{i, pass, t, 0});
      }
      lv.cnt = (int)items.size() - lv.off;
      if (lv.cnt > 0) (dir ? b->adj : b->fwd).push_back(lv);
    }
  hipStream_t st = b->stream;
  upload(b->d_insts, b->insts, st);
  upload(b->d_geoms, b->geoms, st);
  upload(b->d_geoms_adj, b->geoms_adj, st);
  upload(b->d_ops, ops, st);
  upload(b->d_sops, sops, st);
  upload(b->d_op_inst, op_inst, st);
  upload(b->d_stages, stages, st);
  upload(b->d_phases, phases, st);
  upload(b->d_phlist, phlist, st);
  upload(b->d_dpool, dpool, st);
  upload(b->d_btab, btab, st);
  upload(b->d_qang, qang, st);
  upload(b->d_terms, terms, st);
  upload(b->d_slot_pidx, slot_pidx, st);
  upload(b->d_items, items, st);
  {
    std::vector<double> m(mats.size() * 2), q(qtab.size() * 2);
    for (size_t i = 0; i < mats.size(); ++i) { m[2 * i] = mats[i].real(); m[2 * i + 1] = mats[i].imag(); }
    for (size_t i = 0; i < qtab.size(); ++i) { q[2 * i] = qtab[i].real(); q[2 * i + 1] = qtab[i].imag(); }
    if (b->dbl) {
      upload(b->d_matc, m, st);
      upload(b->d_qtab, q, st);
      upload_complex<double>(b->d_ctab, ctab, true, st);
    } else {
      upload(b->d_matc, std::vector<float>(m.begin(), m.end()), st);
      upload(b->d_qtab, std::vector<float>(q.begin(), q.end()), st);
      upload_complex<float>(b->d_ctab, ctab, false, st);
    }
  }
  const size_t esz = b->dbl ? 16 : 8;
  check_mem(size_t(state_elems) * esz + size_t(gp_elems) * 8);
  b->d_states.ensure(size_t(state_elems) * esz + 16);
  b->d_params.ensure(sizeof(double) * std::max(params, 1));
  b->d_gpart.ensure(sizeof(double) * std::max<int64_t>(gp_elems, 1));
  b->d_slot_sum.ensure(sizeof(double) * std::max(slots, 1));
  b->d_epart.ensure(sizeof(double) * std::max(chunks, 1));
  b->d_energies.ensure(sizeof(double) * count);
  b->d_grads.ensure(sizeof(double) * std::max(params, 1));
  hipck(hipHostMalloc((void**)&b->h_params, sizeof(double) * std::max(params, 1), hipHostMallocDefault),
        "hipHostMalloc");
  hipck(hipHostMalloc((void**)&b->h_energies, sizeof(double) * count, hipHostMallocDefault), "hipHostMalloc");
  hipck(hipHostMalloc((void**)&b->h_grads, sizeof(double) * std::max(params, 1), hipHostMallocDefault),
        "hipHostMalloc");
  hipck(hipStreamSynchronize(st), "sync");
  BatchArgs& a = b->args;
  a.insts = b->d_insts.as<BatchInst>();
  a.count = count;
  a.geoms = b->d_geoms.as<PassGeom>();
  a.geoms_adj = b->d_geoms_adj.as<PassGeom>();
  a.dp.ops = b->d_ops.as<TileOp>();
  a.dp.sops = b->d_sops.as<StagedOp>();
  a.dp.stages = b->d_stages.as<StageRec>();
  a.dp.matc = b->d_matc.p;
  a.dp.phases = b->d_phases.as<PhaseRec>();
  a.dp.phlist = b->d_phlist.as<int32_t>();
  a.dp.dpool = b->d_dpool.as<double>();
  a.dp.btab = b->d_btab.as<double>();
  a.dp.qtab = b->d_qtab.p;
  a.dp.ctab = b->d_ctab.p;
  a.dp.qang = b->d_qang.as<double>();
  a.op_inst = b->d_op_inst.as<int32_t>();
  a.nops_total = (int)ops.size();
  a.states = b->d_states.p;
  a.params = b->d_params.as<double>();
  a.terms = b->d_terms.as<PauliTermDev>();
  a.slot_pidx = b->d_slot_pidx.as<int32_t>();
  a.gpart = b->d_gpart.as<double>();
  a.slot_sum = b->d_slot_sum.as<double>();
  a.epart = b->d_epart.as<double>();
  a.energies = b->d_energies.as<double>();
  a.grads = b->d_grads.as<double>();
}
}  // namespace

qs_status qs_batch_create(int32_t count, qs_circuit* const* circs, const qs_obs* const* obs, qs_dtype dt,
                          void* stream, qs_batch** out) {
  return guard([&] {
    if (!out) fail(QS_E_INVALID, "null output handle");
    *out = nullptr;
    if (count < 1) fail(QS_E_INVALID, "count must be >= 1");
    if (!circs || !obs) fail(QS_E_INVALID, "null circuits or observables");
    check_dtype(dt);
    for (int i = 0; i < count; ++i) {
      if (!circs[i] || !obs[i]) fail(QS_E_INVALID, "null circuit or observable in batch");
      if (circs[i]->dens) fail(QS_E_UNSUPPORTED, "batches take state-vector circuits only");
      if (obs[i]->n != circs[i]->hc.n) fail(QS_E_STATE, "observable and circuit sizes differ");
      if (circs[i]->hc.n > 24) fail(QS_E_INVALID, "batch instances are limited to 24 qubits");
      for (uint64_t f : obs[i]->flips)
        if (f != 0) fail(QS_E_UNSUPPORTED, "batch observables must be diagonal (I/Z strings)");
    }
    check_device();
    auto b = std::make_unique<qs_batch>();
    b->count = count;
    b->dbl = dt == QS_C128;
    b->circs.assign(circs, circs + count);
    b->obs.assign(obs, obs + count);
    for (int i = 0; i < count; ++i) b->opts.push_back(circs[i]->hc.opts);
    if (stream) {
      b->stream = static_cast<hipStream_t>(stream);
    } else {
      hipck(hipStreamCreate(&b->stream), "hipStreamCreate");
      b->own_stream = true;
    }
    batch_build(b.get());
    *out = b.release();
  });
}

namespace {
// One run of the batch on its stream: parameters in, rotation matrices,
// |0..0>, the forward levels, energies and lambda, (the adjoint levels,)
// energies and gradients out.  Only kernels and copies from pinned host
// memory: the sequence is captured into a graph as it stands.
void batch_enqueue(qs_batch* b, bool grads) {
  hipStream_t st = b->stream;
  const BatchArgs& a = b->args;
  const BatchItem* items = b->d_items.as<BatchItem>();
  ProfScope pr(8, st);
  hipck(hipMemcpyAsync(b->d_params.p, b->h_params, sizeof(double) * std::max(b->nparams, 1),
                       hipMemcpyHostToDevice, st),
        "params");
  hipck(launch_batch_rot(b->dbl, a, st), "batch rotations");
  hipck(launch_batch_init(b->dbl, a, items + b->chunk_off, b->nchunks, st), "batch init");
  for (const qs_batch::Level& lv : b->fwd)
    hipck(launch_batch_pass(b->dbl, a, items + lv.off, lv.cnt, 0, lv.ctrl, st), "batch forward level");
  hipck(launch_batch_energy(b->dbl, a, items + b->chunk_off, b->nchunks, st), "batch energy");
  if (grads)
    for (const qs_batch::Level& lv : b->adj)
      hipck(launch_batch_pass(b->dbl, a, items + lv.off, lv.cnt, 1, lv.ctrl, st), "batch adjoint level");
  hipck(launch_batch_finish(a, grads, st), "batch finish");
  hipck(hipMemcpyAsync(b->h_energies, b->d_energies.p, sizeof(double) * b->count, hipMemcpyDeviceToHost, st),
        "energies");
  if (grads)
    hipck(hipMemcpyAsync(b->h_grads, b->d_grads.p, sizeof(double) * std::max(b->nparams, 1),
                         hipMemcpyDeviceToHost, st),
          "grads");
}
}  // namespace

namespace {
// One run: parameters in, graph replay (captured on the first run of each
// kind; profiled runs launch eagerly so that their kernels are timed),
// results out.
void batch_run_impl(qs_batch* b, const double* params_packed, double* energies, double* grads) {
  const bool want = grads != nullptr;
  hipck(hipStreamSynchronize(b->stream), "sync");  // the previous run's copies have landed
  if (b->nparams > 0) std::memcpy(b->h_params, params_packed, sizeof(double) * b->nparams);
  if (!b->exec[want] && !g_prof) {
    hipStream_t st = b->stream;
    hipck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      batch_enqueue(b, want);
    } catch (...) {
      hipGraph_t gbad = nullptr;
      (void)hipStreamEndCapture(st, &gbad);
      if (gbad) (void)hipGraphDestroy(gbad);
      throw;
    }
    hipck(hipStreamEndCapture(st, &b->graph[want]), "end capture");
    hipck(hipGraphInstantiate(&b->exec[want], b->graph[want], nullptr, nullptr, 0), "graph instantiate");
  }
  if (b->exec[want] && !g_prof) hipck(hipGraphLaunch(b->exec[want], b->stream), "graph launch");
  else batch_enqueue(b, want);
  hipck(hipStreamSynchronize(b->stream), "sync");
  std::memcpy(energies, b->h_energies, sizeof(double) * b->count);
  if (want && b->nparams > 0) std::memcpy(grads, b->h_grads, sizeof(double) * b->nparams);
}

void batch_release(qs_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (int w = 0; w < 2; ++w) {
    if (b->exec[w]) (void)hipGraphExecDestroy(b->exec[w]);
    if (b->graph[w]) (void)hipGraphDestroy(b->graph[w]);
    b->exec[w] = nullptr;
    b->graph[w] = nullptr;
  }
  if (b->h_params) (void)hipHostFree(b->h_params);
  if (b->h_energies) (void)hipHostFree(b->h_energies);
  if (b->h_grads) (void)hipHostFree(b->h_grads);
  b->h_params = b->h_energies = b->h_grads = nullptr;
}
}  // namespace

qs_status qs_batch_run(qs_batch* b, const double* params_packed, double* energies, double* grads) {
  return guard([&] {
    if (!b) fail(QS_E_INVALID, "null batch");
    if (b->nparams > 0 && !params_packed) fail(QS_E_INVALID, "null params");
    if (!energies) fail(QS_E_INVALID, "null energies");
    batch_run_impl(b, params_packed, energies, grads);
  });
}

qs_status qs_batch_destroy(qs_batch* b) {
  return guard([&] {
    if (!b) return;
    batch_release(b);
    hipStream_t st = b->own_stream ? b->stream : nullptr;
    delete b;
    if (st) (void)hipStreamDestroy(st);
  });
}

namespace {

// FNV-1a over everything that defines the circuit's action.
uint64_t circuit_hash(const HostCircuit& hc) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t nb) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < nb; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&hc.n, sizeof hc.n);
  for (const Gate& g : hc.gates) {
    mix(&g.k, sizeof g.k);
    mix(g.tq, sizeof(int) * g.k);
    for (int q : g.cq) mix(&q, sizeof q);
    mix(&g.is_rot, sizeof g.is_rot);
    mix(&g.pauli, sizeof g.pauli);
    mix(&g.pidx, sizeof g.pidx);
    mix(&g.rsign, sizeof g.rsign);
    if (!g.mat.empty()) mix(g.mat.data(), g.mat.size() * sizeof(g.mat[0]));
  }
  return h;
}

struct TuneChoice {
  int tile_bits, fuse_k, use_mfma, low_bits, lane_ops;
};

extern "C++" {  // C++ helpers: class-type results
TuneOpts opts_of(const TuneChoice& t) {
  TuneOpts o;
  o.tile_bits = t.tile_bits;
  o.fuse_k = t.fuse_k;
  o.use_mfma = t.use_mfma;
  o.low_bits = t.low_bits;
  o.lane_ops = t.lane_ops != 0;
  return o;
}

std::string tune_key(const qs_circuit* c, const qs_state* s) {
  int dev = 0;
  hipck(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t pr;
  hipck(hipGetDeviceProperties(&pr, dev), "hipGetDeviceProperties");
  std::string arch(pr.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  char buf[256];
  std::snprintf(buf, sizeof buf, "n=%d gates=%zu dtype=%s device=%s hash=%016llx", c->hc.n, c->hc.gates.size(),
                s->dbl() ? "c128" : "c64", arch.c_str(), (unsigned long long)circuit_hash(c->hc));
  return buf;
}
}  // extern "C++"

bool cache_lookup(const char* path, const std::string& key, TuneChoice* out) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    const size_t kl = key.size();
    if (std::strncmp(line, key.c_str(), kl) != 0 || line[kl] != ' ') continue;
    TuneChoice t{0, 0, -1, 0, 0};
    const int got = std::sscanf(line + kl, " tile_bits=%d fuse_k=%d use_mfma=%d low_bits=%d lane_ops=%d", &t.tile_bits,
                                &t.fuse_k, &t.use_mfma, &t.low_bits, &t.lane_ops);
    if (got >= 4) {  // lines written before lane_ops existed read as lane_ops=0
      *out = t;      // the last matching line wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_append(const char* path, const std::string& key, const TuneChoice& t, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) fail(QS_E_INVALID, std::string("cannot open tuning cache ") + path);
  std::fprintf(f, "%s tile_bits=%d fuse_k=%d use_mfma=%d low_bits=%d lane_ops=%d ms=%.4f\n", key.c_str(), t.tile_bits,
               t.fuse_k, t.use_mfma, t.low_bits, t.lane_ops, ms);
  std::fclose(f);
}

void compile_with(qs_circuit* c, const TuneChoice& t, bool dbl, hipStream_t s) {
  c->hc.opts = opts_of(t);
  c->planned = false;
  c->dev_ok = false;
  ensure_plan(c, dbl, s);
}

}  // namespace

// Candidates: the default plan first (it is the reference every other
// candidate is checked against), then fusion widths with and without matrix
// cores.  Each is timed over a few runs from |+...+>.
qs_status qs_autotune(qs_circuit* c, qs_state* s, const double* params, const char* cache_path) {
  return guard([&] {
    if (!c) fail(QS_E_INVALID, "null circuit");
    check_state(s);
    if (c->hc.n != s->n) fail(QS_E_STATE, "circuit and state sizes differ");
    if (c->hc.nparams > 0 && !params) fail(QS_E_INVALID, "circuit has parameters but params is null");
    const bool dbl = s->dbl();
    const std::string key = tune_key(c, s);
    TuneChoice hit;
    if (cache_lookup(cache_path, key, &hit)) {
      compile_with(c, hit, dbl, s->stream);
      return;
    }
    const double* dpar = nullptr;
    if (c->hc.nparams > 0) {
      c->dparams.ensure(sizeof(double) * c->hc.nparams);
      hipck(hipMemcpyAsync(c->dparams.p, params, sizeof(double) * c->hc.nparams, hipMemcpyHostToDevice, s->stream),
            "params upload");
      dpar = c->dparams.as<double>();
    }
    // the default plan, lane ops, 13-bit tiles (complex64), low runs of 2^5
    // amplitudes, then fusion widths with matrix cores
    std::vector<TuneChoice> cands = {{0, 0, -1, 0, 0}, {0, 0, -1, 0, 1}, {0, 0, -1, 5, 0}, {0, 2, -1, 0, 0},
                                     {0, 3, 1, 0, 0},  {0, 4, 1, 0, 0},  {0, 5, 1, 0, 0}};
    if (!dbl) cands.push_back({13, 0, -1, 0, 0});
    DBuf ref;
    ref.ensure(s->bytes());
    double* part = scratch_doubles(s, kGridMax + 8);
    hipEvent_t e0, e1;
    hipck(hipEventCreate(&e0), "hipEventCreate");
    hipck(hipEventCreate(&e1), "hipEventCreate");
    struct EvFree {
      hipEvent_t a, b;
      ~EvFree() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } evfree{e0, e1};
    const double tol = dbl ? 1e-9 : 1e-4;  // on the 2-norm distance to the default plan's result
    double ref_n2 = 0, best_ms = 1e300;
    TuneChoice best = cands[0];
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      const TuneChoice& t = cands[ci];
      const TuneOpts o = opts_of(t);
      Plan p;
      try {
        p = plan_circuit(c->hc, o, dbl);
      } catch (const std::exception&) {
        if (ci == 0) throw;
        continue;  // this tiling does not fit the circuit
      }
      DevPlanBuf dp;
      dp.load(p, s->stream);
      hipck(launch_set_plus(dbl, s->ptr, s->n, s->stream), "set_plus");
      run_passes(dp, p, dbl, s->ptr, nullptr, dpar, nullptr, nullptr, s->stream);
      if (ci == 0) {
        hipck(hipMemcpyAsync(ref.p, s->ptr, s->bytes(), hipMemcpyDeviceToDevice, s->stream), "copy");
        hipck(launch_sumsq(dbl, ref.p, s->n, part, s->stream), "norm");
        ref_n2 = download_scalar(part + kGridMax, s->stream);
      } else {
        // |a - b|^2 = |a|^2 + |b|^2 - 2 Re<a|b>
        hipck(launch_sumsq(dbl, s->ptr, s->n, part, s->stream), "norm");
        const double n2 = download_scalar(part + kGridMax, s->stream);
        hipck(launch_dot_re(dbl, ref.p, s->ptr, s->n, part, s->stream), "dot");
        const double d2 = ref_n2 + n2 - 2 * download_scalar(part + kGridMax, s->stream);
        if (!(d2 < tol * tol)) continue;
      }
      double ms = 1e300;
      for (int rep = 0; rep < 3; ++rep) {
        hipck(launch_set_plus(dbl, s->ptr, s->n, s->stream), "set_plus");
        hipck(hipEventRecord(e0, s->stream), "hipEventRecord");
        run_passes(dp, p, dbl, s->ptr, nullptr, dpar, nullptr, nullptr, s->stream);
        hipck(hipEventRecord(e1, s->stream), "hipEventRecord");
        hipck(hipEventSynchronize(e1), "hipEventSynchronize");
        float f = 0;
        hipck(hipEventElapsedTime(&f, e0, e1), "hipEventElapsedTime");
        ms = std::min(ms, (double)f);
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
    compile_with(c, best, dbl, s->stream);
    cache_append(cache_path, key, best, best_ms);
  });
}

// Per size class (the instances with one qubit count), time candidate
// options on a batch of that class alone -- each candidate's launch
// sequence captured and replayed as a graph -- keep the fastest whose
// energies and gradients agree with the default's (1e-4 complex64, 1e-9
// complex128), then rebuild the whole batch with each instance's choice.
qs_status qs_batch_autotune(qs_batch* b, const double* params_packed, const char* cache_path) {
  return guard([&] {
    if (!b) fail(QS_E_INVALID, "null batch");
    if (b->nparams > 0 && !params_packed) fail(QS_E_INVALID, "null params");
    std::vector<int> poff(b->count + 1, 0);
    for (int i = 0; i < b->count; ++i) poff[i + 1] = poff[i] + b->circs[i]->hc.nparams;
    std::map<int, std::vector<int>> classes;
    for (int i = 0; i < b->count; ++i) classes[b->circs[i]->hc.n].push_back(i);
    std::vector<TuneChoice> cands = {{0, 0, -1, 0, 0}, {0, 0, -1, 0, 1}, {0, 0, -1, 5, 0},
                                     {10, 0, -1, 0, 0}, {11, 0, -1, 0, 0}, {0, 2, -1, 0, 0}};
    const double tol = b->dbl ? 1e-9 : 1e-4;
    int dev = 0;
    hipck(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t pr;
    hipck(hipGetDeviceProperties(&pr, dev), "hipGetDeviceProperties");
    std::string arch(pr.gcnArchName);
    for (char& ch : arch)
      if (ch == ' ') ch = '_';
    hipEvent_t e0, e1;
    hipck(hipEventCreate(&e0), "hipEventCreate");
    hipck(hipEventCreate(&e1), "hipEventCreate");
    struct EvFree {
      hipEvent_t a, b;
      ~EvFree() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } evfree{e0, e1};
    for (auto& [n, members] : classes) {
      uint64_t h = 1469598103934665603ull;
      for (int i : members) h = (h ^ circuit_hash(b->circs[i]->hc)) * 1099511628211ull;
      char kb[256];
      std::snprintf(kb, sizeof kb, "batch-class n=%d count=%zu dtype=%s device=%s hash=%016llx", n, members.size(),
                    b->dbl ? "c128" : "c64", arch.c_str(), (unsigned long long)h);
      const std::string key = kb;
      TuneChoice best = cands[0];
      if (!cache_lookup(cache_path, key, &best)) {
        qs_batch sub;
        sub.count = (int)members.size();
        sub.dbl = b->dbl;
        sub.stream = b->stream;
        std::vector<double> P;
        for (int i : members) {
          sub.circs.push_back(b->circs[i]);
          sub.obs.push_back(b->obs[i]);
          P.insert(P.end(), params_packed + poff[i], params_packed + poff[i + 1]);
        }
        struct SubFree {
          qs_batch* s;
          ~SubFree() { batch_release(s); }
        } subfree{&sub};
        std::vector<double> E0, G0, E(sub.count), G(std::max<size_t>(P.size(), 1));
        double best_ms = 1e300;
        for (size_t ci = 0; ci < cands.size(); ++ci) {
          sub.opts.assign(sub.count, opts_of(cands[ci]));
          try {
            batch_build(&sub);
          } catch (const Fail&) {
            if (ci == 0) throw;
            continue;  // a tiling this class cannot use
          } catch (const std::exception&) {
            if (ci == 0) throw;
            continue;
          }
          batch_run_impl(&sub, P.data(), E.data(), G.data());
          if (ci == 0) {
            E0 = E;
            G0 = G;
          } else {
            double d = 0;
            for (size_t k = 0; k < E.size(); ++k) d = std::max(d, std::fabs(E[k] - E0[k]));
            for (size_t k = 0; k < P.size(); ++k) d = std::max(d, std::fabs(G[k] - G0[k]));
            if (!(d < tol)) continue;
          }
          double ms = 1e300;
          for (int rep = 0; rep < 3; ++rep) {
            hipck(hipEventRecord(e0, sub.stream), "hipEventRecord");
            hipck(hipGraphLaunch(sub.exec[1], sub.stream), "graph launch");
            hipck(hipEventRecord(e1, sub.stream), "hipEventRecord");
            hipck(hipEventSynchronize(e1), "hipEventSynchronize");
            float f = 0;
            hipck(hipEventElapsedTime(&f, e0, e1), "hipEventElapsedTime");
            ms = std::min(ms, (double)f);
          }
          if (ms < best_ms) {
            best_ms = ms;
            best = cands[ci];
          }
        }
        cache_append(cache_path, key, best, best_ms);
      }
      for (int i : members) b->opts[i] = opts_of(best);
    }
    batch_build(b);
  });
}

qs_status qs_batch_choice(const qs_batch* b, int32_t i, qs_tune* out) {
  return guard([&] {
    if (!b || !out) fail(QS_E_INVALID, "null argument");
    if (i < 0 || i >= b->count) fail(QS_E_INVALID, "instance index out of range");
    const TuneOpts& o = b->opts[i];
    std::memset(out, 0, sizeof *out);
    out->tile_bits = o.tile_bits;
    out->fuse_k = o.fuse_k;
    out->use_mfma = o.use_mfma;
    out->low_bits = o.low_bits;
    out->lane_ops = o.lane_ops ? 1 : 0;
  });
}

// --------------------------------------------------------------- profiling
qs_status qs_profile_enable(int32_t on) {
  return guard([&] { g_prof = on != 0; });
}
qs_status qs_profile_reset(void) {
  return guard([&] {
    prof_collect();
    for (int i = 0; i < 10; ++i) {
      g_prof_cnt[i] = 0;
      g_prof_ms[i] = 0;
    }
  });
}
qs_status qs_profile_read(int32_t family, int64_t* launches, double* total_ms) {
  return guard([&] {
    if (family < 0 || family > 9) fail(QS_E_INVALID, "family out of range");
    prof_collect();
    if (launches) *launches = g_prof_cnt[family];
    if (total_ms) *total_ms = g_prof_ms[family];
  });
}

}  // extern "C"
