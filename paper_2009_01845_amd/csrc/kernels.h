// Launch wrappers of the gfx950 kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qs_types.h"

namespace qs {

// Device copies of a plan's pools.
struct DevPlan {
  const TileOp* ops = nullptr;
  const StagedOp* sops = nullptr;  // op records of staged passes (same index as ops)
  const double* mat = nullptr;    // complex128 interleaved
  const double* dpool = nullptr;  // phase polynomials
  const PhaseRec* phases = nullptr;
  const void* qtab = nullptr;     // complex table in the state precision
  const double* qang = nullptr;   // the same table as angles
  const StageRec* stages = nullptr;
  const int32_t* phlist = nullptr;
  const double* btab = nullptr;
  void* matc = nullptr;           // matrix pool in the state precision (rotation slots written per run)
  void* ctab = nullptr;           // phase factors in the state precision (scaled records written per run)
  int nops_total = 0;
  int nphases = 0;
};

constexpr int kGridMax = 2048;  // fixed upper bound on streaming grids (deterministic reductions)
constexpr int kGradStride = kGridMax * 4;  // adjoint partials: one slot per (block, wave)

// Fixed device workspace of the no-allocation entry points (noalloc.hip):
// room for the partial sums of an observable with up to kNoAllocMaxSlots
// reduction slots (diagonal polynomial, tile sets, far groups).
constexpr int kNoAllocMaxSlots = 64;
constexpr int64_t kNoAllocScratchDoubles = int64_t(kNoAllocMaxSlots + 1) * kGridMax + kNoAllocMaxSlots + 8;
// Device address of this device's workspace (looked up once per device).
hipError_t noalloc_scratch(double** out);

int tile_grid(const PassGeom& g);

// One tiled pass.  psi2 != nullptr selects the two-state (adjoint) kernel:
// ops run in reverse with inverse matrices on psi and psi2, and every
// trainable rotation writes Im<psi2|Pc P psi> partials to
// gpart[gslot * kGradStride + block * 4 + wave] before being undone.
hipError_t launch_tile_pass(bool dbl, void* psi, void* psi2, const PassGeom& g, const DevPlan& dp,
                            const double* params, const double* scales, double* gpart, hipStream_t s);
struct PauliTermDev {
  uint64_t zy;     // index bits carrying Z or Y
  int32_t ny4;     // number of Y factors mod 4
  int32_t pad;
  double coeff;
};

// Pauli groups evaluated on tiles: a set holds the groups whose flip masks lie
// in one tile bit set (the low L bits and H <= 6 high bits hbits[]).
constexpr int kPauliMaxH = 6;
struct PauliSet {
  int32_t n, L, H, first;         // first: lambda is written, not accumulated
  int32_t hbits[kPauliMaxH];
  int32_t g0, ng;                 // groups [g0, g0 + ng) of the group array
};
struct PauliGroupTile {
  uint32_t fl;                    // flip mask in tile-local bits
  int32_t t0, nt, pad;            // terms [t0, t0 + nt) of the term array
};
struct PauliTermTile {
  uint64_t zo;                    // Z/Y bits outside the tile (global positions)
  uint32_t zl;                    // Z/Y bits inside the tile (tile-local positions)
  int32_t ny4;                    // number of Y factors mod 4
  double coeff;
};

// One instance of a batch: its plan lives at the given bases of the
// concatenated pools (all offsets inside the records are instance-local).
struct BatchInst {
  int32_t n, npass, pass0, nops;
  int32_t ops_base, st_base, mat_base, ph_base;
  int32_t phl_base, dp_base, bt_base, qt_base;
  int32_t ct_base, param_base, nparams, slot_base;
  int32_t nslots, obs_off, obs_nterms, tbits;  // tbits: log2 of the tiles of each pass
  int32_t e0, ne, pad0, pad1;                  // energy / initialisation items [e0, e0 + ne)
  int64_t state_off, lam_off;                  // elements of the batch state buffer
  int64_t gp_off;                              // gradient partials: [slot][tile][wave] from here
};

// One workgroup's share of a batch launch: a tile of one pass of one
// instance (pass launches), or a chunk of 2^kBatchChunkBits amplitudes of one
// instance (initialisation and energy launches).
struct BatchItem {
  int32_t inst, pass, tile, pad;
};
constexpr int kBatchChunkBits = 12;

struct BatchArgs {
  const BatchInst* insts = nullptr;
  int count = 0;
  const PassGeom* geoms = nullptr;
  const PassGeom* geoms_adj = nullptr;  // the two-state form of each pass
  DevPlan dp;                      // concatenated pools; matc is written (rotations)
  const int32_t* op_inst = nullptr;  // instance of every op of the concatenated op array
  int nops_total = 0;
  void* states = nullptr;
  const double* params = nullptr;
  const PauliTermDev* terms = nullptr;  // diagonal observables, per instance
  const int32_t* slot_pidx = nullptr;
  double* gpart = nullptr;         // gradient partials (BatchInst::gp_off)
  double* slot_sum = nullptr;      // per gradient slot, summed over tiles and waves
  double* epart = nullptr;         // per energy item
  double* energies = nullptr;
  double* grads = nullptr;
};

// Batched instances run level by level: every launch takes one pass of every
// instance that has it, one workgroup per tile, so a large instance spreads
// over as many workgroups as it has tiles.
//   rot:    rotation matrices of every op from params
//   init:   every instance's state to |0..0> (energy items)
//   pass:   items[0..nitems) of one level; dir 0 forward, 1 adjoint (psi and
//           lambda, gradient partials); ctrl selects the variant with
//           in-tile controls
//   energy: E = sum d(x) |psi(x)|^2 of each diagonal observable per item,
//           lambda = d psi
//   finish: energies and (with grads) the gradient of every parameter
hipError_t launch_batch_rot(bool dbl, const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_init(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, hipStream_t s);
hipError_t launch_batch_pass(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, int dir, bool ctrl,
                             hipStream_t s);
hipError_t launch_batch_energy(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, hipStream_t s);
hipError_t launch_batch_finish(const BatchArgs& a, bool grads, hipStream_t s);

// Fill the forward and inverse matrices of every rotation op from params.
hipError_t launch_rot_mats(bool dbl, const DevPlan& dp, const double* params, hipStream_t s);
// exp(i scale * angle) factors of every scaled phase record (scales[rec.scale_idx])
hipError_t launch_phase_tabs(bool dbl, const DevPlan& dp, const double* scales, hipStream_t s);
hipError_t launch_perm_pass(bool dbl, void* psi, const PassGeom& g, const int* tau, hipStream_t s);
// Dense k-qubit block (k = 4, 5) with matrix-core instructions; the tile is the
// targets plus 7 other bits (g.m == k + 7), the low bits first; tl[t] =
// tile-local position of target t; mat = 2^k x 2^k complex128 (device).  With
// tl2 and mat2 (else both null) a second k-qubit block on other tile bits is
// applied to the same tile after the first (k = 4 only for complex128).
hipError_t launch_mfma_pass(bool dbl, void* psi, const PassGeom& g, const int* tl, int k, const double* mat,
                            const int* tl2, const double* mat2, hipStream_t s);

hipError_t launch_set_basis(bool dbl, void* psi, int n, uint64_t x, hipStream_t s);
hipError_t launch_set_plus(bool dbl, void* psi, int n, hipStream_t s);

// Reductions: each writes kGridMax-strided float64 partials; final_sum adds
// `count` partials in a fixed order into out[0] (device).
hipError_t launch_sumsq(bool dbl, const void* psi, int n, double* partials, hipStream_t s);
hipError_t launch_dot_re(bool dbl, const void* a, const void* b, int n, double* partials, hipStream_t s);

// One partial per workgroup of sum_x |psi_x|^2 E(x) for a diagonal observable
// written as a quadratic polynomial in the index bits: poly = [c, mu[n],
// lam[n*n] (upper triangle used)]; elo[j] (j < 2^min(n,12)) = the terms of
// the low 12 bits alone, without c.
hipError_t launch_expect_poly(bool dbl, const void* psi, int n, const double* poly, const double* elo,
                              double* partials, hipStream_t s);
// the same, also writing lambda[x] = E(x) psi[x]
hipError_t launch_hpsi_poly(bool dbl, const void* psi, void* lam, int n, const double* poly, const double* elo,
                            double* partials, hipStream_t s);
// one tile set of Pauli groups: partials (one per workgroup) of sum_g Re<psi|P_g psi>;
// with lam, also lambda (+)= sum_g P_g psi (written when set.first)
hipError_t launch_pauli_set(bool dbl, const void* psi, void* lam, const PauliSet& set, const PauliGroupTile* groups,
                            const PauliTermTile* terms, double* partials, hipStream_t s);
// one group whose flip mask does not fit a tile, straight from HBM: partials of
// Re<psi|P psi>; with lam, lambda (+)= P psi (written when first)
hipError_t launch_pauli_far(bool dbl, const void* psi, void* lam, int n, uint64_t flip, const PauliTermDev* terms,
                            int nterms, int first, double* partials, hipStream_t s);

hipError_t launch_final_sum(const double* partials, int count, double* out, hipStream_t s);
// out[slot] = sum of partials[slot*stride + b], b < nblocks, for every slot
hipError_t launch_slot_sums(const double* partials, int nslots, int nblocks, int stride, double* out,
                            hipStream_t s);

// Sampling (see qsim.h): block sums, scan, per-shot search.
// blocksums: sample_nblocks(n) doubles; prefix: sample_nblocks(n) + 1; chunks:
// 2 * sample_nchunks(n) + 1 (chunk totals and their prefix).
hipError_t launch_sample(bool dbl, const void* psi, int n, double* blocksums, double* prefix, double* chunks,
                         int64_t shots, uint64_t seed, const double* uniforms, const int* pos, int m, int64_t* out,
                         hipStream_t s);
// zero `count` doubles with a kernel (graph-capture safe)
// dst <- src, bytes a multiple of 16 and both 16-byte aligned (streaming kernel)
hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
int sample_nblocks(int n);
int sample_nchunks(int n);

// Density matrices (density.hip): an n-qubit rho stored as a 2n-qubit vector,
// rho[r][c] at r * 2^n + c.
// rho = |psi><psi| (psi has 2^n amplitudes, rho 4^n)
hipError_t launch_outer(bool dbl, void* rho, const void* psi, int n, hipStream_t s);
// out[0] (device) = Re Tr(P rho), P = the Pauli groups (flip masks, term
// ranges goff[g]..goff[g+1]); ngroups = 0 gives Re Tr(rho).  partials: kGridMax doubles.
hipError_t launch_dens_pauli(bool dbl, const void* rho, int n, const uint64_t* flips, const int32_t* goff,
                             const PauliTermDev* terms, int ngroups, double* partials, double* out,
                             hipStream_t s);

// Time evolution and reduced density matrices (evolution.hip).
// out = sum_l c_l in_l over 2^n amplitudes (c_l complex, float64 arithmetic);
// out may be one of the inputs.
constexpr int kLinCombMax = 8;
struct LinComb {
  const void* in[kLinCombMax];
  double cre[kLinCombMax], cim[kLinCombMax];
  int nin;
};
hipError_t launch_lincomb(bool dbl, void* out, int n, const LinComb& lc, hipStream_t s);
// H (dense 2^n x 2^n complex128, row-major) += scale * sum of the Pauli groups
hipError_t launch_dense_h_add(double* H, int n, const uint64_t* flips, const int32_t* goff, const PauliTermDev* terms,
                              int ngroups, double scale, hipStream_t s);
// out (complex128) = alpha * op(A) op(B) (+ I), op(A)(i,j) = a[i ars + j acs]
// (conjugated if conja), op(B)(j,k) = b[j brs + k bcs]; M x N, contraction K
// split into zgemm_splits(K, nsplit) chunks, chunk c written to the slab
// out + c M N (complex entries); a, b in the state precision (dbl) or float64.
hipError_t launch_zgemm(bool dbl, const void* a, int64_t ars, int64_t acs, int conja, const void* b, int64_t brs,
                        int64_t bcs, int conjb, int M, int N, int64_t K, int nsplit, double* out, double alpha_re,
                        double alpha_im, int add_identity, hipStream_t s);
int zgemm_splits(int64_t K, int nsplit);
// out[i] = sum of the nsplit slabs (count complex128 entries each), in order
hipError_t launch_split_sum(const double* part, int nsplit, int64_t count, double* out, hipStream_t s);
// P = identity (2^n x 2^n complex128)
hipError_t launch_identity(double* P, int n, hipStream_t s);
// y = U x, U dense 2^n x 2^n complex128; x, y in the state precision
hipError_t launch_matvec(bool dbl, const double* U, const void* x, void* y, int n, hipStream_t s);

}  // namespace qs
