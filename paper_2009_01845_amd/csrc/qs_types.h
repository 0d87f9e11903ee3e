// Plain-old-data records shared by the host planner and the HIP kernels.
// Nothing here includes HIP headers, so the planner compiles as plain C++.
#pragma once
#include <cstdint>

namespace qs {

constexpr int kMaxQubits = 35;
constexpr int kMaxTileBits = 13;
constexpr int kMaxOpsPerPass = 512;
constexpr int kThreads = 256;  // workgroup size of the streaming kernels (4 wave64)

// Op kinds inside a tiled pass.  The tile is the set of 2^m amplitudes that
// share every index bit outside the tile bit set T; T always holds the
// lowest L index bits so that each row of 2^L amplitudes is contiguous in HBM.
enum OpKind : int32_t {
  OP_DENSE1 = 1,  // 2x2 matrix on tile bit b[0]
  OP_DENSE2 = 2,  // 4x4 matrix on tile bits (b[0] = MSB of the matrix index, b[1])
  OP_DENSEK = 3,  // 2^k x 2^k matrix, k = 3..5, on tile bits b[0..k-1]
  OP_ROT = 4,     // exp(-i theta P/2) on tile bit b[0], theta = sign * params[pidx]
  OP_PHASE = 5,   // multiply by exp(i theta(x)), theta a quadratic polynomial in index bits
  OP_DIAG = 6,    // multiply by d[bits of x at up to 6 positions] (any diagonal)
  OP_MFMA = 7,    // 2^k x 2^k matrix (k = 4, 5) applied with matrix-core instructions
};

// In a staged pass (kern == 2) b[] holds register slots instead of tile bits,
// cin holds the controls on tile bits outside the registers and creg those on
// register slots; OP_PHASE keeps its per-pass phase slot in pidx.
struct TileOp {
  int32_t kind;
  int32_t k;         // number of target bits
  int32_t b[5];      // tile-local bit indices of the targets (b[0] = matrix MSB)
  uint32_t cin;      // control mask over tile-local bits (all must be 1)
  uint64_t cout;     // control mask over global index bits outside the tile
  int32_t mat;       // offset (complex entries) into the matrix pool; -1 if none
  int32_t pidx;      // OP_ROT: parameter index
  int32_t pauli;     // OP_ROT: 1 = X, 2 = Y, 3 = Z
  int32_t sign;      // OP_ROT: theta = sign * params[pidx] (sign = +-1)
  int32_t aux;       // OP_PHASE: phase record index; OP_DIAG: offset into diag pool;
                     // OP_ROT with a gradient slot: its index among the pass's gradient ops
  int32_t gslot;     // adjoint: gradient slot of this op (-1 if none)
  uint32_t creg;     // staged passes: control mask over register slots
  uint32_t flags;    // bit 0: the matrix is real; bit 1 (OP_PHASE): every term holds register slot b[0];
                     // bit 2 (OP_PHASE): every coefficient is a multiple of pi (factors are +-1);
                     // staged one-qubit ops: bit 3 [[a, it], [it, a]] form, bit 4 diagonal,
                     // bit 5 lane op (b[0] = lane bit 0..3 of the thread-group index, not a slot)
};

// The op record a staged pass walks, one per TileOp (same index), built on the
// host from the TileOp and its phase record so that everything an op needs
// arrives in one 32-byte load, issued one op ahead of its use.
struct StagedOp {
  int32_t opc;       // dispatch code of an uncontrolled op (-1: none; controlled ops use tab)
  uint32_t ctl;      // in-tile controls cin (bits 0..15) | register-slot controls creg << 16
  uint32_t cout_lo;  // controls on index bits outside the tile (all must be 1)
  uint32_t cout_hi;
  int32_t mat;       // 1-/2-qubit ops: matrix pool offset; general phase ops: ctab_n
  int32_t grad;      // two-state gradient: LDS slot | pauli << 8 | register slot << 12; -1: none
  int32_t ph;        // phase ops: per-pass slot p | kbs << 8 | wr_trivial << 10 | single-slot << 11 | wr_sign << 16
  int32_t tab;       // sign ops: bt_off; general phase ops: ctab_off;
                     // controlled ops: b[0] | b[1] << 4 | real << 8 | two-qubit << 9
};

constexpr int kRegBits = 4;            // register slots per thread in a staged pass
constexpr int kMaxPhasePerPass = 14;   // phase ops whose tile terms are prepared per tile
constexpr int kMaxGradPerPass = 64;    // parameterised rotations per pass (adjoint partials kept in LDS)
constexpr int kGridBits = 11;          // streaming grids hold at most 2^kGridBits workgroups
constexpr int kMaxKBits = 12;          // tile-index bits above the grid: n - m - kGridBits <= 12

// A stage of a staged pass: every thread gathers the 2^kRegBits amplitudes that
// differ only in the tile bits rb[0..kRegBits-1], applies the stage's ops in
// registers and writes them back.
struct StageRec {
  int32_t rb[kRegBits];  // tile-local bit held by register slot k
  int32_t op0;
  int32_t nops;
  uint32_t rbmask;
  int32_t pad;
};

// A quadratic phase polynomial theta(x) = c + sum_p mu_p x_p + sum_{p<q} lam_pq x_p x_q
// over index bits x_p, prepared for one tile bit set.  Stored in a double pool:
//   [0]            c
//   [1 .. n]       mu_p               (global bit p)
//   [1+n .. n+n*n] lam (n x n, symmetric, zero diagonal)
// and a complex table qtab[2^m] = exp(i theta_T(j)) of the polynomial restricted
// to the tile bits (all outside bits zero, constant excluded), in the state's
// precision, at qtab_off (complex entries) of the phase-table pool.
struct PhaseRec {
  int32_t dpool;     // offset of c in the double pool
  int32_t qtab_off;  // offset in the complex phase-table pool
  int32_t scale_idx; // -1: scale 1; else theta is multiplied by scales[scale_idx]
  int32_t wr_off;    // staged passes: exp(i Q_R(e)) over the register slots, 2^kRegBits entries
  int32_t bt_off;    // staged passes: per thread group (theta_T(jg), beta_0..beta_3) pass constants;
                     // sign ops keep only their parities / pi, bit-sliced: word [s][grp / 64],
                     // bit grp % 64, stored as raw 64-bit patterns
  int32_t wr_trivial;  // 1 when Q_R(e) is zero for every e
  int32_t kt_off;    // staged passes: lam(tile bit b, k-bit j) [m][kMaxKBits], then Q_k(kk) [2^kb]
  int32_t wr_sign;   // sign ops: bit e = parity of Q_R(e) / pi
  int32_t ctab_off;  // staged passes: complex factors in the state precision, per thread group
                     // exp(i beta_0..4) [ngroups][kRegBits + 1], then exp(i Q_R(e)) [2^kRegBits]
  int32_t ctab_n;    // entries at ctab_off (scaled records are filled per launch; 0 for sign ops)
};

// Per-pass geometry.
struct PassGeom {
  int32_t n;            // qubits
  int32_t m;            // tile bits
  int32_t L;            // low bits (0..L-1) in the tile
  int32_t H;            // high tile bits
  int32_t hbits[kMaxTileBits];  // global positions of the high tile bits, ascending
  int32_t nops;
  int32_t op0;          // first op in the op array
  int32_t kern;         // 1: one LDS sweep per op; 2: register-blocked stages
  int32_t st0, nst;     // staged passes: stage range
  int32_t ph0, nph;     // staged passes: phase records prepared per tile
  int32_t ctrl;         // staged passes: 1 if an op has controls inside the tile (predicated path)
};

}  // namespace qs
