// gfx950 kernels of the state-vector simulator.
//
// Layout: 2^n interleaved complex amplitudes (float2 or double2), qubit q at
// index bit n-1-q.  Every streaming kernel is bound by HBM bandwidth: it reads
// and writes each amplitude once per pass with 16-byte vector accesses, and
// the index arithmetic is 64-bit throughout (2^35 amplitudes).
//
// Every kernel with a thread loop is launched with kThreads threads and uses
// that constant for its stride: on gfx950 blockDim.x is a vector load from the
// implicit arguments, and each reload waits on all of the wave's outstanding
// vector memory operations (prefetches included).
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace qs {

namespace {

template <typename R> struct CT;
template <> struct CT<float> {
  using C = float2;
  using V = float4;  // 16-byte access = 2 amplitudes
  typedef float NV __attribute__((ext_vector_type(4)));
  static constexpr int VW = 2;
};
template <> struct CT<double> {
  using C = double2;
  using V = double2;  // 16-byte access = 1 amplitude
  typedef double NV __attribute__((ext_vector_type(2)));
  static constexpr int VW = 1;
};

template <typename C> __device__ __forceinline__ C mk(double re, double im) {
  C r;
  r.x = (decltype(r.x))re;
  r.y = (decltype(r.y))im;
  return r;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C> __device__ __forceinline__ C cmadd(C acc, C a, C b) {  // acc + a*b
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
  return acc;
}
template <typename C> __device__ __forceinline__ C cconj(C a) {
  a.y = -a.y;
  return a;
}

// In-place register updates.  An op loop that dispatches over many kinds of
// gate keeps its register array in one set of registers only if every case
// leaves each new value in the register of the old value it replaces;
// otherwise the compiler gives the cases a second array and moves it back
// after every op.  The compiler's own choice, an FMA that accumulates into
// the temporary holding the cross terms, puts the result in the wrong
// register, so the finishing FMA is written with its destination tied to
// the replaced value (VOP3 form).  The cross terms are computed first: they
// pass through an empty asm that the finishing FMAs depend on.
template <typename T> __device__ __forceinline__ void after2(T& a, T& b) { asm("" : "+v"(a), "+v"(b)); }
template <typename T> __device__ __forceinline__ void after4(T& a, T& b, T& c, T& d) {
  asm("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}
// d = x * m + t, in the register of d (whose old value is dead)
__device__ __forceinline__ void fma_to(float& d, float x, float m, float t) {
  asm("v_fma_f32 %0, %1, %2, %3" : "+v"(d) : "v"(x), "v"(m), "v"(t));
}
__device__ __forceinline__ void fma_to(double& d, double x, double m, double t) {
  asm("v_fma_f64 %0, %1, %2, %3" : "+v"(d) : "v"(x), "v"(m), "v"(t));
}
// a = a * m + t, in the register of a
__device__ __forceinline__ void fma_self(float& a, float m, float t) {
  asm("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "v"(m), "v"(t));
}
__device__ __forceinline__ void fma_self(double& a, double m, double t) {
  asm("v_fma_f64 %0, %0, %1, %2" : "+v"(a) : "v"(m), "v"(t));
}
// y = y + m * x and y = y - m * x, in the register of y
__device__ __forceinline__ void fma_acc(float& y, float m, float x) {
  asm("v_fma_f32 %0, %1, %2, %0" : "+v"(y) : "v"(m), "v"(x));
}
__device__ __forceinline__ void fma_acc(double& y, double m, double x) {
  asm("v_fma_f64 %0, %1, %2, %0" : "+v"(y) : "v"(m), "v"(x));
}
__device__ __forceinline__ void fms_acc(float& y, float m, float x) {
  asm("v_fma_f32 %0, -%1, %2, %0" : "+v"(y) : "v"(m), "v"(x));
}
__device__ __forceinline__ void fms_acc(double& y, double m, double x) {
  asm("v_fma_f64 %0, -%1, %2, %0" : "+v"(y) : "v"(m), "v"(x));
}
// (x, y) <- plane rotation by phi of (x, y), |phi| <= pi/2, as three shears
// x -= t y, y += s x, x -= t y with t = tan(phi/2), s = sin(phi): three
// in-place FMAs instead of two multiplies and two FMAs.  NEG rotates by -phi.
template <bool NEG, typename T> __device__ __forceinline__ void shear3(T& x, T& y, T t, T s) {
  if (NEG) {
    fma_acc(x, t, y);
    fms_acc(y, s, x);
    fma_acc(x, t, y);
  } else {
    fms_acc(x, t, y);
    fma_acc(y, s, x);
    fms_acc(x, t, y);
  }
}
// v *= f
template <typename C> __device__ __forceinline__ void cmul_ip(C& v, C f) {
  auto vx = v.x, vy = v.y;
  auto t1 = -vy * f.y, t2 = vy * f.x;
  after2(t1, t2);
  fma_to(vy, vx, f.y, t2);  // the new y is formed before x is overwritten
  fma_self(vx, f.x, t1);
  v.x = vx;
  v.y = vy;
}
// (a, b) <- (m00 a + m01 b, m10 a + m11 b), real coefficients
template <typename T> __device__ __forceinline__ void mix2(T& a, T& b, T m00, T m01, T m10, T m11) {
  auto ta = m01 * b, tb = m10 * a;
  after2(ta, tb);
  fma_self(a, m00, ta);
  fma_self(b, m11, tb);
}

__device__ __forceinline__ uint32_t insert_zeros(uint32_t i, uint32_t mask) {
  while (mask) {
    const int p = __builtin_ctz(mask);
    mask &= mask - 1;
    i = ((i >> p) << (p + 1)) | (i & ((1u << p) - 1u));
  }
  return i;
}
__device__ __forceinline__ uint64_t insert_zero64(uint64_t i, int p) {
  return ((i >> p) << (p + 1)) | (i & ((1ull << p) - 1ull));
}
// index of the tile holding global index x (the bits outside the tile, packed)
__device__ __forceinline__ uint64_t tile_index(uint64_t x, const PassGeom& g) {
  uint64_t y = x >> g.L;
  for (int i = g.H - 1; i >= 0; --i) {
    const int p = g.hbits[i] - g.L;
    y = (y & ((1ull << p) - 1ull)) | ((y >> (p + 1)) << p);
  }
  return y;
}
// Tiles walked by a grid-strided loop (t = block + k * grid): the low bits of t
// differ between workgroups running at the same time.  Rotating them to the
// top of the tile index spreads concurrent workgroups over the highest
// non-tile index bits instead of neighbouring tiles (with a high bit in the
// tile, neighbouring tiles are pairs of runs gigabytes apart, and the
// streaming rate drops by up to 17%).  A bijection on [0, 2^tbits).
__device__ __forceinline__ uint64_t spread_tile(uint64_t t, int tbits) {
  const int s = tbits < kGridBits ? tbits : kGridBits;
  return (t >> s) | ((t & ((1ull << s) - 1ull)) << (tbits - s));
}
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const PassGeom& g) {
  uint64_t b = t << g.L;
  for (int i = 0; i < g.H; ++i) b = insert_zero64(b, g.hbits[i]);
  return b;
}

// Sum of v over the workgroup in a fixed order; the result is valid in thread 0.
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(kThreads >> 6); ++i) r += red[i];
  __syncthreads();
  return r;
}

template <typename C> __device__ __forceinline__ C ldm(const double* mp, int idx) {
  return mk<C>(mp[2 * idx], mp[2 * idx + 1]);
}

// ----------------------------------------------------------------------------
// ops on an LDS tile of M = 2^m amplitudes
// ----------------------------------------------------------------------------

template <typename C>
__device__ __forceinline__ void pair2(C* t, uint32_t j0, uint32_t j1, C m00, C m01, C m10, C m11) {
  const C a = t[j0], b = t[j1];
  t[j0] = cmadd(cmul(m00, a), m01, b);
  t[j1] = cmadd(cmul(m10, a), m11, b);
}

template <typename C, bool TWO>
__device__ void op_dense1(C* t1, C* t2, int M, int b, uint32_t cin, C m00, C m01, C m10, C m11) {
  const uint32_t B = 1u << b;
  const uint32_t mask = B | cin;
  const int np = (M >> 1) >> __popc(cin);
  for (int i = threadIdx.x; i < np; i += kThreads) {
    const uint32_t j = insert_zeros((uint32_t)i, mask) | cin;
    pair2(t1, j, j | B, m00, m01, m10, m11);
    if (TWO) pair2(t2, j, j | B, m00, m01, m10, m11);
  }
}

template <typename C>
__device__ __forceinline__ void quad4(C* t, uint32_t j, uint32_t B0, uint32_t B1, const C* mm) {
  const C a0 = t[j], a1 = t[j | B1], a2 = t[j | B0], a3 = t[j | B0 | B1];
  C o[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    C acc = cmul(mm[4 * r + 0], a0);
    acc = cmadd(acc, mm[4 * r + 1], a1);
    acc = cmadd(acc, mm[4 * r + 2], a2);
    acc = cmadd(acc, mm[4 * r + 3], a3);
    o[r] = acc;
  }
  t[j] = o[0];
  t[j | B1] = o[1];
  t[j | B0] = o[2];
  t[j | B0 | B1] = o[3];
}

template <typename C, bool TWO>
__device__ void op_dense2(C* t1, C* t2, int M, const TileOp& op, const double* mp) {
  C mm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) mm[i] = ldm<C>(mp, i);
  const uint32_t B0 = 1u << op.b[0], B1 = 1u << op.b[1];
  const uint32_t mask = B0 | B1 | op.cin;
  const int nq = (M >> 2) >> __popc(op.cin);
  for (int i = threadIdx.x; i < nq; i += kThreads) {
    const uint32_t j = insert_zeros((uint32_t)i, mask) | op.cin;
    quad4(t1, j, B0, B1, mm);
    if (TWO) quad4(t2, j, B0, B1, mm);
  }
}

template <int K, typename C>
__device__ __forceinline__ void groupk(C* t, uint32_t j0, const uint32_t* offs, const double* mp) {
  constexpr int D = 1 << K;
  C in[D];
#pragma unroll
  for (int r = 0; r < D; ++r) in[r] = t[j0 | offs[r]];
#pragma unroll 1
  for (int r = 0; r < D; ++r) {
    C acc = mk<C>(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < D; ++c) acc = cmadd(acc, ldm<C>(mp, r * D + c), in[c]);
    t[j0 | offs[r]] = acc;
  }
}

template <int K, typename C, bool TWO>
__device__ void op_densek(C* t1, C* t2, int M, const TileOp& op, const double* mp) {
  constexpr int D = 1 << K;
  uint32_t offs[D];
  uint32_t tmask = 0;
#pragma unroll
  for (int t = 0; t < K; ++t) tmask |= 1u << op.b[t];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    uint32_t o = 0;
#pragma unroll
    for (int t = 0; t < K; ++t)
      if ((r >> (K - 1 - t)) & 1) o |= 1u << op.b[t];
    offs[r] = o;
  }
  const uint32_t mask = tmask | op.cin;
  const int ng = (M >> K) >> __popc(op.cin);
  for (int i = threadIdx.x; i < ng; i += kThreads) {
    const uint32_t j0 = insert_zeros((uint32_t)i, mask) | op.cin;
    groupk<K>(t1, j0, offs, mp);
    if (TWO) groupk<K>(t2, j0, offs, mp);
  }
}

// Im< lam | Pc P psi > over the tile, P a Pauli on tile bit b.
template <typename C>
__device__ double rot_grad_partial(const C* ps, const C* la, int M, int b, uint32_t cin, int pauli) {
  const uint32_t B = 1u << b;
  const uint32_t mask = B | cin;
  const int np = (M >> 1) >> __popc(cin);
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) {
    const uint32_t j = insert_zeros((uint32_t)i, mask) | cin;
    const C p0 = ps[j], p1 = ps[j | B], l0 = la[j], l1 = la[j | B];
    // q = P psi on the pair
    double q0r, q0i, q1r, q1i;
    if (pauli == 1) { q0r = p1.x; q0i = p1.y; q1r = p0.x; q1i = p0.y; }
    else if (pauli == 2) { q0r = p1.y; q0i = -p1.x; q1r = -p0.y; q1i = p0.x; }
    else { q0r = p0.x; q0i = p0.y; q1r = -p1.x; q1i = -p1.y; }
    // Im(conj(l) * q) = l.x*q.i - l.y*q.r
    acc += (double)l0.x * q0i - (double)l0.y * q0r + (double)l1.x * q1i - (double)l1.y * q1r;
  }
  return acc;
}

// ----------------------------------------------------------------------------
// tiled pass
// ----------------------------------------------------------------------------

template <typename R, bool TWO>
__global__ __launch_bounds__(256) void k_tile(typename CT<R>::C* __restrict__ psi,
                                              typename CT<R>::C* __restrict__ lam, const PassGeom g,
                                              const DevPlan dp, const double* __restrict__ params,
                                              const double* __restrict__ scales, double* __restrict__ gpart,
                                              int64_t ntiles) {
  using C = typename CT<R>::C;
  using VT = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  extern __shared__ __align__(16) char smem[];
  const int M = 1 << g.m;
  C* t1 = reinterpret_cast<C*>(smem);
  C* t2 = TWO ? t1 + M : nullptr;
  __shared__ uint64_t hoff[128];
  __shared__ double nu[kMaxTileBits];
  __shared__ double Ash;
  __shared__ C rowtab[128];
  __shared__ double red[8];

  const int tid = threadIdx.x;
  const int L = g.L, H = g.H, m = g.m;
  for (int hc = tid; hc < (1 << H); hc += kThreads) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << g.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;

  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = tile_base(spread_tile((uint64_t)t, g.n - g.m), g);
    for (int e = tid * VW; e < M; e += kThreads * VW) {
      const uint64_t a = base | hoff[e >> L] | (uint64_t)(e & lomask);
      *reinterpret_cast<VT*>(t1 + e) = *reinterpret_cast<const VT*>(psi + a);
      if (TWO) *reinterpret_cast<VT*>(t2 + e) = *reinterpret_cast<const VT*>(lam + a);
    }
    __syncthreads();

    for (int oi = 0; oi < g.nops; ++oi) {
      const int o = TWO ? g.nops - 1 - oi : oi;
      const TileOp op = dp.ops[g.op0 + o];
      if ((base & op.cout) != op.cout) continue;  // an outside control is 0 for this whole tile
      const int inv = TWO ? 1 : 0;
      switch (op.kind) {
        case OP_DENSE1: {
          const double* mp = dp.mat + 2 * (op.mat + inv * 4);
          op_dense1<C, TWO>(t1, t2, M, op.b[0], op.cin, ldm<C>(mp, 0), ldm<C>(mp, 1), ldm<C>(mp, 2),
                            ldm<C>(mp, 3));
          break;
        }
        case OP_ROT: {
          const double th = (TWO ? -1.0 : 1.0) * op.sign * params[op.pidx];
          if (TWO && op.gslot >= 0) {
            const double v = block_sum(rot_grad_partial(t1, t2, M, op.b[0], op.cin, op.pauli), red);
            if (tid == 0) gpart[(int64_t)op.gslot * kGradStride + blockIdx.x * 4] += v;
          }
          double s, c;
          sincos(0.5 * th, &s, &c);
          C m00, m01, m10, m11;
          if (op.pauli == 1) { m00 = mk<C>(c, 0); m01 = mk<C>(0, -s); m10 = mk<C>(0, -s); m11 = mk<C>(c, 0); }
          else if (op.pauli == 2) { m00 = mk<C>(c, 0); m01 = mk<C>(-s, 0); m10 = mk<C>(s, 0); m11 = mk<C>(c, 0); }
          else { m00 = mk<C>(c, -s); m01 = mk<C>(0, 0); m10 = mk<C>(0, 0); m11 = mk<C>(c, s); }
          op_dense1<C, TWO>(t1, t2, M, op.b[0], op.cin, m00, m01, m10, m11);
          break;
        }
        case OP_DENSE2:
          op_dense2<C, TWO>(t1, t2, M, op, dp.mat + 2 * (op.mat + inv * 16));
          break;
        case OP_DENSEK:
          if (op.k == 3) op_densek<3, C, TWO>(t1, t2, M, op, dp.mat + 2 * (op.mat + inv * 64));
          else if (op.k == 4) op_densek<4, C, TWO>(t1, t2, M, op, dp.mat + 2 * (op.mat + inv * 256));
          else op_densek<5, C, TWO>(t1, t2, M, op, dp.mat + 2 * (op.mat + inv * 1024));
          break;
        case OP_PHASE: {
          const PhaseRec rec = dp.phases[op.aux];
          const double* P = dp.dpool + rec.dpool;
          const int n = g.n;
          const double scl = (rec.scale_idx >= 0 ? scales[rec.scale_idx] : 1.0) * (TWO ? -1.0 : 1.0);
          if (tid < m) {
            const int p = tid < L ? tid : g.hbits[tid - L];
            double s = 0.0;
            for (uint64_t r = base; r; r &= r - 1) s += P[1 + n + p * n + __builtin_ctzll(r)];
            nu[tid] = s * scl;
          } else if (tid == m) {
            double s = P[0];
            for (uint64_t r = base; r; r &= r - 1) {
              const int q = __builtin_ctzll(r);
              s += P[1 + q];
              for (uint64_t r2 = r & (r - 1); r2; r2 &= r2 - 1) s += P[1 + n + q * n + __builtin_ctzll(r2)];
            }
            Ash = s * scl;
          }
          __syncthreads();
          for (int hc = tid; hc < (1 << H); hc += kThreads) {
            double a = Ash;
            for (int i = 0; i < H; ++i)
              if ((hc >> i) & 1) a += nu[L + i];
            double s, c;
            sincos(a, &s, &c);
            rowtab[hc] = mk<C>(c, s);
          }
          __syncthreads();
          C llc[VW];
#pragma unroll
          for (int v = 0; v < VW; ++v) {
            const uint32_t lo = (uint32_t)(tid * VW + v) & lomask;
            double a = 0.0;
            for (uint32_t r = lo; r; r &= r - 1) a += nu[__builtin_ctz(r)];
            double s, c;
            sincos(a, &s, &c);
            llc[v] = mk<C>(c, s);
          }
          const C* qt = reinterpret_cast<const C*>(dp.qtab) + rec.qtab_off;
          const double* qa = dp.qang + rec.qtab_off;
          for (int e = tid * VW; e < M; e += kThreads * VW) {
#pragma unroll
            for (int v = 0; v < VW; ++v) {
              const int j = e + v;
              C q;
              if (rec.scale_idx >= 0) {
                double s, c;
                sincos(scl * qa[j], &s, &c);
                q = mk<C>(c, s);
              } else {
                q = qt[j];
                if (TWO) q = cconj(q);
              }
              const C f = cmul(cmul(rowtab[j >> L], llc[v]), q);
              t1[j] = cmul(t1[j], f);
              if (TWO) t2[j] = cmul(t2[j], f);
            }
          }
          break;
        }
        default:
          break;
      }
      __syncthreads();
    }

    for (int e = tid * VW; e < M; e += kThreads * VW) {
      const uint64_t a = base | hoff[e >> L] | (uint64_t)(e & lomask);
      *reinterpret_cast<VT*>(psi + a) = *reinterpret_cast<const VT*>(t1 + e);
      if (TWO) *reinterpret_cast<VT*>(lam + a) = *reinterpret_cast<const VT*>(t2 + e);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// involutive bit permutation: the amplitude at x moves to tau(x)
// ----------------------------------------------------------------------------
// XOR the 16-byte granule index inside a 256-byte LDS row with higher index
// bits, so that threads walking any run of tile bits spread over the banks.
template <typename R> __device__ __forceinline__ uint32_t swz(uint32_t j);
template <> __device__ __forceinline__ uint32_t swz<float>(uint32_t j) {
  return j ^ (((j >> 4) ^ (j >> 8)) & 30u);
}
template <> __device__ __forceinline__ uint32_t swz<double>(uint32_t j) {
  return j ^ (((j >> 4) ^ (j >> 8)) & 15u);
}

struct PermArgs {
  int tau[kMaxQubits];
};

// the 16-byte vector of amplitudes t[idx[e]], t[idx[e+1]], ...
template <typename R>
__device__ __forceinline__ typename CT<R>::V gather_vec(const typename CT<R>::C* t, const uint16_t* idx, int e);
template <>
__device__ __forceinline__ float4 gather_vec<float>(const float2* t, const uint16_t* idx, int e) {
  const float2 a = t[swz<float>(idx[e])], b = t[swz<float>(idx[e + 1])];
  return make_float4(a.x, a.y, b.x, b.y);
}
template <>
__device__ __forceinline__ double2 gather_vec<double>(const double2* t, const uint16_t* idx, int e) {
  return t[swz<double>(idx[e])];
}

// NLD > 0: exactly NLD 16-byte vectors per thread and tile; NLD == 0: tiles
// smaller than one vector per thread (guarded)
template <typename R, int NLD>
__global__ __launch_bounds__(256) void k_perm(typename CT<R>::C* __restrict__ psi, const PassGeom g,
                                              const PermArgs pa, int64_t ntiles) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) char smem[];
  const int M = 1 << g.m;
  C* ta = reinterpret_cast<C*>(smem);
  C* tb = ta + M;
  uint16_t* ltau = reinterpret_cast<uint16_t*>(tb + M);
  __shared__ uint64_t hoff[128];
  __shared__ int loc[kMaxQubits];
  __shared__ int tau[kMaxQubits];
  __shared__ int hb[kMaxTileBits];
  const int tid = threadIdx.x, L = g.L, H = g.H;
  for (int b = tid; b < g.n; b += kThreads) {
    loc[b] = b < L ? b : -1;
    tau[b] = pa.tau[b];
  }
  if (tid < kMaxTileBits) hb[tid] = g.hbits[tid];
  __syncthreads();
  if (tid < H) loc[hb[tid]] = L + tid;
  for (int hc = tid; hc < (1 << H); hc += kThreads) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << g.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  for (int j = tid; j < M; j += kThreads) {
    uint32_t lj = 0;
    for (int i = 0; i < g.m; ++i)
      if ((j >> i) & 1) {
        const int gp = i < L ? i : hb[i - L];
        lj |= 1u << loc[tau[gp]];
      }
    ltau[j] = (uint16_t)lj;
  }
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;
  using VT = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  constexpr int kMaxLd = NLD > 0 ? NLD : 1;
  auto off = [&](int e) { return hoff[e >> L] | (uint64_t)(e & lomask); };
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint64_t base = (uint64_t)t << L;
    for (int i = 0; i < H; ++i) base = insert_zero64(base, hb[i]);
    uint64_t pbase = 0;
    for (uint64_t r = base; r; r &= r - 1) pbase |= 1ull << tau[__builtin_ctzll(r)];
    uint64_t tpu = pbase >> L;  // the partner's tile index: its bits outside the tile, packed
    for (int i = H - 1; i >= 0; --i) {
      const int p = hb[i] - L;
      tpu = (tpu & ((1ull << p) - 1ull)) | ((tpu >> (p + 1)) << p);
    }
    const int64_t tp = (int64_t)tpu;
    if (tp < t) continue;  // the partner tile's workgroup moves this pair
    const bool self = tp == t;
    VT ba[kMaxLd], bb[kMaxLd];  // every load of both tiles is issued before the LDS writes
#pragma unroll
    for (int u = 0; u < kMaxLd; ++u) {
      const int e = (u * kThreads + tid) * VW;
      if (NLD > 0 || e < M) {  // a self-paired tile is simply read twice
        ba[u] = *reinterpret_cast<const VT*>(psi + (base | off(e)));
        bb[u] = *reinterpret_cast<const VT*>(psi + (pbase | off(e)));
      }
    }
#pragma unroll
    for (int u = 0; u < kMaxLd; ++u) {
      const int e = (u * kThreads + tid) * VW;
      if (NLD > 0 || e < M) {
        *reinterpret_cast<VT*>(ta + swz<R>(e)) = ba[u];
        *reinterpret_cast<VT*>(tb + swz<R>(e)) = bb[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxLd; ++u) {
      const int e = (u * kThreads + tid) * VW;
      if (NLD > 0 || e < M) {
        *reinterpret_cast<VT*>(psi + (pbase | off(e))) = gather_vec<R>(ta, ltau, e);
        if (!self) *reinterpret_cast<VT*>(psi + (base | off(e))) = gather_vec<R>(tb, ltau, e);
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// initialisation
// ----------------------------------------------------------------------------
template <typename R>
__global__ void k_fill(typename CT<R>::C* psi, int64_t N, double re) {
  using C = typename CT<R>::C;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < N; i += (int64_t)gridDim.x * kThreads)
    psi[i] = mk<C>(re, 0.0);
}
__global__ void k_zero(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < count; i += (int64_t)gridDim.x * kThreads)
    p[i] = 0.0;
}

// Streaming copy of nvec 16-byte vectors: every thread has kCopyUnroll
// non-temporal loads in flight before its first store; consecutive threads
// take consecutive vectors, so each wave moves whole 1 KiB runs.  Also the
// measured streaming ceiling the pass kernels are compared with.
constexpr int kCopyUnroll = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(u32x4* __restrict__ dst, const u32x4* __restrict__ src, int64_t nvec) {
  const int64_t chunk = int64_t(kThreads) * kCopyUnroll;
  const int64_t nfull = nvec / chunk;
  for (int64_t c = blockIdx.x; c < nfull; c += gridDim.x) {
    const int64_t b = c * chunk + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + b + u * kThreads);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + b + u * kThreads);
  }
  // the ragged tail (fewer than kThreads * kCopyUnroll vectors), first workgroup only
  if (blockIdx.x == 0)
    for (int64_t i = nfull * chunk + threadIdx.x; i < nvec; i += kThreads) dst[i] = src[i];
}

template <typename R>
__global__ void k_set_one(typename CT<R>::C* psi, uint64_t x) {
  psi[x] = mk<typename CT<R>::C>(1.0, 0.0);
}

// ----------------------------------------------------------------------------
// reductions (float64 accumulation, fixed order)
// ----------------------------------------------------------------------------
inline int reduce_grid(int64_t units) {
  int64_t g = units / 1024;
  if (g < 1) g = 1;
  if (g > kGridMax) g = kGridMax;
  return (int)g;
}

template <typename R>
__global__ __launch_bounds__(256) void k_sumsq(const typename CT<R>::C* __restrict__ psi, int64_t N,
                                               double* __restrict__ part) {
  __shared__ double red[8];
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < N ? lo + chunk : N;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const auto v = psi[i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename R>
__global__ __launch_bounds__(256) void k_dot_re(const typename CT<R>::C* __restrict__ a,
                                                const typename CT<R>::C* __restrict__ b, int64_t N,
                                                double* __restrict__ part) {
  __shared__ double red[8];
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < N ? lo + chunk : N;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const auto u = a[i], v = b[i];
    acc += (double)u.x * v.x + (double)u.y * v.y;
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// sum_t c_t i^{ny_t} (-1)^{popcount(x & zy_t)}
__device__ __forceinline__ void pauli_factor(uint64_t x, const PauliTermDev* __restrict__ terms, int nt,
                                             double& fr, double& fi) {
  fr = 0.0;
  fi = 0.0;
  for (int t = 0; t < nt; ++t) {
    const PauliTermDev T = terms[t];
    double c = (__popcll(x & T.zy) & 1) ? -T.coeff : T.coeff;
    switch (T.ny4) {
      case 0: fr += c; break;
      case 1: fi += c; break;
      case 2: fr -= c; break;
      default: fi -= c; break;
    }
  }
}

template <typename R, bool WRITE>
__global__ __launch_bounds__(256) void k_expect_poly(const typename CT<R>::C* __restrict__ psi,
                                                     typename CT<R>::C* __restrict__ out, int n,
                                                     const double* __restrict__ poly, const double* __restrict__ elo,
                                                     double* __restrict__ part) {
  using C = typename CT<R>::C;
  using V = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  constexpr int LB = 12;
  constexpr int NV = (1 << LB) / (kThreads * VW);  // 16-byte vectors per thread in a full row
  constexpr int NH = kMaxQubits - LB;              // row-index (high) bits at most
  __shared__ double sElo[1 << LB];
  __shared__ double sLh[NH * NH];  // lam between high bits lb + i and lb + k
  __shared__ double sLx[LB * NH];  // lam between row bit pb and high bit lb + k
  __shared__ double sMu[NH];
  __shared__ double nu[LB];
  __shared__ double N1[64], N2[64];
  __shared__ double sA;
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int lb = n < LB ? n : LB;
  const int nh = n - lb;
  const int rows = 1 << lb;
  const bool full = rows == (1 << LB);
  const int64_t ntiles = 1ll << nh;
  const double* mu = poly + 1;
  const double* lam = poly + 1 + n;
  // the coefficients every row's set-up reads, staged once
  for (int j = tid; j < rows; j += kThreads) sElo[j] = elo[j];
  for (int i = tid; i < nh * nh; i += kThreads) sLh[i] = lam[(lb + i / nh) * n + lb + i % nh];
  for (int i = tid; i < lb * nh; i += kThreads) sLx[i] = lam[(i / nh) * n + lb + i % nh];
  for (int i = tid; i < nh; i += kThreads) sMu[i] = mu[lb + i];
  double acc = 0.0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t hbits = (uint64_t)t << lb;  // the row's high index bits
    V buf[NV];
    if (full) {  // the row's loads are in flight during its set-up
#pragma unroll
      for (int u = 0; u < NV; ++u) buf[u] = *reinterpret_cast<const V*>(psi + hbits + (int64_t)(u * kThreads + tid) * VW);
    }
    __syncthreads();  // staged coefficients ready; the previous row is done with nu, N1, N2, sA
    if (tid < 64) {
      // lane i < nh: the terms whose lowest set high bit is lb + i; lanes 32..: nu
      double a = 0.0;
      if (tid < 32 && tid < nh && ((t >> tid) & 1)) {
        a = sMu[tid];
        for (int k = tid + 1; k < nh; ++k)
          if ((t >> k) & 1) a += sLh[tid * nh + k];
      }
      for (int off = 16; off > 0; off >>= 1) a += __shfl_xor(a, off, 32);
      if (tid == 0) sA = poly[0] + a;
      if (tid >= 32 && tid - 32 < lb) {
        const int pb = tid - 32;
        double v = 0.0;
        for (int k = 0; k < nh; ++k)
          if ((t >> k) & 1) v += sLx[pb * nh + k];
        nu[pb] = v;
      }
    }
    __syncthreads();
    if (tid < 128) {
      const int half = tid >> 6, a = tid & 63;
      double v = 0.0;
      for (int b = 0; b < 6; ++b)
        if (((a >> b) & 1) && 6 * half + b < lb) v += nu[6 * half + b];
      if (half) N2[a] = v;
      else N1[a] = v;
    }
    __syncthreads();
    const double A = sA;
    if (full) {
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const int j0 = (u * kThreads + tid) * VW;
        const V v = buf[u];
        if constexpr (VW == 2) {
          const double e0 = A + sElo[j0] + N1[j0 & 63] + N2[j0 >> 6];
          const double e1 = A + sElo[j0 + 1] + N1[(j0 + 1) & 63] + N2[(j0 + 1) >> 6];
          acc += ((double)v.x * v.x + (double)v.y * v.y) * e0 + ((double)v.z * v.z + (double)v.w * v.w) * e1;
          if (WRITE) {
            V o;
            o.x = (R)(e0 * v.x);
            o.y = (R)(e0 * v.y);
            o.z = (R)(e1 * v.z);
            o.w = (R)(e1 * v.w);
            *reinterpret_cast<V*>(out + hbits + j0) = o;
          }
        } else {
          const double e = A + sElo[j0] + N1[j0 & 63] + N2[j0 >> 6];
          acc += ((double)v.x * v.x + (double)v.y * v.y) * e;
          if (WRITE) {
            V o;
            o.x = (R)(e * v.x);
            o.y = (R)(e * v.y);
            *reinterpret_cast<V*>(out + hbits + j0) = o;
          }
        }
      }
    } else {
      for (int j = tid; j < rows; j += kThreads) {
        const auto v = psi[hbits | (uint64_t)j];
        const double e = A + sElo[j] + N1[j & 63] + N2[j >> 6];
        acc += ((double)v.x * v.x + (double)v.y * v.y) * e;
        if (WRITE) out[hbits | (uint64_t)j] = mk<C>(e * v.x, e * v.y);
      }
    }
  }
  const double r = block_sum(acc, red);
  if (tid == 0) part[blockIdx.x] = r;
}

// Pauli groups on tiles: the tile (the 2^(L+H) amplitudes sharing the bits
// outside the set's tile bits) sits in LDS; for every element y of the tile,
// (P_g psi)[y] = phi_g(y ^ f_g) psi[y ^ f_g] with phi_g(x) = sum_t c_t i^{ny_t}
// (-1)^{|x & zy_t|}.  Accumulates sum_y Re(conj(psi[y]) sum_g (P_g psi)[y]) and,
// when WRITE, adds sum_g (P_g psi)[y] to lambda (or writes it when set.first).
// The complex64 form that writes lambda is held to four waves per SIMD (161
// registers otherwise; the adjoint's lambda = H psi about 1 ms faster at 30 qubits).
template <typename R, bool WRITE>
__global__ __launch_bounds__(256, (sizeof(R) == 4 && WRITE ? 4 : 1)) void k_pauli_tile(const typename CT<R>::C* __restrict__ psi,
                                                    typename CT<R>::C* __restrict__ lam, const PauliSet ps,
                                                    const PauliGroupTile* __restrict__ groups,
                                                    const PauliTermTile* __restrict__ terms,
                                                    double* __restrict__ part) {
  using C = typename CT<R>::C;
  constexpr int EPT = 16;  // elements per thread: tiles hold at most 2^12 = 16 * 256 amplitudes
  extern __shared__ __align__(16) char smem[];
  C* tile = reinterpret_cast<C*>(smem);
  __shared__ uint64_t hoff[1 << kPauliMaxH];
  __shared__ int hb[kPauliMaxH];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int L = ps.L, H = ps.H, m = L + H;
  const int M = 1 << m;
  const int64_t ntiles = 1ll << (ps.n - m);
  const uint32_t lomask = (1u << L) - 1u;
  if (tid < kPauliMaxH) hb[tid] = ps.hbits[tid];
  for (int hc = tid; hc < (1 << H); hc += kThreads) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << ps.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  double acc = 0.0;
  const bool accum = WRITE && !ps.first;
  // element e of a thread: when a complex64 set writes lambda, threads own
  // consecutive pairs (the layout of its 16-byte stores); otherwise a stride
  // of kThreads (fewer registers)
  constexpr bool PAIR = WRITE && sizeof(R) == 4;
  auto yof = [&](int e) { return PAIR ? ((e >> 1) * kThreads + tid) * 2 + (e & 1) : tid + e * kThreads; };
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint64_t base = spread_tile((uint64_t)t, ps.n - m) << L;
    for (int i = 0; i < H; ++i) base = insert_zero64(base, hb[i]);
    auto gaddr = [&](int y) { return base | hoff[y >> L] | (uint64_t)(y & lomask); };
    if (sizeof(R) == 4 && M == EPT * kThreads) {
      // a full complex64 tile: 16-byte loads, all in flight before the first
      // LDS write (complex128 keeps the element loop: the buffer would cost it
      // a wave per SIMD)
      using V = typename CT<R>::V;
      constexpr int VW = CT<R>::VW;
      constexpr int NLD = EPT / VW;
      V buf[NLD];
#pragma unroll
      for (int u = 0; u < NLD; ++u) buf[u] = *reinterpret_cast<const V*>(psi + gaddr((u * kThreads + tid) * VW));
#pragma unroll
      for (int u = 0; u < NLD; ++u) *reinterpret_cast<V*>(tile + (u * kThreads + tid) * VW) = buf[u];
    } else {
      for (int j = tid; j < M; j += kThreads) tile[j] = psi[gaddr(j)];
    }
    __syncthreads();
    R ar[EPT], ai[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) ar[e] = ai[e] = (R)0;
    for (int gi = 0; gi < ps.ng; ++gi) {  // uniform: one term at a time over all elements
      const PauliGroupTile G = groups[ps.g0 + gi];
      for (int ti = 0; ti < G.nt; ++ti) {
        const PauliTermTile T = terms[G.t0 + ti];
        // c i^ny (-1)^{|base & zo|} as a complex coefficient (kr, ki)
        const double c = (__popcll(base & T.zo) & 1) ? -T.coeff : T.coeff;
        const R kr = (R)(T.ny4 == 0 ? c : T.ny4 == 2 ? -c : 0.0);
        const R ki = (R)(T.ny4 == 1 ? c : T.ny4 == 3 ? -c : 0.0);
        const uint32_t zl = T.zl;
        if (zl == 0 && !(T.ny4 & 1)) {  // uniform: a real coefficient for the whole tile
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int y = yof(e);
            if (y < M) {
              const C px = tile[(uint32_t)y ^ G.fl];
              ar[e] += kr * px.x;
              ai[e] += kr * px.y;
            }
          }
        } else if (zl == 0) {  // an imaginary one
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int y = yof(e);
            if (y < M) {
              const C px = tile[(uint32_t)y ^ G.fl];
              ar[e] -= ki * px.y;
              ai[e] += ki * px.x;
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int y = yof(e);
            if (y < M) {
              const uint32_t x = (uint32_t)y ^ G.fl;
              const C px = tile[x];
              const bool neg = (__popc(x & zl) & 1) != 0;
              const R sr = neg ? -kr : kr, si = neg ? -ki : ki;
              ar[e] += sr * px.x - si * px.y;
              ai[e] += sr * px.y + si * px.x;
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int y = yof(e);
      if (y < M) {
        const C py = tile[y];
        acc += (double)py.x * ar[e] + (double)py.y * ai[e];
      }
    }
    bool written = false;
    if constexpr (PAIR) {
      if (WRITE && M == EPT * kThreads) {
      // lambda as 16-byte vectors: the old values of the set's tile in two
      // batches of loads, then the sums
      using V = typename CT<R>::V;
#pragma unroll
      for (int h = 0; h < EPT / 2; h += 4) {
        V lv[4];
        if (accum) {
#pragma unroll
          for (int u = 0; u < 4; ++u) lv[u] = *reinterpret_cast<const V*>(lam + gaddr(((h + u) * kThreads + tid) * 2));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = 2 * (h + u);
          V o;
          o.x = ar[e];
          o.y = ai[e];
          o.z = ar[e + 1];
          o.w = ai[e + 1];
          if (accum) {
            o.x = (R)((double)lv[u].x + ar[e]);
            o.y = (R)((double)lv[u].y + ai[e]);
            o.z = (R)((double)lv[u].z + ar[e + 1]);
            o.w = (R)((double)lv[u].w + ai[e + 1]);
          }
          *reinterpret_cast<V*>(lam + gaddr(((h + u) * kThreads + tid) * 2)) = o;
        }
      }
      written = true;
      }
    }
    if (WRITE && !written) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int y = yof(e);
        if (y < M) {
          const uint64_t ga = gaddr(y);
          if (accum) {
            const C l = lam[ga];
            lam[ga] = mk<C>((double)l.x + ar[e], (double)l.y + ai[e]);
          } else {
            lam[ga] = mk<C>(ar[e], ai[e]);
          }
        }
      }
    }
    __syncthreads();
  }
  const double r = block_sum(acc, red);
  if (tid == 0) part[blockIdx.x] = r;
}

// one Pauli group with a flip mask spread over many high bits: every thread
// gathers psi[y ^ flip] for its outputs y straight from HBM
template <typename R, bool WRITE>
__global__ __launch_bounds__(256) void k_pauli_far(const typename CT<R>::C* __restrict__ psi,
                                                   typename CT<R>::C* __restrict__ lam, int n, uint64_t flip,
                                                   const PauliTermDev* __restrict__ terms, int nt, int first,
                                                   double* __restrict__ part) {
  using C = typename CT<R>::C;
  __shared__ double red[8];
  const int64_t N = 1ll << n;
  double acc = 0.0;
  for (int64_t y = blockIdx.x * (int64_t)kThreads + threadIdx.x; y < N; y += (int64_t)gridDim.x * kThreads) {
    const uint64_t x = (uint64_t)y ^ flip;
    double fr, fi;
    pauli_factor(x, terms, nt, fr, fi);
    const C px = psi[x], py = psi[y];
    const double ar = fr * px.x - fi * px.y, ai = fr * px.y + fi * px.x;
    acc += (double)py.x * ar + (double)py.y * ai;
    if (WRITE) {
      if (first) {
        lam[y] = mk<C>(ar, ai);
      } else {
        const C l = lam[y];
        lam[y] = mk<C>((double)l.x + ar, (double)l.y + ai);
      }
    }
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_final_sum(const double* __restrict__ part, int count, double* out) {
  __shared__ double red[8];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += kThreads) acc += part[i];
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = r;
}

__global__ __launch_bounds__(256) void k_slot_sums(const double* __restrict__ part, int nblocks, int stride,
                                                  double* out) {
  __shared__ double red[8];
  double acc = 0.0;
  const double* p = part + (int64_t)blockIdx.x * stride;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) acc += p[i];
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// ----------------------------------------------------------------------------
// sampling: blocks of 1024 amplitudes = 64 lanes x 16 consecutive
// ----------------------------------------------------------------------------
constexpr int kSampBlock = 1024;
constexpr int kSampPerLane = 16;
constexpr int kSampChunk = 1024;  // block sums per chunk of the prefix scan

// inclusive wave scan of lane sums in a fixed (Hillis-Steele) order
__device__ __forceinline__ double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

template <typename R>
__device__ __forceinline__ double lane_mass(const typename CT<R>::C* psi, int64_t N, int64_t blk, int lane) {
  double s = 0.0;
  const int64_t first = blk * kSampBlock + (int64_t)lane * kSampPerLane;
  for (int e = 0; e < kSampPerLane; ++e) {
    const int64_t x = first + e;
    if (x < N) {
      const auto v = psi[x];
      s += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  return s;
}

__device__ __forceinline__ double vec_mass(float4 v) {
  return ((double)v.x * v.x + (double)v.y * v.y) + ((double)v.z * v.z + (double)v.w * v.w);
}
__device__ __forceinline__ double vec_mass(double2 v) { return v.x * v.x + v.y * v.y; }

// one wave per block of kSampBlock amplitudes: the block's total mass from
// coalesced 16-byte loads, summed in a fixed order (the shot search rebuilds
// the block's split over lanes itself)
template <typename R>
__global__ __launch_bounds__(256) void k_samp_blocks(const typename CT<R>::C* __restrict__ psi, int64_t N,
                                                     int64_t nb, double* __restrict__ S) {
  using V = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  const int64_t blk = blockIdx.x * (int64_t)(kThreads >> 6) + (threadIdx.x >> 6);
  if (blk >= nb) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const int64_t first = blk * kSampBlock;
  double s = 0.0;
  if (first + kSampBlock <= N) {
#pragma unroll
    for (int e = 0; e < kSampBlock / (64 * VW); ++e)
      s += vec_mass(*reinterpret_cast<const V*>(psi + first + (int64_t)(e * 64 + lane) * VW));
  } else {
    for (int64_t x = first + lane; x < N; x += 64) {
      const auto v = psi[x];
      s += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) S[blk] = s;
}

// block sums -> totals of chunks of kSampChunk blocks (fixed-order tree sum)
__global__ __launch_bounds__(256) void k_samp_chunks(const double* __restrict__ S, int64_t nb,
                                                     double* __restrict__ Ctot) {
  __shared__ double red[8];
  const int64_t c0 = blockIdx.x * (int64_t)kSampChunk;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kSampChunk / kThreads; ++k) {
    const int64_t i = c0 + k * kThreads + threadIdx.x;
    if (i < nb) s += S[i];
  }
  const double r = block_sum(s, red);
  if (threadIdx.x == 0) Ctot[blockIdx.x] = r;
}

// exclusive prefix of the block sums inside each chunk, offset by the chunk's
// exclusive prefix Coff; P[nb] = Coff[nc], the total
__global__ __launch_bounds__(256) void k_samp_prefix(const double* __restrict__ S, int64_t nb,
                                                     const double* __restrict__ Coff, int64_t nc,
                                                     double* __restrict__ P) {
  constexpr int PT = kSampChunk / kThreads;  // consecutive blocks per thread
  __shared__ double wsum[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = blockIdx.x * (int64_t)kSampChunk + (int64_t)tid * PT;
  double v[PT];
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    v[k] = i0 + k < nb ? S[i0 + k] : 0.0;
    t += v[k];
  }
  const double incl = wave_incl_scan(t);
  double excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 0.0;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  double run = Coff[blockIdx.x];
  for (int k = 0; k < w; ++k) run += wsum[k];
  run += excl;
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    if (i0 + k < nb) P[i0 + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && tid == 0) P[nb] = Coff[nc];
}

// exclusive prefix of S into P[0..nb], one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_samp_scan(const double* __restrict__ S, int64_t nb, double* __restrict__ P) {
  __shared__ double tot[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (nb + 1023) / 1024;
  const int64_t lo = tid * chunk, hi = lo + chunk < nb ? lo + chunk : nb;
  double s = 0.0;
  for (int64_t i = lo; i < hi; ++i) s += S[i];
  tot[tid] = s;
  __syncthreads();
  if (tid == 0) {  // sequential exclusive scan of 1024 chunk totals
    double run = 0.0;
    for (int i = 0; i < 1024; ++i) {
      const double v = tot[i];
      tot[i] = run;
      run += v;
    }
    P[nb] = run;
  }
  __syncthreads();
  double run = tot[tid];
  for (int64_t i = lo; i < hi; ++i) {
    P[i] = run;
    run += S[i];
  }
}

struct SampArgs {
  int m;
  int pos[64];  // index bit of outcome bit m-1-i is pos[i]
};

__device__ __forceinline__ double philox_uniform(uint64_t j, uint64_t seed) {
  uint32_t x0 = (uint32_t)j, x1 = (uint32_t)(j >> 32), x2 = 0, x3 = 0;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  const uint64_t w = ((uint64_t)x0 << 32) | x1;
  return (double)(w >> 11) * 0x1.0p-53;
}

template <typename R>
__global__ __launch_bounds__(256) void k_samp_shots(const typename CT<R>::C* __restrict__ psi, int64_t N,
                                                    int64_t nb, const double* __restrict__ P, int64_t shots,
                                                    uint64_t seed, const double* __restrict__ uni,
                                                    const SampArgs sa, int64_t* __restrict__ out) {
  using C = typename CT<R>::C;
  const int64_t j = blockIdx.x * (int64_t)(kThreads >> 6) + (threadIdx.x >> 6);
  if (j >= shots) return;
  const int lane = threadIdx.x & 63;
  const double u = uni ? uni[j] : philox_uniform((uint64_t)j, seed);
  const double target = u * P[nb];
  // block: first b with P[b+1] > target
  int64_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (P[mid + 1] > target) hi = mid;
    else lo = mid + 1;
  }
  const int64_t b = lo;
  const double mass = lane_mass<R>(psi, N, b, lane);
  const double incl = wave_incl_scan(mass);
  const double excl = __shfl_up(incl, 1, 64);
  const double before = P[b] + (lane == 0 ? 0.0 : excl);
  const unsigned long long hit = __ballot(P[b] + incl > target);
  int sel;
  if (hit) {
    sel = __builtin_ctzll(hit);
  } else {
    // rounding: the target sits past this block's own total (its lane sums
    // are added in another order than the block sum).  Take the last lane
    // that holds any mass, so the outcome never has probability zero
    const unsigned long long nz = __ballot(mass > 0.0);
    sel = nz ? 63 - __builtin_clzll(nz) : 63;
  }
  if (lane == sel) {
    const int64_t first = b * kSampBlock + (int64_t)lane * kSampPerLane;
    double run = before;
    int64_t x = -1, lastnz = -1;
    for (int e = 0; e < kSampPerLane; ++e) {
      const int64_t xi = first + e;
      if (xi >= N) break;
      const C v = psi[xi];
      const double p = (double)v.x * v.x + (double)v.y * v.y;
      if (p > 0.0) lastnz = xi;
      run += p;
      if (run > target) {
        x = xi;
        break;
      }
    }
    if (x < 0) x = lastnz >= 0 ? lastnz : (first < N ? first : N - 1);
    int64_t y = 0;
    for (int i = 0; i < sa.m; ++i) y = (y << 1) | (((uint64_t)x >> sa.pos[i]) & 1ull);
    out[j] = y;
  }
}

// ----------------------------------------------------------------------------
// staged tiled pass: the tile sits in LDS (bank-swizzled); each stage gathers
// 2^kRegBits amplitudes per thread, applies its ops in registers, scatters.
// ----------------------------------------------------------------------------
constexpr int NR = kRegBits;
constexpr int NE = 1 << kRegBits;


// parity of a / pi for a phase angle that is a multiple of pi
__device__ __forceinline__ bool pi_parity(double a) {
  return (__double2ll_rn(a * 0.31830988618379067154) & 1ll) != 0;
}
// register elements whose slot-k bit is set
__device__ __forceinline__ uint32_t slot_pattern(int k) {
  return k == 0 ? 0xAAAAu : k == 1 ? 0xCCCCu : k == 2 ? 0xF0F0u : 0xFF00u;
}
template <typename C> __device__ __forceinline__ C cneg(C a) {
  a.x = -a.x;
  a.y = -a.y;
  return a;
}

template <typename C> __device__ __forceinline__ C expi(double a);
template <> __device__ __forceinline__ float2 expi<float2>(double a) {
  const double r = a - 6.283185307179586 * rint(a * 0.15915494309189535);
  float s, c;
  sincosf((float)r, &s, &c);
  return make_float2(c, s);
}
template <> __device__ __forceinline__ double2 expi<double2>(double a) {
  double s, c;
  sincos(a, &s, &c);
  return make_double2(c, s);
}

template <int K, bool REAL, bool CTRL, typename C>
__device__ __forceinline__ void r1(C* v, C m00, C m01, C m10, C m11, uint32_t creg) {
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & (1 << K)) continue;
    if (CTRL && (e & creg) != creg) continue;
    const int f = e | (1 << K);
    auto ax = v[e].x, ay = v[e].y, bx = v[f].x, by = v[f].y;
    if (REAL) {
      mix2(ax, bx, m00.x, m01.x, m10.x, m11.x);
      mix2(ay, by, m00.x, m01.x, m10.x, m11.x);
    } else {
      // every output reads all four inputs: the three terms without the
      // replaced input first, then the finishing FMA
      auto tax = -m00.y * ay + m01.x * bx - m01.y * by;
      auto tay = m00.y * ax + m01.x * by + m01.y * bx;
      auto tbx = m10.x * ax - m10.y * ay - m11.y * by;
      auto tby = m10.x * ay + m10.y * ax + m11.y * bx;
      after4(tax, tay, tbx, tby);
      fma_self(ax, m00.x, tax);
      fma_self(ay, m00.x, tay);
      fma_self(bx, m11.x, tbx);
      fma_self(by, m11.x, tby);
    }
    v[e].x = ax;
    v[e].y = ay;
    v[f].x = bx;
    v[f].y = by;
  }
}

template <bool REAL, typename C>
__device__ __forceinline__ void r1_any(C* v, int k, C m00, C m01, C m10, C m11, uint32_t creg) {
  if (creg == 0) {  // uniform: no register-slot controls
    switch (k) {
      case 0: r1<0, REAL, false>(v, m00, m01, m10, m11, 0); break;
      case 1: r1<1, REAL, false>(v, m00, m01, m10, m11, 0); break;
      case 2: r1<2, REAL, false>(v, m00, m01, m10, m11, 0); break;
      default: r1<3, REAL, false>(v, m00, m01, m10, m11, 0); break;
    }
    return;
  }
  switch (k) {
    case 0: r1<0, REAL, true>(v, m00, m01, m10, m11, creg); break;
    case 1: r1<1, REAL, true>(v, m00, m01, m10, m11, creg); break;
    case 2: r1<2, REAL, true>(v, m00, m01, m10, m11, creg); break;
    default: r1<3, REAL, true>(v, m00, m01, m10, m11, creg); break;
  }
}

template <int KH, int KL, bool CTRL, typename C>
__device__ __forceinline__ void r2(C* v, const C* __restrict__ mm, uint32_t creg) {
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & ((1 << KH) | (1 << KL))) continue;
    if (CTRL && (e & creg) != creg) continue;
    const int idx[4] = {e, e | (1 << KL), e | (1 << KH), e | (1 << KL) | (1 << KH)};
    decltype(C().x) x[4], y[4], tx[4], ty[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      x[r] = v[idx[r]].x;
      y[r] = v[idx[r]].y;
    }
    // output r without its diagonal term on the component it replaces
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const C d = mm[4 * r + r];
      tx[r] = -d.y * y[r];
      ty[r] = d.y * x[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c == r) continue;
        const C m = mm[4 * r + c];
        tx[r] += m.x * x[c] - m.y * y[c];
        ty[r] += m.x * y[c] + m.y * x[c];
      }
    }
    after4(tx[0], tx[1], tx[2], tx[3]);
    after4(ty[0], ty[1], ty[2], ty[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const auto dx = mm[4 * r + r].x;
      fma_self(x[r], dx, tx[r]);
      fma_self(y[r], dx, ty[r]);
      v[idx[r]].x = x[r];
      v[idx[r]].y = y[r];
    }
  }
}

template <typename C>
__device__ __forceinline__ void r2_any(C* v, int kh, int kl, const C* __restrict__ mp, uint32_t creg) {
  if (creg == 0) {  // uniform: no register-slot controls
    switch (kh * 4 + kl) {
      case 4: r2<1, 0, false>(v, mp, 0); break;
      case 8: r2<2, 0, false>(v, mp, 0); break;
      case 9: r2<2, 1, false>(v, mp, 0); break;
      case 12: r2<3, 0, false>(v, mp, 0); break;
      case 13: r2<3, 1, false>(v, mp, 0); break;
      default: r2<3, 2, false>(v, mp, 0); break;
    }
    return;
  }
  switch (kh * 4 + kl) {
    case 4: r2<1, 0, true>(v, mp, creg); break;
    case 8: r2<2, 0, true>(v, mp, creg); break;
    case 9: r2<2, 1, true>(v, mp, creg); break;
    case 12: r2<3, 0, true>(v, mp, creg); break;
    case 13: r2<3, 1, true>(v, mp, creg); break;
    default: r2<3, 2, true>(v, mp, creg); break;
  }
}

// k-qubit matrix on register slots 0..K-1 (slot K-1 = matrix MSB)
template <int K, typename C>
__device__ __forceinline__ void rk(C* v, const double* mp, uint32_t creg) {
  constexpr int D = 1 << K;
#pragma unroll
  for (int g0 = 0; g0 < NE; g0 += D) {
    if ((g0 & creg) != creg) continue;
    C in[D];
#pragma unroll
    for (int i = 0; i < D; ++i) in[i] = v[g0 + i];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      C acc = mk<C>(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < D; ++c) acc = cmadd(acc, ldm<C>(mp, r * D + c), in[c]);
      v[g0 + r] = acc;
    }
  }
}

// negate where `bit` is 1 (flip the sign bits, no branch)
__device__ __forceinline__ float2 flip_sign(float2 a, uint32_t bit) {
  const uint32_t m = bit << 31;
  a.x = __uint_as_float(__float_as_uint(a.x) ^ m);
  a.y = __uint_as_float(__float_as_uint(a.y) ^ m);
  return a;
}
__device__ __forceinline__ double2 flip_sign(double2 a, uint32_t bit) {
  const unsigned long long m = (unsigned long long)bit << 63;
  a.x = __longlong_as_double(__double_as_longlong(a.x) ^ m);
  a.y = __longlong_as_double(__double_as_longlong(a.y) ^ m);
  return a;
}

// uncontrolled ops with compile-time register slots (the fast dispatch)
template <int K, bool REAL, bool TWO, typename C>
__device__ __forceinline__ void op1(C* v, C* w, const C* __restrict__ mp) {
  const C a = mp[0], b = mp[1], c = mp[2], d = mp[3];
  r1<K, REAL, false>(v, a, b, c, d, 0u);
  if (TWO) r1<K, REAL, false>(w, a, b, c, d, 0u);
}
template <int KH, int KL, bool TWO, typename C>
__device__ __forceinline__ void op2(C* v, C* w, const C* __restrict__ mp) {
  r2<KH, KL, false>(v, mp, 0u);
  if (TWO) r2<KH, KL, false>(w, mp, 0u);
}
// [[a, i t], [i t, a]] (a, t real: X rotations) and diagonal 2x2 on slot K
template <int K, typename C>
__device__ __forceinline__ void r1x(C* v, C m00, C m01) {
  const auto a = m00.x, t = m01.y;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & (1 << K)) continue;
    const int f = e | (1 << K);
    auto px = v[e].x, py = v[e].y, qx = v[f].x, qy = v[f].y;
    mix2(px, qy, a, -t, t, a);  // (p.x, q.y) and (p.y, q.x) mix separately
    mix2(py, qx, a, t, -t, a);
    v[e].x = px;
    v[e].y = py;
    v[f].x = qx;
    v[f].y = qy;
  }
}
// a Y (X = false) or X (X = true) rotation on slot K in three-shear form, up
// to the sign (-1)^k of its angle reduction: a Y rotation turns (p.x, q.x)
// and (p.y, q.y) by phi; an X rotation turns (p.y, q.x) by phi and (p.x, q.y)
// by -phi
template <int K, bool X, typename C, typename T>
__device__ __forceinline__ void r1s(C* v, T t, T s) {
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & (1 << K)) continue;
    const int f = e | (1 << K);
    auto px = v[e].x, py = v[e].y, qx = v[f].x, qy = v[f].y;
    if (X) {
      shear3<false>(py, qx, t, s);
      shear3<true>(px, qy, t, s);
    } else {
      shear3<false>(px, qx, t, s);
      shear3<false>(py, qy, t, s);
    }
    v[e].x = px;
    v[e].y = py;
    v[f].x = qx;
    v[f].y = qy;
  }
}
template <int K, bool X, bool TWO, typename C>
__device__ __forceinline__ void op1s(C* v, C* w, const C* __restrict__ sp) {
  const C ts = sp[0];
  r1s<K, X>(v, ts.x, ts.y);
  if (TWO) r1s<K, X>(w, ts.x, ts.y);
}
template <int K, typename C>
__device__ __forceinline__ void r1d(C* v, C d0, C d1) {
#pragma unroll
  for (int e = 0; e < NE; ++e) cmul_ip(v[e], (e >> K) & 1 ? d1 : d0);
}
template <int K, bool TWO, typename C>
__device__ __forceinline__ void op1x(C* v, C* w, const C* __restrict__ mp) {
  const C a = mp[0], b = mp[1];
  r1x<K>(v, a, b);
  if (TWO) r1x<K>(w, a, b);
}
template <int K, bool TWO, typename C>
__device__ __forceinline__ void op1d(C* v, C* w, const C* __restrict__ mp) {
  const C a = mp[0], d = mp[3];
  r1d<K>(v, a, d);
  if (TWO) r1d<K>(w, a, d);
}

// ---- lane ops: a one-qubit op on the tile bit held by lane bit J (J < 4) of
// the stage's thread-group index.  The partner amplitude of register element
// e sits in the same element of lane (lane ^ 2^J), in the same row of 16
// lanes, and is read with DPP moves: quad_perm for J = 0, 1; row_half_mirror
// (lane ^ 7) then quad_perm (^ 3) for J = 2; row_ror:8 for J = 3.  Each lane
// computes its own output: own * a + partner * c, with (a, c) = (m00, m01)
// where its bit is 0 and (m11, m10) where it is 1.  Only one-state passes
// hold lane ops: the planner stages the two-state (adjoint) form of a pass
// without them.
template <int J> __device__ __forceinline__ int lane_xor32(int v) {
  if (J == 0) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  if (J == 1) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  if (J == 2) return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
  return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
}
template <int J> __device__ __forceinline__ float lane_xor(float x) {
  return __int_as_float(lane_xor32<J>(__float_as_int(x)));
}
template <int J> __device__ __forceinline__ double lane_xor(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = lane_xor32<J>((int)(b & 0xffffffffll)), hi = lane_xor32<J>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// FORM 0: general complex matrix; 1: real; 2: diagonal; 3: [[a, i t], [i t, a]]
template <int J, int FORM, typename C>
__device__ __forceinline__ void rlane(C* v, const C* __restrict__ mp, int tid) {
  const bool hi = (tid >> J) & 1;
  const C a = hi ? mp[3] : mp[0];
  const C c = hi ? mp[2] : mp[1];
  if (FORM == 2) {
#pragma unroll
    for (int e = 0; e < NE; ++e) cmul_ip(v[e], a);
    return;
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    // keep one element's exchange in flight at a time (the empty asm is
    // ordered against the previous element's): hoisting all sixteen would
    // hold 32 more registers across the whole op dispatch
    asm volatile("" : "+v"(v[e].x), "+v"(v[e].y));
    const auto px = lane_xor<J>(v[e].x), py = lane_xor<J>(v[e].y);
    auto x = v[e].x, y = v[e].y;
    if (FORM == 1) {
      x = a.x * x + c.x * px;
      y = a.x * y + c.x * py;
    } else if (FORM == 3) {  // a = (a, 0), c = (0, t)
      x = a.x * x - c.y * py;
      y = a.x * y + c.y * px;
    } else {
      const auto tx = -a.y * y + c.x * px - c.y * py;
      const auto ty = a.y * x + c.x * py + c.y * px;
      x = a.x * x + tx;
      y = a.x * y + ty;
    }
    v[e].x = x;
    v[e].y = y;
  }
}
template <int J, int FORM, bool TWO, typename C>
__device__ __forceinline__ void oplane(C* v, C* w, const C* __restrict__ mp, int tid) {
  rlane<J, FORM>(v, mp, tid);
  if (TWO) rlane<J, FORM>(w, mp, tid);
}
template <bool TWO, typename C>
__device__ __forceinline__ void apply_signs(C* v, C* w, uint32_t S) {
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const uint32_t bit = (S >> e) & 1u;
    v[e] = flip_sign(v[e], bit);
    if (TWO) w[e] = flip_sign(w[e], bit);
  }
}

template <int K, bool TWO, typename C>
__device__ __forceinline__ void phase1(C* v, C* w, C F, bool wtriv, bool wscaled, const C* __restrict__ qt,
                                       const double* __restrict__ qa, double scl) {
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (!(e & (1 << K))) continue;
    C fe = F;
    if (!wtriv) {
      C wr;
      if (wscaled) wr = expi<C>(scl * qa[e]);
      else wr = TWO ? cconj(qt[e]) : qt[e];
      fe = cmul(fe, wr);
    }
    cmul_ip(v[e], fe);
    if (TWO) cmul_ip(w[e], fe);
  }
}

template <int K, typename C>
__device__ __forceinline__ double rgrad(const C* ps, const C* la, uint32_t creg, int pauli) {
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & (1 << K)) continue;
    if ((e & creg) != creg) continue;
    const int f = e | (1 << K);
    const C p0 = ps[e], p1 = ps[f], l0 = la[e], l1 = la[f];
    double q0r, q0i, q1r, q1i;
    if (pauli == 1) { q0r = p1.x; q0i = p1.y; q1r = p0.x; q1i = p0.y; }
    else if (pauli == 2) { q0r = p1.y; q0i = -p1.x; q1r = -p0.y; q1i = p0.x; }
    else { q0r = p0.x; q0i = p0.y; q1r = -p1.x; q1i = -p1.y; }
    acc += (double)l0.x * q0i - (double)l0.y * q0r + (double)l1.x * q1i - (double)l1.y * q1r;
  }
  return acc;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Im <lambda| P psi> over the 8 pairs of slot K, P a Pauli known at compile
// time, accumulated in the state's precision (per thread: 16 amplitudes)
template <int K, int PAULI, typename C>
__device__ __forceinline__ auto rgrad_fast(const C* ps, const C* la) {
  using T = decltype(C().x);
  // two FMA chains, one per amplitude of the pair (four FMAs per pair)
  T acc0 = 0, acc1 = 0;
  bool first = true;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e & (1 << K)) continue;
    const int f = e | (1 << K);
    const C p0 = ps[e], p1 = ps[f], l0 = la[e], l1 = la[f];
    T q0r, q0i, q1r, q1i;
    if (PAULI == 1) { q0r = p1.x; q0i = p1.y; q1r = p0.x; q1i = p0.y; }
    else if (PAULI == 2) { q0r = p1.y; q0i = -p1.x; q1r = -p0.y; q1i = p0.x; }
    else { q0r = p0.x; q0i = p0.y; q1r = -p1.x; q1i = -p1.y; }
    if (first) {
      acc0 = l0.x * q0i;
      acc1 = l1.x * q1i;
      first = false;
    } else {
      acc0 = fma_t(l0.x, q0i, acc0);
      acc1 = fma_t(l1.x, q1i, acc1);
    }
    acc0 = fma_t(-l0.y, q0r, acc0);
    acc1 = fma_t(-l1.y, q1r, acc1);
  }
  return acc0 + acc1;
}

template <typename C>
__device__ __forceinline__ double rgrad_fast_any(const C* ps, const C* la, int k, int pauli) {
#define QS_RG(K)                                               \
  case K:                                                      \
    return pauli == 1   ? (double)rgrad_fast<K, 1>(ps, la)     \
           : pauli == 2 ? (double)rgrad_fast<K, 2>(ps, la)     \
                        : (double)rgrad_fast<K, 3>(ps, la);
  switch (k) {
    QS_RG(0)
    QS_RG(1)
    QS_RG(2)
    default:
      return pauli == 1 ? (double)rgrad_fast<3, 1>(ps, la)
                        : pauli == 2 ? (double)rgrad_fast<3, 2>(ps, la) : (double)rgrad_fast<3, 3>(ps, la);
  }
#undef QS_RG
}

// sum over each 16-lane row of the wave (DPP: quad swaps, then row rotations
// by 4 and 8), returned in every lane of the row
__device__ __forceinline__ float row_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
  return x;
}
template <int CTRL> __device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row_sum(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x124>(x);
  x += dpp_d<0x128>(x);
  return x;
}
// whole-wave sum (in lane 63) from row sums held in every lane of each row:
// lane 15 of rows 0 / 2 is added into rows 1 / 3, then lane 31 into rows 2, 3
__device__ __forceinline__ float wave_sum_rows(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, false));
  return x;
}
template <int CTRL, int ROWMASK> __device__ __forceinline__ double dpp_dm(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_rows(double x) {
  x += dpp_dm<0x142, 0xA>(x);
  x += dpp_dm<0x143, 0xC>(x);
  return x;
}

template <typename C>
__device__ __forceinline__ double rgrad_any(const C* ps, const C* la, int k, uint32_t creg, int pauli) {
  switch (k) {
    case 0: return rgrad<0>(ps, la, creg, pauli);
    case 1: return rgrad<1>(ps, la, creg, pauli);
    case 2: return rgrad<2>(ps, la, creg, pauli);
    default: return rgrad<3>(ps, la, creg, pauli);
  }
}

// LDS scratch of a staged pass (besides the tile itself)
struct PassSmem {
  uint64_t hoff[128];
  double phA0[kMaxPhasePerPass];
  double phNu0[kMaxPhasePerPass][kMaxTileBits];
  double phCk[kMaxPhasePerPass][kMaxKBits];
  uint32_t phS[kMaxPhasePerPass];  // sign records: bit b set when the tile-bit-b angle / pi is odd, bit 31 for the constant
  int hb[kMaxTileBits];
  int kpos[kMaxKBits];
};
constexpr int kEnRow = kMaxTileBits + 1;  // exp(i angle) of tile bit b's coefficient, the constant's at b = kMaxTileBits

// One staged pass over tiles t_first, t_first + t_step, ... < ntiles; the
// tile-index bits above gbits are the "k bits" of the phase tables.  GUARD:
// tiles may be smaller than one full sweep of the workgroup.  Gradient
// partials are summed in LDS over the workgroup's tiles and stored once, at
// gpart[gslot * gstride + gcol + wave] (each op owns its slot, so every entry
// has exactly one writer).
template <typename R, bool TWO, int NLD, bool GUARD, bool CTRL>
__device__ __forceinline__ void pass_body(
    typename CT<R>::C* __restrict__ psi, typename CT<R>::C* __restrict__ lam, const PassGeom& g,
    const TileOp* __restrict__ ops, const StagedOp* __restrict__ sops, const StageRec* __restrict__ stages,
    const typename CT<R>::C* __restrict__ matc, const PhaseRec* __restrict__ phases,
    const int32_t* __restrict__ phlist, const double* __restrict__ dpool, const double* __restrict__ btab,
    const typename CT<R>::C* __restrict__ qtab, const double* __restrict__ qang,
    const double* __restrict__ scales, const typename CT<R>::C* __restrict__ ctab, double* __restrict__ gpart,
    int64_t gstride, int gcol,
    int64_t t_first, int64_t t_step, int64_t ntiles, int gbits, PassSmem& sm, char* smem,
    typename CT<R>::C* __restrict__ en, double* __restrict__ gacc) {
  using C = typename CT<R>::C;
  using VT = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  const int M = 1 << g.m;
  // complex64 two-state passes without controls pass both states through one
  // LDS tile in turn (SEQ): 41 KB per workgroup instead of 74 KB, three
  // workgroups per CU instead of two, for three more barriers per stage
  constexpr bool SEQ = TWO && !GUARD && !CTRL && sizeof(R) == 4 && NLD == 8;  // 12-bit tiles: one group per thread
  C* t1 = reinterpret_cast<C*>(smem);
  C* t2 = TWO && !SEQ ? t1 + M : nullptr;
  uint64_t* hoff = sm.hoff;
  auto& phA0 = sm.phA0;
  auto& phNu0 = sm.phNu0;
  auto& phCk = sm.phCk;
  int* hb = sm.hb;
  int* kpos = sm.kpos;

  const int tid = threadIdx.x;
  const int L = g.L, H = g.H, m = g.m, n = g.n;
  const int nph = g.nph, ph0 = g.ph0, nst = g.nst, st0 = g.st0, op0 = g.op0;
  const int kb = (n - m) - gbits;
  if (tid < kMaxTileBits) hb[tid] = g.hbits[tid];
  if (tid < kMaxPhasePerPass) sm.phS[tid] = 0u;
  if (TWO)
    for (int i = tid; i < kMaxGradPerPass * (kThreads / 64); i += kThreads) gacc[i] = 0.0;
  if (tid == 0) {  // global positions of the tile-index bits above the grid
    int idx = 0;
    uint64_t tm = (1ull << L) - 1;
    for (int i = 0; i < H; ++i) tm |= 1ull << g.hbits[i];
    for (int q = 0; q < n; ++q) {
      if ((tm >> q) & 1) continue;
      if (idx < kb && idx < kMaxKBits) kpos[idx] = q;
      ++idx;
    }
  }
  for (int hc = tid; hc < (1 << H); hc += kThreads) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << g.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;
  auto pos = [&](int b) { return b < L ? b : hb[b - L]; };
  // every thread moves NLD 16-byte vectors per tile and state
  auto tbase = [&](int64_t tt) {
    // the grid bits of the tile index (which differ between workgroups running
    // at the same time) fill the highest non-tile index positions, the
    // per-workgroup walk the lowest ones
    const uint64_t tr = ((uint64_t)tt >> gbits) | (((uint64_t)tt & ((1ull << gbits) - 1ull)) << kb);
    uint64_t b = tr << L;
    for (int i = 0; i < H; ++i) b = insert_zero64(b, hb[i]);
    return b;
  };
  auto gaddr = [&](uint64_t b, int u) {
    const int e = (u * kThreads + tid) * VW;
    return b | hoff[e >> L] | (uint64_t)(e & lomask);
  };
  // phase polynomials, part fixed for this workgroup (tile t0 = blockIdx.x,
  // k bits zero): constant, tile-bit coefficients and k-bit coefficients
  {
    const uint64_t base0 = tbase(t_first);
    for (int idx = tid; idx < nph * 32; idx += kThreads) {
      const int p = idx >> 5, r = idx & 31;
      const PhaseRec rec = phases[phlist[ph0 + p]];
      const double* P = dpool + rec.dpool;
      const double scl = (rec.scale_idx >= 0 ? scales[rec.scale_idx] : 1.0) * (TWO ? -1.0 : 1.0);
      int q0 = -1;
      double s = 0.0;
      if (r < m) q0 = pos(r);
      else if (r >= 14 && r - 14 < kb) {
        q0 = kpos[r - 14];
        s = P[1 + q0];
      }
      if (q0 >= 0) {
        for (uint64_t rr = base0; rr; rr &= rr - 1) s += P[1 + n + q0 * n + __builtin_ctzll(rr)];
        if (r < m) phNu0[p][r] = s * scl;
        else phCk[p][r - 14] = s * scl;
      } else if (r == 13) {
        s = P[0];
        for (uint64_t rr = base0; rr; rr &= rr - 1) {
          const int q = __builtin_ctzll(rr);
          s += P[1 + q];
          for (uint64_t r2 = rr & (rr - 1); r2; r2 &= r2 - 1) s += P[1 + n + q * n + __builtin_ctzll(r2)];
        }
        phA0[p] = s * scl;
      }
    }
    __syncthreads();
  }

  // the two-state pass runs two workgroups per CU (its tiles fill the LDS),
  // too few to hide the loads behind another workgroup's arithmetic: it
  // loads the next tile into registers while the current one is processed
  // (not in the variant with controls, whose registers are already full)
  constexpr bool PF = TWO && !GUARD && !CTRL && !SEQ;
  using NV = typename CT<R>::NV;  // native vector: stays in registers when indexed
  NV pre[PF ? 2 * NLD : 1];
#define QS_PREFETCH(TT)                                                                     \
  {                                                                                         \
    const uint64_t pb = tbase(TT);                                                          \
    _Pragma("unroll") for (int u = 0; u < NLD; ++u) pre[u] = *reinterpret_cast<const NV*>(psi + gaddr(pb, u)); \
    _Pragma("unroll") for (int u = 0; u < NLD; ++u) pre[NLD + u] = *reinterpret_cast<const NV*>(lam + gaddr(pb, u)); \
  }
  if (PF && t_first < ntiles) QS_PREFETCH(t_first);
  NV seqb[SEQ ? NLD : 1], seql[SEQ ? NLD : 1];  // SEQ: the tile's two states on their way in
  C v[NE], w[NE];  // a stage's register elements (SEQ keeps w from stage to stage)
  // walk the register elements of stage s (LDS byte offsets, Gray order)
  auto lds_walk = [&](const StageRec& sr, auto&& fn) {
    constexpr uint32_t CBw = sizeof(C) == 8 ? 3 : 4;
    const uint32_t i0 = swz<R>(1u << sr.rb[0]) << CBw, i1 = swz<R>(1u << sr.rb[1]) << CBw;
    const uint32_t i2 = swz<R>(1u << sr.rb[2]) << CBw, i3 = swz<R>(1u << sr.rb[3]) << CBw;
    uint32_t ad = swz<R>(insert_zeros((uint32_t)tid, sr.rbmask)) << CBw;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      if (i) {
        const int fb = __builtin_ctz(i);
        ad ^= fb == 0 ? i0 : fb == 1 ? i1 : fb == 2 ? i2 : i3;
        asm volatile("" : "+v"(ad));
      }
      fn(ad, i ^ (i >> 1));
    }
  };

  for (int64_t t = t_first; t < ntiles; t += t_step) {
    const uint64_t base = tbase(t);
    if (PF) {
#pragma unroll
      for (int u = 0; u < NLD; ++u) {
        const int e = swz<R>((u * kThreads + tid) * VW);
        *reinterpret_cast<NV*>(t1 + e) = pre[u];
        *reinterpret_cast<NV*>(t2 + e) = pre[NLD + u];
      }
    } else if (SEQ) {
#pragma unroll
      for (int u = 0; u < NLD; ++u) seqb[u] = *reinterpret_cast<const NV*>(psi + gaddr(base, u));
#pragma unroll
      for (int u = 0; u < NLD; ++u) *reinterpret_cast<NV*>(t1 + swz<R>((u * kThreads + tid) * VW)) = seqb[u];
    } else {
      for (int half = 0; half < (TWO ? 2 : 1); ++half) {
        const C* src = half ? lam : psi;
        C* dst = half ? t2 : t1;
        // issue every load of the tile before the first LDS write; threads
        // past a small tile load its first vector instead (every element of
        // buf is assigned, so it stays in registers) and drop it
        VT buf[NLD];
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
          const bool ok = !GUARD || (u * kThreads + tid) * VW < M;
          buf[u] = *reinterpret_cast<const VT*>(src + (ok ? gaddr(base, u) : base));
        }
#pragma unroll
        for (int u = 0; u < NLD; ++u)
          if (!GUARD || (u * kThreads + tid) * VW < M)
            *reinterpret_cast<VT*>(dst + swz<R>((u * kThreads + tid) * VW)) = buf[u];
      }
    }
    // per-tile coefficients of the pass's phase polynomials (the part of theta
    // fixed by the bits outside the tile) from the workgroup part and the k bits
    {
      const uint32_t kk = (uint32_t)((uint64_t)t >> gbits);
      for (int idx = tid; idx < nph * 16; idx += kThreads) {
        const int p = idx >> 4, b = idx & 15;
        const PhaseRec rec = phases[phlist[ph0 + p]];
        const double scl = (rec.scale_idx >= 0 ? scales[rec.scale_idx] : 1.0) * (TWO ? -1.0 : 1.0);
        const double* kt = btab + rec.kt_off;
        if (b < m) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < kMaxKBits; ++j)
            if ((kk >> j) & 1) s += kt[b * kMaxKBits + j];
          const double a = phNu0[p][b] + scl * s;
          // a sign record (every angle a multiple of pi: no complex factors,
          // ctab_n = 0) needs only the parities, the others only the factors
          if (rec.ctab_n == 0) {
            if (pi_parity(a)) atomicOr(&sm.phS[p], 1u << b);
          } else {
            en[p * kEnRow + b] = expi<C>(a);
          }
        } else if (b == 15) {
          double s = phA0[p];
#pragma unroll
          for (int j = 0; j < kMaxKBits; ++j)
            if ((kk >> j) & 1) s += phCk[p][j];
          const double a = s + scl * kt[m * kMaxKBits + kk];
          if (rec.ctab_n == 0) {
            if (pi_parity(a)) atomicOr(&sm.phS[p], 1u << 31);
          } else {
            en[p * kEnRow + kMaxTileBits] = expi<C>(a);
          }
        }
      }
      __syncthreads();
    }
    if (PF && t + t_step < ntiles) QS_PREFETCH(t + t_step);  // the LDS copies of pre are done
#undef QS_PREFETCH

    bool neg = false;  // odd count of shear-form rotations with sign -1: negate after the last stage
    for (int si = 0; si < nst; ++si) {
      const StageRec st = stages[st0 + (TWO ? nst - 1 - si : si)];
      // register element e sits at tile index jg | jr(e), jr(e) = the bits of e
      // placed at the stage's register bits.  The swizzle is linear over
      // GF(2) and jg, jr(e) are disjoint, so its LDS byte offset is
      // swz(jg) * sizeof(C) XOR sr(e), sr(e) the XOR of four uniform images.
      constexpr uint32_t CB = sizeof(C) == 8 ? 3 : 4;
      const uint32_t s0 = swz<R>(1u << st.rb[0]) << CB, s1 = swz<R>(1u << st.rb[1]) << CB;
      const uint32_t s2 = swz<R>(1u << st.rb[2]) << CB, s3 = swz<R>(1u << st.rb[3]) << CB;
      // walk the sixteen elements in Gray-code order g(i) = i ^ (i >> 1): step i
      // flips slot bit ctz(i), i.e. XORs one of the four uniform images into
      // the address; the empty asm keeps the chain from being folded into
      // sixteen precomputed constants (which costs scalar registers)
      auto step = [&](uint32_t& ad, int i) {
        const int fb = __builtin_ctz(i);
        ad ^= fb == 0 ? s0 : fb == 1 ? s1 : fb == 2 ? s2 : s3;
        asm volatile("" : "+v"(ad));
      };
      char* const b1 = reinterpret_cast<char*>(t1);
      char* const b2 = reinterpret_cast<char*>(t2);
      for (int gb = 0; gb < (M >> NR); gb += kThreads) {
        const bool valid = !GUARD || gb + tid < (M >> NR);
        const uint32_t jg = valid ? insert_zeros((uint32_t)(gb + tid), st.rbmask) : 0u;
        const int grp = valid ? gb + tid : 0;  // per-group table row (threads past the tile read row 0)
        uint32_t A = swz<R>(jg) << CB;
        {
          uint32_t ad = A;
#pragma unroll
          for (int i = 0; i < NE; ++i) {
            if (i) step(ad, i);
            const int e = i ^ (i >> 1);
            v[e] = *reinterpret_cast<const C*>(b1 + ad);
            if (TWO && !SEQ) w[e] = *reinterpret_cast<const C*>(b2 + ad);
          }
        }
        if (SEQ) {  // lambda through the buffer psi has just left
          __syncthreads();
          if (si == 0) {  // lambda's tile arrives now: fewer registers live across the set-up
#pragma unroll
            for (int u = 0; u < NLD; ++u) seql[u] = *reinterpret_cast<const NV*>(lam + gaddr(base, u));
#pragma unroll
            for (int u = 0; u < NLD; ++u) *reinterpret_cast<NV*>(t1 + swz<R>((u * kThreads + tid) * VW)) = seql[u];
          } else {
            lds_walk(stages[st0 + (nst - si)], [&](uint32_t ad, int e) { *reinterpret_cast<C*>(b1 + ad) = w[e]; });
          }
          __syncthreads();
          lds_walk(st, [&](uint32_t ad, int e) { w[e] = *reinterpret_cast<const C*>(b1 + ad); });
        }
        // an empty asm that "redefines" A: the scatter recomputes its
        // addresses instead of keeping sixteen of them live across the ops
        asm volatile("" : "+v"(A));
        // sign mask of a phase whose coefficients are all multiples of pi:
        // the factor of register element e is (-1)^bit e.  Every angle is a
        // multiple of pi, so the parity of a sum is the XOR of the parities:
        // tile part from phS, group part from the bit-sliced table (one
        // 64-bit word per wave and slice: scalar loads)
        auto sign_mask = [&](const StagedOp& so, const StageRec& sr, int grp, uint32_t jgl) -> uint32_t {
          const int p = so.ph & 0xFF;
          const int nw = ((M >> NR) + 63) >> 6;
          const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)grp >> 6);
          const uint64_t* sb = reinterpret_cast<const uint64_t*>(btab + so.tab) + wv;
          const uint32_t ln = (uint32_t)grp & 63u;
          auto gbit = [&](int sl) { return (uint32_t)(sb[sl * nw] >> ln) & 1u; };
          const uint32_t ts = sm.phS[p];
          uint32_t S;
          if ((so.ph >> 11) & 1) {
            const int kbs = (so.ph >> 8) & 3;
            const int rbk = kbs == 0 ? sr.rb[0] : kbs == 1 ? sr.rb[1] : kbs == 2 ? sr.rb[2] : sr.rb[3];
            S = (((ts >> rbk) ^ gbit(1 + kbs)) & 1u) ? slot_pattern(kbs) : 0u;
          } else {
            S = (((uint32_t)__builtin_popcount(ts & jgl) ^ (ts >> 31) ^ gbit(0)) & 1u) ? 0xFFFFu : 0u;
            if (((ts >> sr.rb[0]) ^ gbit(1)) & 1u) S ^= 0xAAAAu;
            if (((ts >> sr.rb[1]) ^ gbit(2)) & 1u) S ^= 0xCCCCu;
            if (((ts >> sr.rb[2]) ^ gbit(3)) & 1u) S ^= 0xF0F0u;
            if (((ts >> sr.rb[3]) ^ gbit(4)) & 1u) S ^= 0xFF00u;
          }
          return S ^ ((uint32_t)so.ph >> 16);
        };
        // general phase: factor of register element e = exp(i theta_tile) *
        // exp(i beta_0) * prod_{tile bits r in jg} EN[r] * prod_{k in e}
        // EN[rb_k] exp(i beta_k) * exp(i Q_R(e)), every factor from a table
        auto phase_general = [&](const StagedOp& so, const StageRec& sr, int grp, uint32_t jgl) {
          const int p = so.ph & 0xFF;
          const C* bc = ctab + so.tab + grp * (NR + 1);
          const C* wc = ctab + so.tab + (so.mat - NE);
          auto EN = [&](int b) { return en[p * kEnRow + b]; };
          auto B = [&](int k) { return TWO ? cconj(bc[k]) : bc[k]; };
          const bool wtriv = (so.ph >> 10) & 1;
          C f = cmul(EN(kMaxTileBits), B(0));
          for (uint32_t r = jgl; r; r &= r - 1) f = cmul(f, EN(__builtin_ctz(r)));
          const C F0 = cmul(EN(sr.rb[0]), B(1));
          const C F1 = cmul(EN(sr.rb[1]), B(2));
          const C F2 = cmul(EN(sr.rb[2]), B(3));
          const C F3 = cmul(EN(sr.rb[3]), B(4));
          auto apply = [&](int e, C fe) {
            if (!wtriv) fe = cmul(fe, TWO ? cconj(wc[e]) : wc[e]);
            cmul_ip(v[e], fe);
            if (TWO) cmul_ip(w[e], fe);
          };
          // Gray-code order with one running factor: each step sets a bit
          // (times F_k) or clears one (times conj F_k, |F_k| = 1)
          apply(0, f);
          f = cmul(f, F0); apply(1, f);
          f = cmul(f, F1); apply(3, f);
          f = cmul(f, cconj(F0)); apply(2, f);
          f = cmul(f, F2); apply(6, f);
          f = cmul(f, F0); apply(7, f);
          f = cmul(f, cconj(F1)); apply(5, f);
          f = cmul(f, cconj(F0)); apply(4, f);
          f = cmul(f, F3); apply(12, f);
          f = cmul(f, F0); apply(13, f);
          f = cmul(f, F1); apply(15, f);
          f = cmul(f, cconj(F0)); apply(14, f);
          f = cmul(f, cconj(F2)); apply(10, f);
          f = cmul(f, F0); apply(11, f);
          f = cmul(f, cconj(F1)); apply(9, f);
          f = cmul(f, cconj(F0)); apply(8, f);
        };
        // every term holds register slot KBS: factor 1 where that bit is 0
        auto phase_single = [&](const StagedOp& so, const StageRec& sr, int grp, auto kbs_c) {
          constexpr int KBS = decltype(kbs_c)::value;
          const int p = so.ph & 0xFF;
          const C* bc = ctab + so.tab + grp * (NR + 1);
          const C* wc = ctab + so.tab + (so.mat - NE);
          const C b = TWO ? cconj(bc[1 + KBS]) : bc[1 + KBS];
          const C F = cmul(en[p * kEnRow + sr.rb[KBS]], b);
          const bool wtriv = (so.ph >> 10) & 1;
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            if (!((e >> KBS) & 1)) continue;
            const C fe = wtriv ? F : cmul(F, TWO ? cconj(wc[e]) : wc[e]);
            cmul_ip(v[e], fe);
            if (TWO) cmul_ip(w[e], fe);
          }
        };
        // the stage's op records in the order they run, each fetched one op
        // ahead: its scalar loads are in flight while the previous op runs
        const StagedOp* __restrict__ sop = sops + op0 + st.op0;
        const int nso = st.nops;
        StagedOp cur = sop[TWO ? nso - 1 : 0], nx;
        for (int oi = 0; oi < nso; ++oi, cur = nx) {
          nx = sop[TWO ? (nso - 2 - oi > 0 ? nso - 2 - oi : 0) : (oi + 1 < nso ? oi + 1 : oi)];
          const uint32_t cin = cur.ctl & 0xFFFFu, creg = cur.ctl >> 16;
          const uint64_t cout = ((uint64_t)cur.cout_hi << 32) | cur.cout_lo;
          const bool uact = (base & cout) == cout;  // uniform
          bool act = valid && uact;
          if (cin) act = act && ((jg & cin) == cin);
          if (TWO && cur.grad >= 0) {
            // per-thread partial, summed across the wave with DPP; lane 63 adds
            // the wave's total to its slot (a single writer per slot)
            using T = decltype(C().x);
            const int gk = (cur.grad >> 12) & 3, gp = (cur.grad >> 8) & 3;
            T pg = 0;
            if (creg == 0 && cin == 0) {
              if (valid) pg = (T)rgrad_fast_any(v, w, gk, gp);
            } else if (CTRL && act) {
              pg = (T)rgrad_any(v, w, gk, creg, gp);
            }
            if (!uact) pg = 0;
            pg = wave_sum_rows(row_sum(pg));
            // no returned value: nothing waits on the LDS add
            if ((tid & 63) == 63) atomicAdd(&gacc[(cur.grad & 0xFF) * (kThreads / 64) + (tid >> 6)], (double)pg);
          }
          if (!uact) continue;
          if (cin == 0 && creg == 0) {
            // one flat switch over a uniform opcode with compile-time slots:
            // straight-line cases keep the register array in place
            const C* m1 = matc + cur.mat + (TWO ? 4 : 0);
            const C* m2 = matc + cur.mat + (TWO ? 16 : 0);
            const C* sp = matc + cur.mat + (TWO ? 10 : 8);
            switch (cur.opc) {
              case 0: op1<0, false, TWO>(v, w, m1); break;
              case 1: op1<1, false, TWO>(v, w, m1); break;
              case 2: op1<2, false, TWO>(v, w, m1); break;
              case 3: op1<3, false, TWO>(v, w, m1); break;
              case 4: op1<0, true, TWO>(v, w, m1); break;
              case 5: op1<1, true, TWO>(v, w, m1); break;
              case 6: op1<2, true, TWO>(v, w, m1); break;
              case 7: op1<3, true, TWO>(v, w, m1); break;
              case 8: op2<1, 0, TWO>(v, w, m2); break;
              case 9: op2<2, 0, TWO>(v, w, m2); break;
              case 10: op2<2, 1, TWO>(v, w, m2); break;
              case 11: op2<3, 0, TWO>(v, w, m2); break;
              case 12: op2<3, 1, TWO>(v, w, m2); break;
              case 13: op2<3, 2, TWO>(v, w, m2); break;
              case 14: apply_signs<TWO>(v, w, sign_mask(cur, st, grp, jg)); break;
              case 19: phase_general(cur, st, grp, jg); break;
              case 20: phase_single(cur, st, grp, std::integral_constant<int, 0>()); break;
              case 21: phase_single(cur, st, grp, std::integral_constant<int, 1>()); break;
              case 22: phase_single(cur, st, grp, std::integral_constant<int, 2>()); break;
              case 23: phase_single(cur, st, grp, std::integral_constant<int, 3>()); break;
              case 24: op1d<0, TWO>(v, w, m1); break;
              case 25: op1d<1, TWO>(v, w, m1); break;
              case 26: op1d<2, TWO>(v, w, m1); break;
              case 27: op1d<3, TWO>(v, w, m1); break;
              case 28: op1x<0, TWO>(v, w, m1); break;
              case 29: op1x<1, TWO>(v, w, m1); break;
              case 30: op1x<2, TWO>(v, w, m1); break;
              case 31: op1x<3, TWO>(v, w, m1); break;
              case 32: op1s<0, false, TWO>(v, w, sp); break;
              case 33: op1s<1, false, TWO>(v, w, sp); break;
              case 34: op1s<2, false, TWO>(v, w, sp); break;
              case 35: op1s<3, false, TWO>(v, w, sp); break;
              case 36: op1s<0, true, TWO>(v, w, sp); break;
              case 37: op1s<1, true, TWO>(v, w, sp); break;
              case 38: op1s<2, true, TWO>(v, w, sp); break;
              case 39: op1s<3, true, TWO>(v, w, sp); break;
              case 40: if constexpr (!TWO) oplane<0, 0, TWO>(v, w, m1, tid); break;
              case 41: if constexpr (!TWO) oplane<1, 0, TWO>(v, w, m1, tid); break;
              case 42: if constexpr (!TWO) oplane<2, 0, TWO>(v, w, m1, tid); break;
              case 43: if constexpr (!TWO) oplane<3, 0, TWO>(v, w, m1, tid); break;
              case 44: if constexpr (!TWO) oplane<0, 1, TWO>(v, w, m1, tid); break;
              case 45: if constexpr (!TWO) oplane<1, 1, TWO>(v, w, m1, tid); break;
              case 46: if constexpr (!TWO) oplane<2, 1, TWO>(v, w, m1, tid); break;
              case 47: if constexpr (!TWO) oplane<3, 1, TWO>(v, w, m1, tid); break;
              case 48: if constexpr (!TWO) oplane<0, 2, TWO>(v, w, m1, tid); break;
              case 49: if constexpr (!TWO) oplane<1, 2, TWO>(v, w, m1, tid); break;
              case 50: if constexpr (!TWO) oplane<2, 2, TWO>(v, w, m1, tid); break;
              case 51: if constexpr (!TWO) oplane<3, 2, TWO>(v, w, m1, tid); break;
              case 52: if constexpr (!TWO) oplane<0, 3, TWO>(v, w, m1, tid); break;
              case 53: if constexpr (!TWO) oplane<1, 3, TWO>(v, w, m1, tid); break;
              case 54: if constexpr (!TWO) oplane<2, 3, TWO>(v, w, m1, tid); break;
              case 55: if constexpr (!TWO) oplane<3, 3, TWO>(v, w, m1, tid); break;
              default: break;
            }
            if (cur.opc >= 32 && cur.opc < 40) neg = neg != (sp[1].x < 0);
            continue;
          }
          // controlled ops (register-slot or in-tile controls): predicated per
          // thread, compiled only into the variant for passes that hold them
          if (!CTRL || !act || cur.tab < 0) continue;
          const int k0 = cur.tab & 15, k1 = (cur.tab >> 4) & 15;
          if (!((cur.tab >> 9) & 1)) {
            const C* mp = matc + cur.mat + (TWO ? 4 : 0);
            const C a = mp[0], b = mp[1], c = mp[2], d = mp[3];
            if ((cur.tab >> 8) & 1) {
              r1_any<true>(v, k0, a, b, c, d, creg);
              if (TWO) r1_any<true>(w, k0, a, b, c, d, creg);
            } else {
              r1_any<false>(v, k0, a, b, c, d, creg);
              if (TWO) r1_any<false>(w, k0, a, b, c, d, creg);
            }
          } else {
            const C* mp = matc + cur.mat + (TWO ? 16 : 0);
            r2_any(v, k0, k1, mp, creg);
            if (TWO) r2_any(w, k0, k1, mp, creg);
          }
        }
        if (si == nst - 1 && neg) {  // the tile's shear-form rotations left it negated
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            v[e].x = -v[e].x;
            v[e].y = -v[e].y;
            if (TWO) {
              w[e].x = -w[e].x;
              w[e].y = -w[e].y;
            }
          }
        }
        // (no barrier before the scatter in the two-state pass: every thread
        // writes psi back to exactly the buffer entries it read lambda from)
        if (valid) {
          uint32_t ad = A;
#pragma unroll
          for (int i = 0; i < NE; ++i) {
            if (i) step(ad, i);
            const int e = i ^ (i >> 1);
            *reinterpret_cast<C*>(b1 + ad) = v[e];
            if (TWO && !SEQ) *reinterpret_cast<C*>(b2 + ad) = w[e];
          }
        }
      }
      __syncthreads();
    }
    if (tid < nph) sm.phS[tid] = 0u;  // the stages are done with it; the next tile ORs afresh

    for (int half = 0; half < (TWO ? 2 : 1); ++half) {
      C* dstg = half ? lam : psi;
      const C* src = half && !SEQ ? t2 : t1;
      if (SEQ && half) {  // lambda's last stage registers into the buffer psi has left
        __syncthreads();
        lds_walk(stages[st0], [&](uint32_t ad, int e) { *reinterpret_cast<C*>(reinterpret_cast<char*>(t1) + ad) = w[e]; });
        __syncthreads();
      }
      VT buf[NLD];
#pragma unroll
      for (int u = 0; u < NLD; ++u) {
        const bool ok = !GUARD || (u * kThreads + tid) * VW < M;
        buf[u] = *reinterpret_cast<const VT*>(src + swz<R>(ok ? (u * kThreads + tid) * VW : 0));
      }
#pragma unroll
      for (int u = 0; u < NLD; ++u)
        if (!GUARD || (u * kThreads + tid) * VW < M) *reinterpret_cast<VT*>(dstg + gaddr(base, u)) = buf[u];
    }
    __syncthreads();
  }
  if (TWO) {  // the partials are complete after the last barrier above
    for (int i = tid; i < g.nops * (kThreads / 64); i += kThreads) {
      const int oi = i / (kThreads / 64), w = i % (kThreads / 64);
      const TileOp& op = ops[op0 + oi];
      if (op.kind == OP_ROT && op.gslot >= 0)
        gpart[(int64_t)op.gslot * gstride + gcol + w] = gacc[op.aux * (kThreads / 64) + w];
    }
    __syncthreads();  // a following pass in the same workgroup reuses gacc
  }
}

// The complex64 two-state pass without controls is asked to fit four waves per
// SIMD (at most 128 registers; its 40 KB of LDS already lets four workgroups
// share a CU): 156 registers and three waves before, and the adjoint of the
// 30-qubit variational circuit took 193 ms instead of 173 ms.  Every other
// instance keeps the compiler's choice (forcing complex128 to four waves
// spills to scratch).
template <typename R, bool TWO, bool CTRL, int NLD> struct Tile2Waves {
  static constexpr int value = (sizeof(R) == 4 && TWO && !CTRL && NLD == 8) ? 4 : 1;
};

template <typename R, bool TWO, int NLD, bool CTRL>
__global__ __launch_bounds__(256, (Tile2Waves<R, TWO, CTRL, NLD>::value)) void k_tile2(
    typename CT<R>::C* __restrict__ psi, typename CT<R>::C* __restrict__ lam, const PassGeom g,
    const TileOp* __restrict__ ops, const StagedOp* __restrict__ sops, const StageRec* __restrict__ stages,
    const typename CT<R>::C* __restrict__ matc, const PhaseRec* __restrict__ phases,
    const int32_t* __restrict__ phlist, const double* __restrict__ dpool, const double* __restrict__ btab,
    const typename CT<R>::C* __restrict__ qtab, const double* __restrict__ qang,
    const double* __restrict__ scales, const typename CT<R>::C* __restrict__ ctab, double* __restrict__ gpart,
    int64_t ntiles) {
  extern __shared__ __align__(16) char smem[];
  __shared__ PassSmem sm;
  __shared__ typename CT<R>::C en[kMaxPhasePerPass * kEnRow];
  __shared__ double gacc[TWO ? kMaxGradPerPass * (kThreads / 64) : 1];
  pass_body<R, TWO, NLD, false, CTRL>(psi, lam, g, ops, sops, stages, matc, phases, phlist, dpool, btab, qtab, qang, scales,
                                ctab, gpart, kGradStride, blockIdx.x * 4, blockIdx.x, gridDim.x, ntiles,
                                __builtin_ctz(gridDim.x), sm, smem, en, gacc);
}

// ----------------------------------------------------------------------------
// dense k-qubit block (k = 4, 5) on matrix cores.  A tile holds the 2^k target
// values of 128 columns (the 7 lowest non-target bits); with the gate realified
// as GR = [[Gr, -Gi], [Gi, Gr]] (2^(k+1) square) every column is updated by one
// real product [Yr; Yi] = GR [Xr; Xi].  v_mfma_*_16x16x4: A is 16x4 (lane l
// holds row l%16, column l/16), B is 4x16 (row l/16, column l%16), D is 16x16
// with column l%16 and row 4*(l/16)+v (f32) or 4*v+l/16 (f64) in element v.
// A fused pass applies a second k-qubit block on other bits of the same tile:
// its targets lie among the first block's columns and the other way round, so
// the tile is taken from HBM once for both.
// ----------------------------------------------------------------------------
struct MfmaArgs {
  int tl[5];   // tile-local position of target t (t = 0 is the matrix MSB)
  int tl2[5];  // fused passes: the same for the second block
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R> struct MfmaT;
template <> struct MfmaT<float> {
  using Acc = f32x4;
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row held in accumulator element v (column = lane % 16)
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct MfmaT<double> {
  using Acc = f64x4;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the f64 form interleaves its output rows across the four lane groups
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// row and column offsets of a block with targets tl inside the tile
template <int K, int NCOL>
__device__ __forceinline__ void mfma_offsets(const int (&tl)[5], uint32_t* rowoff, uint32_t* coloff, int tid) {
  uint32_t tmask = 0;
#pragma unroll
  for (int t = 0; t < K; ++t) tmask |= 1u << tl[t];
  for (int r = tid; r < (1 << K); r += kThreads) {
    uint32_t o = 0;
#pragma unroll
    for (int t = 0; t < K; ++t)
      if ((r >> (K - 1 - t)) & 1) o |= 1u << tl[t];
    rowoff[r] = o;
  }
  for (int c = tid; c < NCOL; c += kThreads) coloff[c] = insert_zeros((uint32_t)c, tmask);
}

// A fragments of the realified gate, resident for the whole launch
template <typename R, int K>
__device__ __forceinline__ void mfma_frags(const double* __restrict__ mat, R (&a)[2 * (1 << K) / 16][2 * (1 << K) / 4],
                                           int lane) {
  constexpr int D = 1 << K;
#pragma unroll
  for (int rb = 0; rb < 2 * D / 16; ++rb)
#pragma unroll
    for (int ks = 0; ks < 2 * D / 4; ++ks) {
      const int i = 16 * rb + (lane & 15), j = 4 * ks + (lane >> 4);
      const int gi = i & (D - 1), gj = j & (D - 1);
      const double re = mat[2 * (gi * D + gj)], im = mat[2 * (gi * D + gj) + 1];
      a[rb][ks] = (R)((i < D) == (j < D) ? re : (i < D ? -im : im));
    }
}

// one block on the tile in LDS: each wave takes 16 columns at a time, reads
// their 2^K values, and writes the products back to the same entries
template <typename R, int K>
__device__ __forceinline__ void mfma_apply(typename CT<R>::C* tile, const uint32_t* rowoff, const uint32_t* coloff,
                                           const R (&a)[2 * (1 << K) / 16][2 * (1 << K) / 4], int lane, int wave) {
  using C = typename CT<R>::C;
  using Acc = typename MfmaT<R>::Acc;
  constexpr int D = 1 << K, RB = 2 * D / 16, KS = 2 * D / 4, NCOL = 128;
  for (int cb = wave; cb < NCOL / 16; cb += (int)(kThreads >> 6)) {
    const uint32_t co = coloff[16 * cb + (lane & 15)];
    Acc acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int row = 4 * ks + (lane >> 4);  // realified row of X
      const C x = tile[swz<R>(rowoff[row & (D - 1)] | co)];
      const R bval = row < D ? x.x : x.y;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = MfmaT<R>::mma(a[rb][ks], bval, acc[rb]);
    }
    // output row 16*rb + 4*(lane/16) + v: real parts in the first RB/2 blocks,
    // imaginary parts of the same rows RB/2 blocks later
#pragma unroll
    for (int rb = 0; rb < RB / 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + MfmaT<R>::out_row(lane, v);
        tile[swz<R>(rowoff[row] | co)] = mk<C>(acc[rb][v], acc[rb + RB / 2][v]);
      }
  }
}

template <typename R, int K, int NLD, bool TWO_M>
__global__ __launch_bounds__(256) void k_mfma(typename CT<R>::C* __restrict__ psi, const PassGeom g,
                                              const MfmaArgs ma, const double* __restrict__ mat,
                                              const double* __restrict__ mat2, int64_t ntiles) {
  using C = typename CT<R>::C;
  using VT = typename CT<R>::V;
  constexpr int VW = CT<R>::VW;
  constexpr int D = 1 << K;      // complex dimension
  constexpr int RB = 2 * D / 16;  // 16-row blocks of the realified output
  constexpr int KS = 2 * D / 4;   // 4-deep steps of the contraction
  constexpr int NCOL = 128;      // columns per tile
  constexpr int NB = TWO_M ? 2 : 1;
  extern __shared__ __align__(16) char smem[];
  C* tile = reinterpret_cast<C*>(smem);
  __shared__ uint32_t rowoff[NB][D];
  __shared__ uint32_t coloff[NB][NCOL];
  __shared__ uint64_t hoff[128];
  __shared__ int hb[kMaxTileBits];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = g.L, H = g.H;
  if (tid < kMaxTileBits) hb[tid] = g.hbits[tid];
  __syncthreads();
  for (int hc = tid; hc < (1 << H); hc += kThreads) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << hb[i];
    hoff[hc] = off;
  }
  mfma_offsets<K, NCOL>(ma.tl, rowoff[0], coloff[0], tid);
  if constexpr (TWO_M) mfma_offsets<K, NCOL>(ma.tl2, rowoff[NB - 1], coloff[NB - 1], tid);
  R a[RB][KS], a2[TWO_M ? RB : 1][TWO_M ? KS : 1];
  mfma_frags<R, K>(mat, a, lane);
  if constexpr (TWO_M) mfma_frags<R, K>(mat2, a2, lane);
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint64_t base = spread_tile((uint64_t)t, g.n - g.m) << L;
    for (int i = 0; i < H; ++i) base = insert_zero64(base, hb[i]);
    VT buf[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e = (u * kThreads + tid) * VW;
      buf[u] = *reinterpret_cast<const VT*>(psi + (base | hoff[e >> L] | (uint64_t)(e & lomask)));
    }
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e = (u * kThreads + tid) * VW;
      *reinterpret_cast<VT*>(tile + swz<R>(e)) = buf[u];
    }
    __syncthreads();
    mfma_apply<R, K>(tile, rowoff[0], coloff[0], a, lane, wave);
    if constexpr (TWO_M) {
      __syncthreads();
      mfma_apply<R, K>(tile, rowoff[NB - 1], coloff[NB - 1], a2, lane, wave);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e = (u * kThreads + tid) * VW;
      buf[u] = *reinterpret_cast<const VT*>(tile + swz<R>(e));
    }
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e = (u * kThreads + tid) * VW;
      *reinterpret_cast<VT*>(psi + (base | hoff[e >> L] | (uint64_t)(e & lomask))) = buf[u];
    }
    __syncthreads();
  }
}

// matrices of a rotation exp(-i theta P/2) (slot 0..3) and of its inverse
// (4..7); then, for X and Y, the three-shear form of the plane rotation by
// phi = theta/2 (slots 8..9, inverse 10..11): phi = phi' + k pi with
// |phi'| <= pi/2, slot 8/10 = (tan(phi'/2), sin(phi')), slot 9/11 = ((-1)^k, 0)
template <typename C>
__device__ __forceinline__ void rot_fill(C* m, int pauli, double theta) {
  double s, c;
  sincos(0.5 * theta, &s, &c);
  for (int inv = 0; inv < 2; ++inv) {
    const double si = inv ? -s : s;
    C* o = m + 4 * inv;
    if (pauli == 1) {
      o[0] = mk<C>(c, 0); o[1] = mk<C>(0, -si); o[2] = mk<C>(0, -si); o[3] = mk<C>(c, 0);
    } else if (pauli == 2) {
      o[0] = mk<C>(c, 0); o[1] = mk<C>(-si, 0); o[2] = mk<C>(si, 0); o[3] = mk<C>(c, 0);
    } else {
      o[0] = mk<C>(c, -si); o[1] = mk<C>(0, 0); o[2] = mk<C>(0, 0); o[3] = mk<C>(c, si);
    }
  }
  if (pauli == 1 || pauli == 2) {
    const double phi = 0.5 * theta, k = rint(phi * 0.3183098861837907);
    const double r = phi - 3.141592653589793 * k;
    const double t = tan(0.5 * r), sr = sin(r), sg = fmod(k, 2.0) == 0.0 ? 1.0 : -1.0;
    m[8] = mk<C>(t, sr);
    m[9] = mk<C>(sg, 0);
    m[10] = mk<C>(-t, -sr);
    m[11] = mk<C>(sg, 0);
  }
}

// ----------------------------------------------------------------------------
// batched instances, one level (one pass of every instance that has it) per
// launch; each workgroup takes one tile of one instance's pass
// ----------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_batch_rot(const BatchArgs a) {
  using C = typename CT<R>::C;
  const int o = blockIdx.x * kThreads + threadIdx.x;
  if (o >= a.nops_total) return;
  const TileOp op = a.dp.ops[o];
  if (op.kind != OP_ROT || op.mat < 0) return;
  const BatchInst& in = a.insts[a.op_inst[o]];
  rot_fill(reinterpret_cast<C*>(a.dp.matc) + in.mat_base + op.mat, op.pauli,
           op.sign * a.params[in.param_base + op.pidx]);
}

// psi = |0..0> over one chunk of one instance
template <typename R>
__global__ __launch_bounds__(256) void k_batch_init(const BatchArgs a, const BatchItem* __restrict__ items) {
  using C = typename CT<R>::C;
  const BatchItem it = items[blockIdx.x];
  const BatchInst& in = a.insts[it.inst];
  C* psi = reinterpret_cast<C*>(a.states) + in.state_off;
  const int64_t N = 1ll << in.n;
  const int64_t x0 = (int64_t)it.tile << kBatchChunkBits;
  const int64_t x1 = x0 + (1ll << kBatchChunkBits) < N ? x0 + (1ll << kBatchChunkBits) : N;
  for (int64_t x = x0 + threadIdx.x; x < x1; x += kThreads) psi[x] = mk<C>(x == 0 ? 1.0 : 0.0, 0.0);
}

// complex64 forward batch passes are held to four waves per SIMD (166
// registers otherwise; an 84-byte scratch spill): the 512-instance replay
// 8.51 against 8.81 ms, energies only 2.90 against 3.16 ms.  Bounding the
// two-state batch pass as well spilled more and was slower.
template <typename R, bool TWO, int NLD, bool CTRL>
__global__ __launch_bounds__(256, (sizeof(R) == 4 && !TWO ? 4 : 1)) void k_batch_pass(const BatchArgs a, const BatchItem* __restrict__ items) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) char smem[];
  __shared__ PassSmem sm;
  __shared__ C en[kMaxPhasePerPass * kEnRow];
  __shared__ double gacc[TWO ? kMaxGradPerPass * (kThreads / 64) : 1];
  const BatchItem it = items[blockIdx.x];
  const BatchInst& in = a.insts[it.inst];
  C* psi = reinterpret_cast<C*>(a.states) + in.state_off;
  C* lam = TWO ? reinterpret_cast<C*>(a.states) + in.lam_off : nullptr;
  const PassGeom& g = (TWO ? a.geoms_adj : a.geoms)[in.pass0 + it.pass];
  const int64_t nt = 1ll << in.tbits;
  pass_body<R, TWO, NLD, true, CTRL>(
      psi, lam, g, a.dp.ops + in.ops_base, a.dp.sops + in.ops_base, a.dp.stages + in.st_base,
      reinterpret_cast<const C*>(a.dp.matc) + in.mat_base, a.dp.phases + in.ph_base, a.dp.phlist + in.phl_base,
      a.dp.dpool + in.dp_base, a.dp.btab + in.bt_base, reinterpret_cast<const C*>(a.dp.qtab) + in.qt_base,
      a.dp.qang + in.qt_base, nullptr, reinterpret_cast<const C*>(a.dp.ctab) + in.ct_base, a.gpart + in.gp_off,
      4 * nt, it.tile * 4, it.tile, nt, nt, in.tbits, sm, smem, en, gacc);
}

// energy of the diagonal observable over one chunk, lambda = d psi there
template <typename R>
__global__ __launch_bounds__(256) void k_batch_energy(const BatchArgs a, const BatchItem* __restrict__ items) {
  using C = typename CT<R>::C;
  __shared__ double red[kThreads / 64];
  const BatchItem it = items[blockIdx.x];
  const BatchInst& in = a.insts[it.inst];
  const C* psi = reinterpret_cast<const C*>(a.states) + in.state_off;
  C* lam = reinterpret_cast<C*>(a.states) + in.lam_off;
  const int64_t N = 1ll << in.n;
  const int64_t x0 = (int64_t)it.tile << kBatchChunkBits;
  const int64_t x1 = x0 + (1ll << kBatchChunkBits) < N ? x0 + (1ll << kBatchChunkBits) : N;
  double acc = 0.0;
  for (int64_t x = x0 + threadIdx.x; x < x1; x += kThreads) {
    double d = 0.0;
    for (int t = 0; t < in.obs_nterms; ++t) {
      const PauliTermDev T = a.terms[in.obs_off + t];
      d += (__popcll((uint64_t)x & T.zy) & 1) ? -T.coeff : T.coeff;
    }
    const C v = psi[x];
    acc += d * ((double)v.x * v.x + (double)v.y * v.y);
    lam[x] = mk<C>(d * v.x, d * v.y);
  }
  const double e = block_sum(acc, red);
  if (threadIdx.x == 0) a.epart[in.e0 + it.tile] = e;  // the instance's chunks in index order
}

// one workgroup per instance: energy from its items in order; with grads,
// every slot summed over its tiles and waves in order, then added into the
// gradient of its parameter in slot order
__global__ __launch_bounds__(256) void k_batch_finish(const BatchArgs a, int grads) {
  const BatchInst& in = a.insts[blockIdx.x];
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int i = 0; i < in.ne; ++i) e += a.epart[in.e0 + i];
    a.energies[blockIdx.x] = e;
  }
  if (!grads) return;
  const int cols = 4 << in.tbits;
  for (int sl = threadIdx.x; sl < in.nslots; sl += kThreads) {
    const double* p = a.gpart + in.gp_off + (int64_t)sl * cols;
    double v = 0.0;
    for (int c = 0; c < cols; ++c) v += p[c];
    a.slot_sum[in.slot_base + sl] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* gr = a.grads + in.param_base;
    for (int j = 0; j < in.nparams; ++j) gr[j] = 0.0;
    for (int sl = 0; sl < in.nslots; ++sl) {
      const int pidx = a.slot_pidx[in.slot_base + sl];
      if (pidx >= 0) gr[pidx] += a.slot_sum[in.slot_base + sl];
    }
  }
}

// the unit factors of scaled phase records: exp(i s angle), s = scales[rec.scale_idx];
// one workgroup per phase record
template <typename R>
__global__ void k_phase_tabs(const PhaseRec* __restrict__ phases, const double* __restrict__ btab,
                             const double* __restrict__ qang, const double* __restrict__ scales,
                             typename CT<R>::C* __restrict__ ctab) {
  using C = typename CT<R>::C;
  const PhaseRec rec = phases[blockIdx.x];
  if (rec.scale_idx < 0 || rec.ctab_off < 0) return;
  const double sc = scales[rec.scale_idx];
  const int nb = rec.ctab_n - NE;
  for (int i = threadIdx.x; i < rec.ctab_n; i += kThreads) {
    const double a = i < nb ? btab[rec.bt_off + i] : qang[rec.wr_off + (i - nb)];
    ctab[rec.ctab_off + i] = expi<C>(sc * a);
  }
}

// forward and inverse rotation matrices, exp(-i theta P / 2) and its inverse,
// with their three-shear parameters (rot_fill)
template <typename R>
__global__ void k_rot_mats(const TileOp* __restrict__ ops, int nops, const double* __restrict__ params,
                           typename CT<R>::C* __restrict__ matc) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= nops) return;
  const TileOp op = ops[i];
  if (op.kind != OP_ROT || op.mat < 0) return;
  rot_fill(matc + op.mat, op.pauli, op.sign * params[op.pidx]);
}

hipError_t set_lds_fn(void* fn, size_t lds) {
  if (lds <= 32768) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename R> void* fn_tile(bool two) {
  return two ? (void*)k_tile<R, true> : (void*)k_tile<R, false>;
}
template <typename R, int NLD, bool CTRL> void* fn_tile2(bool two) {
  return two ? (void*)k_tile2<R, true, NLD, CTRL> : (void*)k_tile2<R, false, NLD, CTRL>;
}

template <typename R, int NLD, bool CTRL>
hipError_t launch_tile2_c(void* psi, void* psi2, const PassGeom& g, const DevPlan& dp, const double* scales,
                          double* gpart, int64_t nt, int grid, size_t lds, hipStream_t s) {
  using C = typename CT<R>::C;
  const bool two = psi2 != nullptr;
  hipError_t e = set_lds_fn(fn_tile2<R, NLD, CTRL>(two), lds);
  if (e != hipSuccess) return e;
  if (two)
    hipLaunchKernelGGL((k_tile2<R, true, NLD, CTRL>), dim3(grid), dim3(kThreads), lds, s, (C*)psi, (C*)psi2, g,
                       dp.ops, dp.sops, dp.stages, (const C*)dp.matc, dp.phases, dp.phlist, dp.dpool, dp.btab,
                       (const C*)dp.qtab, dp.qang, scales, (const C*)dp.ctab, gpart, nt);
  else
    hipLaunchKernelGGL((k_tile2<R, false, NLD, CTRL>), dim3(grid), dim3(kThreads), lds, s, (C*)psi, nullptr, g,
                       dp.ops, dp.sops, dp.stages, (const C*)dp.matc, dp.phases, dp.phlist, dp.dpool, dp.btab,
                       (const C*)dp.qtab, dp.qang, scales, (const C*)dp.ctab, gpart, nt);
  return hipGetLastError();
}

// passes without controlled ops run a variant compiled without that path
template <typename R, int NLD>
hipError_t launch_tile2_t(void* psi, void* psi2, const PassGeom& g, const DevPlan& dp, const double* params,
                          const double* scales, double* gpart, int64_t nt, int grid, size_t lds, hipStream_t s) {
  (void)params;
  if (g.ctrl) return launch_tile2_c<R, NLD, true>(psi, psi2, g, dp, scales, gpart, nt, grid, lds, s);
  return launch_tile2_c<R, NLD, false>(psi, psi2, g, dp, scales, gpart, nt, grid, lds, s);
}

}  // namespace

// ============================================================================
// launch wrappers
// ============================================================================

int tile_grid(const PassGeom& g) {
  const int64_t nt = 1ll << (g.n - g.m);
  return (int)(nt < kGridMax ? nt : kGridMax);
}

// The kernels index fixed-size LDS tables by the tile geometry: reject any
// geometry they were not written for before launching.
static bool geom_ok(const PassGeom& g) {
  if (g.n < 1 || g.n > kMaxQubits || g.m < 1 || g.m > g.n || g.m > kMaxTileBits) return false;
  if (g.L < 1 || g.L > 8 || g.H < 0 || g.H > 7 || g.L + g.H != g.m) return false;
  for (int i = 0; i < g.H; ++i) {
    if (g.hbits[i] < g.L || g.hbits[i] >= g.n) return false;
    if (i && g.hbits[i] <= g.hbits[i - 1]) return false;
  }
  return true;
}

static hipError_t set_lds(void* fn, size_t lds) {
  if (lds <= 32768) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_tile_pass(bool dbl, void* psi, void* psi2, const PassGeom& g, const DevPlan& dp,
                            const double* params, const double* scales, double* gpart, hipStream_t s) {
  if (!geom_ok(g) || g.nops < 0 || g.nops > kMaxOpsPerPass * 8) return hipErrorInvalidValue;
  const int64_t nt = 1ll << (g.n - g.m);
  const int grid = tile_grid(g);
  const size_t esz = dbl ? 16 : 8;
  const bool two = psi2 != nullptr;
  size_t lds = (size_t(1) << g.m) * esz * (two ? 2 : 1);
  if (g.kern == 2) {
    if (g.m < 12 || g.nst < 1 || g.nph < 0 || g.nph > kMaxPhasePerPass) return hipErrorInvalidValue;
    const int nld = (1 << g.m) / (kThreads * (dbl ? 1 : 2));
    // complex64 two-state passes of 12-bit tiles without controls hold one
    // tile in LDS and pass the two states through it in turn
    if (two && !dbl && !g.ctrl && nld == 8) lds = (size_t(1) << g.m) * esz;
    if (dbl && nld == 16) return launch_tile2_t<double, 16>(psi, psi2, g, dp, params, scales, gpart, nt, grid, lds, s);
    if (!dbl && nld == 8) return launch_tile2_t<float, 8>(psi, psi2, g, dp, params, scales, gpart, nt, grid, lds, s);
    if (!dbl && nld == 16) return launch_tile2_t<float, 16>(psi, psi2, g, dp, params, scales, gpart, nt, grid, lds, s);
    return hipErrorInvalidValue;
  }
  void* fn = dbl ? fn_tile<double>(two) : fn_tile<float>(two);
  {
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
  }
  if (dbl) {
    if (two)
      hipLaunchKernelGGL((k_tile<double, true>), dim3(grid), dim3(kThreads), lds, s, (double2*)psi,
                         (double2*)psi2, g, dp, params, scales, gpart, nt);
    else
      hipLaunchKernelGGL((k_tile<double, false>), dim3(grid), dim3(kThreads), lds, s, (double2*)psi, nullptr, g,
                         dp, params, scales, gpart, nt);
  } else {
    if (two)
      hipLaunchKernelGGL((k_tile<float, true>), dim3(grid), dim3(kThreads), lds, s, (float2*)psi, (float2*)psi2,
                         g, dp, params, scales, gpart, nt);
    else
      hipLaunchKernelGGL((k_tile<float, false>), dim3(grid), dim3(kThreads), lds, s, (float2*)psi, nullptr, g,
                         dp, params, scales, gpart, nt);
  }
  return hipGetLastError();
}

hipError_t launch_phase_tabs(bool dbl, const DevPlan& dp, const double* scales, hipStream_t s) {
  if (dp.nphases <= 0 || !scales) return hipSuccess;
  if (dbl)
    hipLaunchKernelGGL((k_phase_tabs<double>), dim3(dp.nphases), dim3(256), 0, s, dp.phases, dp.btab, dp.qang, scales,
                       (double2*)dp.ctab);
  else
    hipLaunchKernelGGL((k_phase_tabs<float>), dim3(dp.nphases), dim3(256), 0, s, dp.phases, dp.btab, dp.qang, scales,
                       (float2*)dp.ctab);
  return hipGetLastError();
}

hipError_t launch_rot_mats(bool dbl, const DevPlan& dp, const double* params, hipStream_t s) {
  if (dp.nops_total <= 0 || !params) return hipSuccess;
  const int grid = (dp.nops_total + 255) / 256;
  if (dbl)
    hipLaunchKernelGGL((k_rot_mats<double>), dim3(grid), dim3(256), 0, s, dp.ops, dp.nops_total, params,
                       (double2*)dp.matc);
  else
    hipLaunchKernelGGL((k_rot_mats<float>), dim3(grid), dim3(256), 0, s, dp.ops, dp.nops_total, params,
                       (float2*)dp.matc);
  return hipGetLastError();
}

template <typename R, int NLD>
hipError_t perm_launch_t(void* psi, const PassGeom& g, const PermArgs& pa, int64_t nt, int grid, size_t lds,
                         hipStream_t s) {
  hipError_t e = set_lds_fn((void*)k_perm<R, NLD>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_perm<R, NLD>), dim3(grid), dim3(kThreads), lds, s, (typename CT<R>::C*)psi, g, pa, nt);
  return hipGetLastError();
}

template <typename R>
hipError_t perm_launch(int nld, void* psi, const PassGeom& g, const PermArgs& pa, int64_t nt, int grid, size_t lds,
                       hipStream_t s) {
  switch (nld) {
    case 0: return perm_launch_t<R, 0>(psi, g, pa, nt, grid, lds, s);
    case 1: return perm_launch_t<R, 1>(psi, g, pa, nt, grid, lds, s);
    case 2: return perm_launch_t<R, 2>(psi, g, pa, nt, grid, lds, s);
    case 4: return perm_launch_t<R, 4>(psi, g, pa, nt, grid, lds, s);
    case 8: return perm_launch_t<R, 8>(psi, g, pa, nt, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int K, bool TWO_M>
hipError_t mfma_launch_t(void* psi, const PassGeom& g, const MfmaArgs& ma, const double* mat, const double* mat2,
                         hipStream_t s) {
  constexpr int NLD = (1 << (K + 7)) / (kThreads * CT<R>::VW);
  const int64_t nt = 1ll << (g.n - g.m);
  const int grid = (int)(nt < kGridMax ? nt : kGridMax);
  const size_t lds = (size_t(1) << g.m) * sizeof(typename CT<R>::C);
  hipError_t e = set_lds_fn((void*)k_mfma<R, K, NLD, TWO_M>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_mfma<R, K, NLD, TWO_M>), dim3(grid), dim3(kThreads), lds, s, (typename CT<R>::C*)psi, g, ma,
                     mat, mat2, nt);
  return hipGetLastError();
}

hipError_t launch_mfma_pass(bool dbl, void* psi, const PassGeom& g, const int* tl, int k, const double* mat,
                            const int* tl2, const double* mat2, hipStream_t s) {
  // tile = targets + 7 other bits: L may reach 12 when the targets are low bits
  if (k < 4 || k > 5 || g.m != k + 7 || g.m > g.n || g.n > kMaxQubits) return hipErrorInvalidValue;
  if (g.L < 7 || g.L > 12 || g.H < 0 || g.H > 5 || g.L + g.H != g.m) return hipErrorInvalidValue;
  for (int i = 0; i < g.H; ++i)
    if (g.hbits[i] < g.L || g.hbits[i] >= g.n || (i && g.hbits[i] <= g.hbits[i - 1])) return hipErrorInvalidValue;
  const bool two = tl2 != nullptr;
  if (two != (mat2 != nullptr)) return hipErrorInvalidValue;
  if (two && dbl && k == 5) return hipErrorInvalidValue;  // two complex128 blocks of 32 do not fit the registers
  MfmaArgs ma;
  for (int t = 0; t < 5; ++t) ma.tl[t] = ma.tl2[t] = 0;
  uint32_t seen = 0;
  for (int t = 0; t < k; ++t) {
    if (tl[t] < 0 || tl[t] >= g.m || ((seen >> tl[t]) & 1)) return hipErrorInvalidValue;
    seen |= 1u << tl[t];
    ma.tl[t] = tl[t];
  }
  for (int t = 0; two && t < k; ++t) {  // the second block's targets: other tile bits
    if (tl2[t] < 0 || tl2[t] >= g.m || ((seen >> tl2[t]) & 1)) return hipErrorInvalidValue;
    seen |= 1u << tl2[t];
    ma.tl2[t] = tl2[t];
  }
  if (dbl) {
    if (two) return mfma_launch_t<double, 4, true>(psi, g, ma, mat, mat2, s);
    if (k == 4) return mfma_launch_t<double, 4, false>(psi, g, ma, mat, nullptr, s);
    return mfma_launch_t<double, 5, false>(psi, g, ma, mat, nullptr, s);
  }
  if (k == 4) return two ? mfma_launch_t<float, 4, true>(psi, g, ma, mat, mat2, s)
                         : mfma_launch_t<float, 4, false>(psi, g, ma, mat, nullptr, s);
  return two ? mfma_launch_t<float, 5, true>(psi, g, ma, mat, mat2, s)
             : mfma_launch_t<float, 5, false>(psi, g, ma, mat, nullptr, s);
}

hipError_t launch_batch_rot(bool dbl, const BatchArgs& a, hipStream_t s) {
  if (a.nops_total <= 0) return hipSuccess;
  const int grid = (a.nops_total + kThreads - 1) / kThreads;
  if (dbl) hipLaunchKernelGGL((k_batch_rot<double>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_batch_rot<float>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_init(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (dbl) hipLaunchKernelGGL((k_batch_init<double>), dim3(nitems), dim3(kThreads), 0, s, a, items);
  else hipLaunchKernelGGL((k_batch_init<float>), dim3(nitems), dim3(kThreads), 0, s, a, items);
  return hipGetLastError();
}

template <typename R, bool TWO, int NLD, bool CTRL>
hipError_t batch_pass_t(const BatchArgs& a, const BatchItem* items, int nitems, hipStream_t s) {
  // tiles of up to 2^12 amplitudes; the two-state form keeps both in LDS
  const size_t lds = (size_t(1) << 12) * sizeof(typename CT<R>::C) * (TWO ? 2 : 1);
  hipError_t e = set_lds_fn((void*)k_batch_pass<R, TWO, NLD, CTRL>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch_pass<R, TWO, NLD, CTRL>), dim3(nitems), dim3(kThreads), lds, s, a, items);
  return hipGetLastError();
}

hipError_t launch_batch_pass(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, int dir, bool ctrl,
                             hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (dbl) {
    if (dir) return ctrl ? batch_pass_t<double, true, 16, true>(a, items, nitems, s)
                         : batch_pass_t<double, true, 16, false>(a, items, nitems, s);
    return ctrl ? batch_pass_t<double, false, 16, true>(a, items, nitems, s)
                : batch_pass_t<double, false, 16, false>(a, items, nitems, s);
  }
  if (dir) return ctrl ? batch_pass_t<float, true, 8, true>(a, items, nitems, s)
                       : batch_pass_t<float, true, 8, false>(a, items, nitems, s);
  return ctrl ? batch_pass_t<float, false, 8, true>(a, items, nitems, s)
              : batch_pass_t<float, false, 8, false>(a, items, nitems, s);
}

hipError_t launch_batch_energy(bool dbl, const BatchArgs& a, const BatchItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (dbl) hipLaunchKernelGGL((k_batch_energy<double>), dim3(nitems), dim3(kThreads), 0, s, a, items);
  else hipLaunchKernelGGL((k_batch_energy<float>), dim3(nitems), dim3(kThreads), 0, s, a, items);
  return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchArgs& a, bool grads, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_finish, dim3(a.count), dim3(kThreads), 0, s, a, grads ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_perm_pass(bool dbl, void* psi, const PassGeom& g, const int* tau, hipStream_t s) {
  PermArgs pa;
  for (int i = 0; i < kMaxQubits; ++i) pa.tau[i] = i < g.n ? tau[i] : i;
  if (!geom_ok(g)) return hipErrorInvalidValue;
  for (int i = 0; i < g.n; ++i)
    if (tau[i] < 0 || tau[i] >= g.n || tau[tau[i]] != i) return hipErrorInvalidValue;  // an involution
  {
    uint64_t tm = (1ull << g.L) - 1;  // the tile bit set must be closed under tau
    for (int i = 0; i < g.H; ++i) tm |= 1ull << g.hbits[i];
    for (int b = 0; b < g.n; ++b)
      if (((tm >> b) & 1) && !((tm >> tau[b]) & 1)) return hipErrorInvalidValue;
  }
  const int64_t nt = 1ll << (g.n - g.m);
  const int grid = (int)(nt < kGridMax ? nt : kGridMax);
  const size_t esz = dbl ? 16 : 8;
  const size_t lds = (size_t(1) << g.m) * (2 * esz + 2);
  const int nld = (1 << g.m) / (kThreads * (dbl ? 1 : 2));
  if (nld > 8) return hipErrorInvalidValue;
  return dbl ? perm_launch<double>(nld, psi, g, pa, nt, grid, lds, s)
             : perm_launch<float>(nld, psi, g, pa, nt, grid, lds, s);
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  if (bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return hipErrorInvalidValue;
  const int64_t nvec = bytes / 16;
  const int64_t chunks = nvec / (int64_t(kThreads) * kCopyUnroll);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(chunks, 4096));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, s, static_cast<u32x4*>(dst),
                     static_cast<const u32x4*>(src), nvec);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_set_basis(bool dbl, void* psi, int n, uint64_t x, hipStream_t s) {
  const int64_t N = 1ll << n;
  const int grid = (int)std::min<int64_t>((N + 255) / 256, 8192);
  if (dbl) hipLaunchKernelGGL((k_fill<double>), dim3(grid), dim3(256), 0, s, (double2*)psi, N, 0.0);
  else hipLaunchKernelGGL((k_fill<float>), dim3(grid), dim3(256), 0, s, (float2*)psi, N, 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dbl) hipLaunchKernelGGL((k_set_one<double>), dim3(1), dim3(1), 0, s, (double2*)psi, x);
  else hipLaunchKernelGGL((k_set_one<float>), dim3(1), dim3(1), 0, s, (float2*)psi, x);
  return hipGetLastError();
}

hipError_t launch_set_plus(bool dbl, void* psi, int n, hipStream_t s) {
  const int64_t N = 1ll << n;
  const double a = std::pow(2.0, -0.5 * n);
  const int grid = (int)std::min<int64_t>((N + 255) / 256, 8192);
  if (dbl) hipLaunchKernelGGL((k_fill<double>), dim3(grid), dim3(256), 0, s, (double2*)psi, N, a);
  else hipLaunchKernelGGL((k_fill<float>), dim3(grid), dim3(256), 0, s, (float2*)psi, N, a);
  return hipGetLastError();
}

hipError_t launch_sumsq(bool dbl, const void* psi, int n, double* partials, hipStream_t s) {
  const int64_t N = 1ll << n;
  const int grid = reduce_grid(N);
  if (dbl) hipLaunchKernelGGL((k_sumsq<double>), dim3(grid), dim3(256), 0, s, (const double2*)psi, N, partials);
  else hipLaunchKernelGGL((k_sumsq<float>), dim3(grid), dim3(256), 0, s, (const float2*)psi, N, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_final_sum(partials, grid, partials + kGridMax, s);
}

hipError_t launch_dot_re(bool dbl, const void* a, const void* b, int n, double* partials, hipStream_t s) {
  const int64_t N = 1ll << n;
  const int grid = reduce_grid(N);
  if (dbl)
    hipLaunchKernelGGL((k_dot_re<double>), dim3(grid), dim3(256), 0, s, (const double2*)a, (const double2*)b, N,
                       partials);
  else
    hipLaunchKernelGGL((k_dot_re<float>), dim3(grid), dim3(256), 0, s, (const float2*)a, (const float2*)b, N,
                       partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_final_sum(partials, grid, partials + kGridMax, s);
}

template <bool WRITE>
hipError_t expect_poly_t(bool dbl, const void* psi, void* lam, int n, const double* poly, const double* elo,
                         double* partials, hipStream_t s) {
  if (n < 1 || n > kMaxQubits) return hipErrorInvalidValue;
  const int lb = n < 12 ? n : 12;
  const int64_t nt = 1ll << (n - lb);
  const int grid = (int)(nt < kGridMax ? nt : kGridMax);
  if (dbl)
    hipLaunchKernelGGL((k_expect_poly<double, WRITE>), dim3(grid), dim3(256), 0, s, (const double2*)psi,
                       (double2*)lam, n, poly, elo, partials);
  else
    hipLaunchKernelGGL((k_expect_poly<float, WRITE>), dim3(grid), dim3(256), 0, s, (const float2*)psi,
                       (float2*)lam, n, poly, elo, partials);
  return hipGetLastError();
}

hipError_t launch_expect_poly(bool dbl, const void* psi, int n, const double* poly, const double* elo,
                              double* partials, hipStream_t s) {
  return expect_poly_t<false>(dbl, psi, nullptr, n, poly, elo, partials, s);
}

hipError_t launch_hpsi_poly(bool dbl, const void* psi, void* lam, int n, const double* poly, const double* elo,
                            double* partials, hipStream_t s) {
  if (!lam) return hipErrorInvalidValue;
  return expect_poly_t<true>(dbl, psi, lam, n, poly, elo, partials, s);
}

hipError_t launch_pauli_far(bool dbl, const void* psi, void* lam, int n, uint64_t flip, const PauliTermDev* terms,
                            int nterms, int first, double* partials, hipStream_t s) {
  if (n < 1 || n > kMaxQubits || (flip >> n) != 0) return hipErrorInvalidValue;
  const int grid = reduce_grid(1ll << n);
  if (dbl) {
    if (lam)
      hipLaunchKernelGGL((k_pauli_far<double, true>), dim3(grid), dim3(256), 0, s, (const double2*)psi, (double2*)lam,
                         n, flip, terms, nterms, first, partials);
    else
      hipLaunchKernelGGL((k_pauli_far<double, false>), dim3(grid), dim3(256), 0, s, (const double2*)psi, nullptr, n,
                         flip, terms, nterms, first, partials);
  } else {
    if (lam)
      hipLaunchKernelGGL((k_pauli_far<float, true>), dim3(grid), dim3(256), 0, s, (const float2*)psi, (float2*)lam, n,
                         flip, terms, nterms, first, partials);
    else
      hipLaunchKernelGGL((k_pauli_far<float, false>), dim3(grid), dim3(256), 0, s, (const float2*)psi, nullptr, n,
                         flip, terms, nterms, first, partials);
  }
  return hipGetLastError();
}

hipError_t launch_pauli_set(bool dbl, const void* psi, void* lam, const PauliSet& set, const PauliGroupTile* groups,
                            const PauliTermTile* terms, double* partials, hipStream_t s) {
  const int m = set.L + set.H;
  if (set.n < 1 || set.n > kMaxQubits || set.L < 0 || set.H < 0 || set.H > kPauliMaxH || m > 12 || m > set.n)
    return hipErrorInvalidValue;
  for (int i = 0; i < set.H; ++i)
    if (set.hbits[i] < set.L || set.hbits[i] >= set.n || (i && set.hbits[i] <= set.hbits[i - 1]))
      return hipErrorInvalidValue;
  const int64_t nt = 1ll << (set.n - m);
  const int grid = (int)(nt < kGridMax ? nt : kGridMax);
  const size_t lds = (size_t(1) << m) * (dbl ? 16 : 8);
  if (dbl) {
    hipError_t e = set_lds_fn(lam ? (void*)k_pauli_tile<double, true> : (void*)k_pauli_tile<double, false>, lds);
    if (e != hipSuccess) return e;
    if (lam)
      hipLaunchKernelGGL((k_pauli_tile<double, true>), dim3(grid), dim3(256), lds, s, (const double2*)psi,
                         (double2*)lam, set, groups, terms, partials);
    else
      hipLaunchKernelGGL((k_pauli_tile<double, false>), dim3(grid), dim3(256), lds, s, (const double2*)psi, nullptr,
                         set, groups, terms, partials);
  } else {
    hipError_t e = set_lds_fn(lam ? (void*)k_pauli_tile<float, true> : (void*)k_pauli_tile<float, false>, lds);
    if (e != hipSuccess) return e;
    if (lam)
      hipLaunchKernelGGL((k_pauli_tile<float, true>), dim3(grid), dim3(256), lds, s, (const float2*)psi,
                         (float2*)lam, set, groups, terms, partials);
    else
      hipLaunchKernelGGL((k_pauli_tile<float, false>), dim3(grid), dim3(256), lds, s, (const float2*)psi, nullptr,
                         set, groups, terms, partials);
  }
  return hipGetLastError();
}

hipError_t launch_final_sum(const double* partials, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, partials, count, out);
  return hipGetLastError();
}

hipError_t launch_slot_sums(const double* partials, int nslots, int nblocks, int stride, double* out,
                            hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_sums, dim3(nslots), dim3(256), 0, s, partials, nblocks, stride, out);
  return hipGetLastError();
}

int sample_nblocks(int n) {
  const int64_t N = 1ll << n;
  return (int)((N + kSampBlock - 1) / kSampBlock);
}

int sample_nchunks(int n) { return (sample_nblocks(n) + kSampChunk - 1) / kSampChunk; }

hipError_t launch_sample(bool dbl, const void* psi, int n, double* blocksums, double* prefix, double* chunks,
                         int64_t shots, uint64_t seed, const double* uniforms, const int* pos, int m, int64_t* out,
                         hipStream_t s) {
  const int64_t N = 1ll << n;
  const int64_t nb = sample_nblocks(n);
  const int64_t nc = sample_nchunks(n);
  const int g1 = (int)((nb + 3) / 4);
  if (dbl) hipLaunchKernelGGL((k_samp_blocks<double>), dim3(g1), dim3(256), 0, s, (const double2*)psi, N, nb, blocksums);
  else hipLaunchKernelGGL((k_samp_blocks<float>), dim3(g1), dim3(256), 0, s, (const float2*)psi, N, nb, blocksums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // prefix of the block sums: chunk totals, their exclusive prefix (one
  // workgroup: at most 2^15 chunks), then each chunk's own prefix
  double* ctot = chunks;
  double* coff = chunks + nc;
  hipLaunchKernelGGL(k_samp_chunks, dim3((unsigned)nc), dim3(kThreads), 0, s, blocksums, nb, ctot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_samp_scan, dim3(1), dim3(1024), 0, s, ctot, nc, coff);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_samp_prefix, dim3((unsigned)nc), dim3(kThreads), 0, s, blocksums, nb, coff, nc, prefix);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (shots == 0) return hipSuccess;
  SampArgs sa;
  sa.m = m;
  for (int i = 0; i < 64; ++i) sa.pos[i] = i < m ? pos[i] : 0;
  const int64_t g3 = (shots + 3) / 4;
  if (dbl)
    hipLaunchKernelGGL((k_samp_shots<double>), dim3((unsigned)g3), dim3(256), 0, s, (const double2*)psi, N, nb,
                       prefix, shots, seed, uniforms, sa, out);
  else
    hipLaunchKernelGGL((k_samp_shots<float>), dim3((unsigned)g3), dim3(256), 0, s, (const float2*)psi, N, nb,
                       prefix, shots, seed, uniforms, sa, out);
  return hipGetLastError();
}

}  // namespace qs
