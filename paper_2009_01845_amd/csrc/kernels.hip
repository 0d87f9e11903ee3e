// gfx950 kernels of the state-vector simulator.
//
// Layout: 2^n interleaved complex amplitudes (float2 or double2), qubit q at
// index bit n-1-q.  Every streaming kernel is bound by HBM bandwidth: it reads
// and writes each amplitude once per pass with 16-byte vector accesses, and
// the index arithmetic is 64-bit throughout (2^35 amplitudes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace qs {

namespace {

template <typename R> struct CT;
template <> struct CT<float> {
  using C = float2;
  using V = float4;  // 16-byte access = 2 amplitudes
  static constexpr int VW = 2;
};
template <> struct CT<double> {
  using C = double2;
  using V = double2;  // 16-byte access = 1 amplitude
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
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += red[i];
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
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
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
  for (int i = threadIdx.x; i < nq; i += blockDim.x) {
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
  for (int i = threadIdx.x; i < ng; i += blockDim.x) {
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
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
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
  for (int hc = tid; hc < (1 << H); hc += blockDim.x) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << g.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;

  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = tile_base((uint64_t)t, g);
    for (int e = tid * VW; e < M; e += blockDim.x * VW) {
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
          const double th = (TWO ? -1.0 : 1.0) * params[op.pidx];
          if (TWO && op.gslot >= 0) {
            const double v = block_sum(rot_grad_partial(t1, t2, M, op.b[0], op.cin, op.pauli), red);
            if (tid == 0) gpart[(int64_t)op.gslot * kGridMax + blockIdx.x] += v;
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
          for (int hc = tid; hc < (1 << H); hc += blockDim.x) {
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
          for (int e = tid * VW; e < M; e += blockDim.x * VW) {
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

    for (int e = tid * VW; e < M; e += blockDim.x * VW) {
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
struct PermArgs {
  int tau[kMaxQubits];
};

template <typename R>
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
  const int tid = threadIdx.x, L = g.L, H = g.H;
  for (int b = tid; b < g.n; b += blockDim.x) loc[b] = b < L ? b : -1;
  __syncthreads();
  if (tid < H) loc[g.hbits[tid]] = L + tid;
  for (int hc = tid; hc < (1 << H); hc += blockDim.x) {
    uint64_t off = 0;
    for (int i = 0; i < H; ++i)
      if ((hc >> i) & 1) off |= 1ull << g.hbits[i];
    hoff[hc] = off;
  }
  __syncthreads();
  for (int j = tid; j < M; j += blockDim.x) {
    uint32_t lj = 0;
    for (int i = 0; i < g.m; ++i)
      if ((j >> i) & 1) {
        const int gp = i < L ? i : g.hbits[i - L];
        lj |= 1u << loc[pa.tau[gp]];
      }
    ltau[j] = (uint16_t)lj;
  }
  __syncthreads();
  const uint32_t lomask = (1u << L) - 1u;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = tile_base((uint64_t)t, g);
    uint64_t pbase = 0;
    for (uint64_t r = base; r; r &= r - 1) pbase |= 1ull << pa.tau[__builtin_ctzll(r)];
    const int64_t tp = (int64_t)tile_index(pbase, g);
    if (tp < t) continue;  // the partner tile's workgroup moves this pair
    const bool self = tp == t;
    for (int e = tid; e < M; e += blockDim.x) {
      const uint64_t off = hoff[e >> L] | (uint64_t)(e & lomask);
      ta[e] = psi[base | off];
      if (!self) tb[e] = psi[pbase | off];
    }
    __syncthreads();
    for (int e = tid; e < M; e += blockDim.x) {
      const uint64_t off = hoff[e >> L] | (uint64_t)(e & lomask);
      psi[pbase | off] = ta[ltau[e]];
      if (!self) psi[base | off] = tb[ltau[e]];
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
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    psi[i] = mk<C>(re, 0.0);
}
__global__ void k_zero(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
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
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
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
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
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

template <typename R>
__global__ __launch_bounds__(256) void k_expect(const typename CT<R>::C* __restrict__ psi, int n, uint64_t flip,
                                                const PauliTermDev* __restrict__ terms, int nt,
                                                double* __restrict__ part) {
  __shared__ double red[8];
  const int64_t N = 1ll << n;
  const int64_t units = flip ? N >> 1 : N;
  const int hb = flip ? 63 - __builtin_clzll(flip) : 0;
  const int64_t chunk = (units + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < units ? lo + chunk : units;
  double acc = 0.0;
  for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
    const uint64_t x = flip ? insert_zero64((uint64_t)u, hb) : (uint64_t)u;
    double fr, fi;
    pauli_factor(x, terms, nt, fr, fi);
    const auto px = psi[x];
    if (!flip) {
      acc += ((double)px.x * px.x + (double)px.y * px.y) * fr;
    } else {
      const auto py = psi[x ^ flip];
      // conj(py) * px
      const double zr = (double)py.x * px.x + (double)py.y * px.y;
      const double zi = (double)py.x * px.y - (double)py.y * px.x;
      acc += 2.0 * (zr * fr - zi * fi);
    }
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename R>
__global__ __launch_bounds__(256) void k_apply_ham(const typename CT<R>::C* __restrict__ psi,
                                                   typename CT<R>::C* __restrict__ lam, int n,
                                                   const uint64_t* __restrict__ flips,
                                                   const int* __restrict__ goff, int ng,
                                                   const PauliTermDev* __restrict__ terms) {
  using C = typename CT<R>::C;
  const int64_t N = 1ll << n;
  for (int64_t y = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; y < N; y += (int64_t)gridDim.x * blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int gi = 0; gi < ng; ++gi) {
      const uint64_t x = (uint64_t)y ^ flips[gi];
      double fr, fi;
      pauli_factor(x, terms + goff[gi], goff[gi + 1] - goff[gi], fr, fi);
      const C v = psi[x];
      ar += fr * v.x - fi * v.y;
      ai += fr * v.y + fi * v.x;
    }
    lam[y] = mk<C>(ar, ai);
  }
}

__global__ __launch_bounds__(256) void k_final_sum(const double* __restrict__ part, int count, double* out) {
  __shared__ double red[8];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += part[i];
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = r;
}

__global__ __launch_bounds__(256) void k_slot_sums(const double* __restrict__ part, int nblocks, double* out) {
  __shared__ double red[8];
  double acc = 0.0;
  const double* p = part + (int64_t)blockIdx.x * kGridMax;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += p[i];
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// ----------------------------------------------------------------------------
// sampling: blocks of 1024 amplitudes = 64 lanes x 16 consecutive
// ----------------------------------------------------------------------------
constexpr int kSampBlock = 1024;
constexpr int kSampPerLane = 16;

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

template <typename R>
__global__ __launch_bounds__(256) void k_samp_blocks(const typename CT<R>::C* __restrict__ psi, int64_t N,
                                                     int64_t nb, double* __restrict__ S) {
  const int64_t blk = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (blk >= nb) return;
  const int lane = threadIdx.x & 63;
  const double incl = wave_incl_scan(lane_mass<R>(psi, N, blk, lane));
  if (lane == 63) S[blk] = incl;
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
  const int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
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
  const double incl = wave_incl_scan(lane_mass<R>(psi, N, b, lane));
  const double excl = __shfl_up(incl, 1, 64);
  const double before = P[b] + (lane == 0 ? 0.0 : excl);
  const unsigned long long hit = __ballot(P[b] + incl > target);
  int sel;
  if (hit) sel = __builtin_ctzll(hit);
  else sel = 63;  // rounding: the target sits past this block's own total
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

template <typename R> void* fn_tile(bool two) {
  return two ? (void*)k_tile<R, true> : (void*)k_tile<R, false>;
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
  const size_t lds = (size_t(1) << g.m) * esz * (two ? 2 : 1);
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
  {
    hipError_t e = set_lds(dbl ? (void*)k_perm<double> : (void*)k_perm<float>, lds);
    if (e != hipSuccess) return e;
  }
  if (dbl)
    hipLaunchKernelGGL((k_perm<double>), dim3(grid), dim3(kThreads), lds, s, (double2*)psi, g, pa, nt);
  else
    hipLaunchKernelGGL((k_perm<float>), dim3(grid), dim3(kThreads), lds, s, (float2*)psi, g, pa, nt);
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

hipError_t launch_expect_group(bool dbl, const void* psi, int n, uint64_t flip, const PauliTermDev* terms,
                               int nterms, double* partials, hipStream_t s) {
  const int64_t units = flip ? (1ll << (n - 1)) : (1ll << n);
  const int grid = reduce_grid(units);
  if (dbl)
    hipLaunchKernelGGL((k_expect<double>), dim3(grid), dim3(256), 0, s, (const double2*)psi, n, flip, terms,
                       nterms, partials);
  else
    hipLaunchKernelGGL((k_expect<float>), dim3(grid), dim3(256), 0, s, (const float2*)psi, n, flip, terms, nterms,
                       partials);
  return hipGetLastError();
}

hipError_t launch_apply_hamiltonian(bool dbl, const void* psi, void* lam, int n, const uint64_t* flips,
                                    const int* group_off, int ngroups, const PauliTermDev* terms,
                                    hipStream_t s) {
  const int64_t N = 1ll << n;
  const int grid = (int)std::min<int64_t>((N + 255) / 256, 8192);
  if (dbl)
    hipLaunchKernelGGL((k_apply_ham<double>), dim3(grid), dim3(256), 0, s, (const double2*)psi, (double2*)lam, n,
                       flips, group_off, ngroups, terms);
  else
    hipLaunchKernelGGL((k_apply_ham<float>), dim3(grid), dim3(256), 0, s, (const float2*)psi, (float2*)lam, n,
                       flips, group_off, ngroups, terms);
  return hipGetLastError();
}

hipError_t launch_final_sum(const double* partials, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, partials, count, out);
  return hipGetLastError();
}

hipError_t launch_slot_sums(const double* partials, int nslots, int nblocks, double* out, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_sums, dim3(nslots), dim3(256), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

int sample_nblocks(int n) {
  const int64_t N = 1ll << n;
  return (int)((N + kSampBlock - 1) / kSampBlock);
}

hipError_t launch_sample(bool dbl, const void* psi, int n, double* blocksums, double* prefix, int64_t shots,
                         uint64_t seed, const double* uniforms, const int* pos, int m, int64_t* out,
                         hipStream_t s) {
  const int64_t N = 1ll << n;
  const int64_t nb = sample_nblocks(n);
  const int g1 = (int)((nb + 3) / 4);
  if (dbl) hipLaunchKernelGGL((k_samp_blocks<double>), dim3(g1), dim3(256), 0, s, (const double2*)psi, N, nb, blocksums);
  else hipLaunchKernelGGL((k_samp_blocks<float>), dim3(g1), dim3(256), 0, s, (const float2*)psi, N, nb, blocksums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_samp_scan, dim3(1), dim3(1024), 0, s, blocksums, nb, prefix);
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
