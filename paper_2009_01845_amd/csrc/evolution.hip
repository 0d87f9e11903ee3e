// Kernels of the non-Trotter time evolution (Sec. 2.6) and of the
// entanglement-entropy callback (Sec. 2.4.4).
//
//  * k_lincomb: out = sum_l c_l in_l over whole state vectors (the stages of
//    the Runge-Kutta integrators: y = psi + dt sum_l a_jl k_l and the final
//    combination), float64 arithmetic, stored in the state precision.
//  * k_dense_h_add: H += scale * P for the Pauli groups of an observable,
//    written into a dense 2^n x 2^n complex128 matrix (the "exp" solver
//    builds the full Hamiltonian matrix).
//  * k_zgemm: complex128 matrix product on FP64 matrix cores
//    (v_mfma_f64_16x16x4f64) with strided, optionally conjugated operands and
//    a split contraction: the Taylor/squaring steps of the evolution operator
//    exp(-i H dt), and the Gram matrix M M^dagger of a reshaped state (the
//    reduced density matrix of a bipartition).
//  * k_matvec: psi <- U psi for a dense complex128 U.
#include "devmath.h"
#include "kernels.h"

namespace qs {

namespace {

using dm::Z;

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename R>
__global__ __launch_bounds__(256) void k_lincomb(typename dm::CT<R>::C* __restrict__ out, int64_t N,
                                                 LinComb lc) {
  using C = typename dm::CT<R>::C;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < N; x += stride) {
    Z acc{0.0, 0.0};
#pragma unroll 1
    for (int l = 0; l < lc.nin; ++l) {
      const Z v = dm::wide(static_cast<const C*>(lc.in[l])[x]);
      acc.x += lc.cre[l] * v.x - lc.cim[l] * v.y;
      acc.y += lc.cre[l] * v.y + lc.cim[l] * v.x;
    }
    out[x] = dm::narrow<C>(acc);
  }
}

// H[(x ^ m_g) * D + x] += scale * f_g(x): column x of a Pauli group with flip
// mask m_g holds f_g(x) = sum_t c_t i^{ny_t} (-1)^{popcount(x & zy_t)} in row
// x ^ m_g.  Distinct x write distinct columns and distinct groups distinct
// rows, so the updates do not collide.
__global__ __launch_bounds__(256) void k_dense_h_add(double2* __restrict__ H, int n,
                                                     const uint64_t* __restrict__ flips,
                                                     const int32_t* __restrict__ goff,
                                                     const PauliTermDev* __restrict__ terms, int ngroups,
                                                     double scale) {
  const int64_t D = int64_t(1) << n;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
    for (int g = 0; g < ngroups; ++g) {
      double fr = 0.0, fi = 0.0;
      for (int t = goff[g]; t < goff[g + 1]; ++t) {
        const PauliTermDev T = terms[t];
        const double c = (__popcll((uint64_t)x & T.zy) & 1) ? -T.coeff : T.coeff;
        switch (T.ny4) {
          case 0: fr += c; break;
          case 1: fi += c; break;
          case 2: fr -= c; break;
          default: fi -= c; break;
        }
      }
      double2& h = H[(int64_t)((uint64_t)x ^ flips[g]) * D + x];
      h.x += scale * fr;
      h.y += scale * fi;
    }
  }
}

// C = alpha * op(A) op(B) (+ I), M x N, contraction length K split into
// chunks of kchunk (blockIdx.y = chunk; each chunk writes its own M x N slab
// of `out`, slab stride M*N, so a split product is summed afterwards in a
// fixed order).  op(A)(i, j) = a[i*ars + j*acs] (conjugated if conja), and
// op(B)(j, k) = b[j*brs + k*bcs] likewise.  A workgroup computes a 64 x 64
// block of C with four waves of 32 x 32; each wave holds 2 x 2 blocks of
// 16 x 16, real and imaginary accumulators apart, and a complex product is
// four real MFMAs: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
template <typename R>
__global__ __launch_bounds__(256) void k_zgemm(const typename dm::CT<R>::C* __restrict__ a, int64_t ars,
                                               int64_t acs, int conja, const typename dm::CT<R>::C* __restrict__ b,
                                               int64_t brs, int64_t bcs, int conjb, int M, int N, int64_t K,
                                               int64_t kchunk, double2* __restrict__ out, double alpha_re,
                                               double alpha_im, int add_identity) {
  constexpr int TM = 64, TK = 16, PADA = TK + 1;
  __shared__ double2 As[TM][PADA];
  __shared__ double2 Bs[TK][TM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntn = (N + TM - 1) / TM;
  const int i0 = (blockIdx.x / ntn) * TM, k0 = (blockIdx.x % ntn) * TM;
  const int64_t jbeg = int64_t(blockIdx.y) * kchunk;
  const int64_t jend = jbeg + kchunk < K ? jbeg + kchunk : K;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 cr[2][2], ci[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      cr[p][q] = f64x4{0, 0, 0, 0};
      ci[p][q] = f64x4{0, 0, 0, 0};
    }
  // load maps: consecutive threads walk the unit-stride index of each operand
  const bool a_rowmajor = acs == 1;
  const bool b_rowmajor = bcs == 1;
  for (int64_t j0 = jbeg; j0 < jend; j0 += TK) {
#pragma unroll
    for (int r = 0; r < (TM * TK) / kThreads; ++r) {
      const int e = r * kThreads + tid;
      const int ii = a_rowmajor ? e / TK : e % TM, jj = a_rowmajor ? e % TK : e / TM;
      const int64_t gi = i0 + ii, gj = j0 + jj;
      Z v{0.0, 0.0};
      if (gi < M && gj < jend) {
        v = dm::wide(a[gi * ars + gj * acs]);
        if (conja) v.y = -v.y;
      }
      As[ii][jj] = double2{v.x, v.y};
    }
#pragma unroll
    for (int r = 0; r < (TM * TK) / kThreads; ++r) {
      const int e = r * kThreads + tid;
      const int jj = b_rowmajor ? e / TM : e % TK, kk = b_rowmajor ? e % TM : e / TK;
      const int64_t gj = j0 + jj, gk = k0 + kk;
      Z v{0.0, 0.0};
      if (gk < N && gj < jend) {
        v = dm::wide(b[gj * brs + gk * bcs]);
        if (conjb) v.y = -v.y;
      }
      Bs[jj][kk] = double2{v.x, v.y};
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kj = 4 * ks + (lane >> 4);
      double2 af[2], bf[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) af[p] = As[wr + 16 * p + (lane & 15)][kj];
#pragma unroll
      for (int q = 0; q < 2; ++q) bf[q] = Bs[kj][wc + 16 * q + (lane & 15)];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          cr[p][q] = mma64(af[p].x, bf[q].x, cr[p][q]);
          cr[p][q] = mma64(-af[p].y, bf[q].y, cr[p][q]);
          ci[p][q] = mma64(af[p].x, bf[q].y, ci[p][q]);
          ci[p][q] = mma64(af[p].y, bf[q].x, ci[p][q]);
        }
    }
    __syncthreads();
  }
  double2* slab = out + int64_t(blockIdx.y) * M * N;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + wr + 16 * p + 4 * v + (lane >> 4);  // f64 MFMA output row of element v
        const int col = k0 + wc + 16 * q + (lane & 15);
        if (row < M && col < N) {
          const double xr = cr[p][q][v], xi = ci[p][q][v];
          double2 o{alpha_re * xr - alpha_im * xi, alpha_re * xi + alpha_im * xr};
          if (add_identity && row == col) o.x += 1.0;
          slab[int64_t(row) * N + col] = o;
        }
      }
}

// out[i] = sum_s part[s * count + i], s = 0..nsplit-1 in order
__global__ __launch_bounds__(256) void k_split_sum(const double2* __restrict__ part, int nsplit, int64_t count,
                                                   double2* __restrict__ out) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < count; i += stride) {
    double2 acc{0.0, 0.0};
    for (int s = 0; s < nsplit; ++s) {
      const double2 v = part[int64_t(s) * count + i];
      acc.x += v.x;
      acc.y += v.y;
    }
    out[i] = acc;
  }
}

// y = U x for a dense D x D complex128 U: one wave per row, lanes stride the
// row (coalesced reads of U), float64 accumulation, fixed-order wave sum.
template <typename R>
__global__ __launch_bounds__(256) void k_matvec(const double2* __restrict__ U, const typename dm::CT<R>::C* __restrict__ x,
                                                typename dm::CT<R>::C* __restrict__ y, int64_t D) {
  using C = typename dm::CT<R>::C;
  const int lane = threadIdx.x & 63;
  const int64_t row = int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
  if (row >= D) return;
  double sr = 0.0, si = 0.0;
  for (int64_t j = lane; j < D; j += 64) {
    const double2 u = U[row * D + j];
    const Z v = dm::wide(x[j]);
    sr += u.x * v.x - u.y * v.y;
    si += u.x * v.y + u.y * v.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (lane == 0) y[row] = dm::narrow<C>(Z{sr, si});
}

// P = I (D x D complex128)
__global__ __launch_bounds__(256) void k_identity(double2* __restrict__ P, int64_t D) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < D * D; i += stride)
    P[i] = double2{(i / D == i % D) ? 1.0 : 0.0, 0.0};
}

int grid_for(int64_t units, int64_t per_block) {
  int64_t g = (units + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > kGridMax) g = kGridMax;
  return (int)g;
}

}  // namespace

hipError_t launch_lincomb(bool dbl, void* out, int n, const LinComb& lc, hipStream_t s) {
  const int64_t N = int64_t(1) << n;
  const int grid = grid_for(N, int64_t(kThreads) * 4);
  if (dbl) hipLaunchKernelGGL((k_lincomb<double>), dim3(grid), dim3(kThreads), 0, s, (double2*)out, N, lc);
  else hipLaunchKernelGGL((k_lincomb<float>), dim3(grid), dim3(kThreads), 0, s, (float2*)out, N, lc);
  return hipGetLastError();
}

hipError_t launch_dense_h_add(double* H, int n, const uint64_t* flips, const int32_t* goff, const PauliTermDev* terms,
                              int ngroups, double scale, hipStream_t s) {
  const int64_t D = int64_t(1) << n;
  const int grid = grid_for(D, kThreads);
  hipLaunchKernelGGL(k_dense_h_add, dim3(grid), dim3(kThreads), 0, s, (double2*)H, n, flips, goff, terms, ngroups,
                     scale);
  return hipGetLastError();
}

hipError_t launch_zgemm(bool dbl, const void* a, int64_t ars, int64_t acs, int conja, const void* b, int64_t brs,
                        int64_t bcs, int conjb, int M, int N, int64_t K, int nsplit, double* out, double alpha_re,
                        double alpha_im, int add_identity, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0 || nsplit < 1) return hipErrorInvalidValue;
  int64_t kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 15) / 16 * 16;
  const int splits = (int)((K + kchunk - 1) / kchunk);
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (dbl)
    hipLaunchKernelGGL((k_zgemm<double>), dim3(tiles, splits), dim3(kThreads), 0, s, (const double2*)a, ars, acs,
                       conja, (const double2*)b, brs, bcs, conjb, M, N, K, kchunk, (double2*)out, alpha_re, alpha_im,
                       add_identity);
  else
    hipLaunchKernelGGL((k_zgemm<float>), dim3(tiles, splits), dim3(kThreads), 0, s, (const float2*)a, ars, acs,
                       conja, (const float2*)b, brs, bcs, conjb, M, N, K, kchunk, (double2*)out, alpha_re, alpha_im,
                       add_identity);
  return hipGetLastError();
}

int zgemm_splits(int64_t K, int nsplit) {
  int64_t kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 15) / 16 * 16;
  return (int)((K + kchunk - 1) / kchunk);
}

hipError_t launch_split_sum(const double* part, int nsplit, int64_t count, double* out, hipStream_t s) {
  const int grid = grid_for(count, kThreads);
  hipLaunchKernelGGL(k_split_sum, dim3(grid), dim3(kThreads), 0, s, (const double2*)part, nsplit, count,
                     (double2*)out);
  return hipGetLastError();
}

hipError_t launch_identity(double* P, int n, hipStream_t s) {
  const int64_t D = int64_t(1) << n;
  hipLaunchKernelGGL(k_identity, dim3(grid_for(D * D, kThreads * 4)), dim3(kThreads), 0, s, (double2*)P, D);
  return hipGetLastError();
}

hipError_t launch_matvec(bool dbl, const double* U, const void* x, void* y, int n, hipStream_t s) {
  const int64_t D = int64_t(1) << n;
  const int grid = (int)((D + 3) / 4);
  if (dbl)
    hipLaunchKernelGGL((k_matvec<double>), dim3(grid), dim3(kThreads), 0, s, (const double2*)U, (const double2*)x,
                       (double2*)y, D);
  else
    hipLaunchKernelGGL((k_matvec<float>), dim3(grid), dim3(kThreads), 0, s, (const double2*)U, (const float2*)x,
                       (float2*)y, D);
  return hipGetLastError();
}

}  // namespace qs
