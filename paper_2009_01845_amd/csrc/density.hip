// Density matrices on gfx950 (Sec. 2.4.3: circuits with noise channels act on
// density matrices instead of state vectors).
//
// An n-qubit density matrix rho is stored as a 2n-qubit state vector,
// rho[r][c] at flat index r * 2^n + c: the row index occupies the n most
// significant bits (qubits 0..n-1 of the 2n-qubit register), the column
// index the n least significant ones (qubits n..2n-1).  A gate U then acts as
// U on the row qubits and conj(U) on the column qubits, and a channel with
// Kraus operators K_i as the superoperator sum_i K_i (x) conj(K_i) on both,
// so the tiled state-vector passes evolve rho unchanged.  The kernels here
// cover what a state vector does not have: the outer product |psi><psi| and
// the traces Tr(rho) and Tr(P rho).
#include "devmath.h"
#include "kernels.h"

namespace qs {

namespace {

using dm::Z;

// rho[r 2^n + c] = psi[r] conj(psi[c]): each thread writes consecutive
// columns of one row, so the row amplitude is loaded once per thread and the
// stores are coalesced.
template <typename R>
__global__ __launch_bounds__(256) void k_outer(typename dm::CT<R>::C* __restrict__ rho,
                                               const typename dm::CT<R>::C* __restrict__ psi, int n) {
  using C = typename dm::CT<R>::C;
  const int64_t D = int64_t(1) << n;
  const int64_t total = D * D;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
    const Z a = dm::wide(psi[i >> n]);
    const Z b = dm::wide(psi[i & (D - 1)]);
    rho[i] = dm::narrow<C>(dm::zmul(a, dm::zconj(b)));
  }
}

// One float64 partial per workgroup of Re sum_x sum_g f_g(x) rho[x][x ^ m_g]
// (Tr(P rho) for P = sum of the groups' Pauli terms: P|x> = f(x)|x ^ m>, so
// Tr(P rho) = sum_x f(x) <x|rho|x ^ m>).  f_g(x) = sum_t c_t i^{ny_t}
// (-1)^{popcount(x & zy_t)}.  ngroups = 0 sums the diagonal: Re Tr(rho).
// Rows are split into contiguous ranges, one per workgroup, so the result
// does not depend on timing.
template <typename R>
__global__ __launch_bounds__(256) void k_dens_pauli(const typename dm::CT<R>::C* __restrict__ rho, int n,
                                                    const uint64_t* __restrict__ flips,
                                                    const int32_t* __restrict__ goff,
                                                    const PauliTermDev* __restrict__ terms, int ngroups,
                                                    double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int64_t D = int64_t(1) << n;
  const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t lo = int64_t(blockIdx.x) * chunk, hi = lo + chunk < D ? lo + chunk : D;
  double acc = 0.0;
  for (int64_t x = lo + threadIdx.x; x < hi; x += kThreads) {
    if (ngroups == 0) {
      acc += (double)rho[(x << n) | x].x;
      continue;
    }
    for (int g = 0; g < ngroups; ++g) {
      const Z v = dm::wide(rho[(x << n) | (x ^ (int64_t)flips[g])]);
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
      acc += fr * v.x - fi * v.y;
    }
  }
  const double r = dm::wg_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

int dens_grid(int64_t units, int64_t per_block) {
  int64_t g = (units + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > kGridMax) g = kGridMax;
  return (int)g;
}

}  // namespace

hipError_t launch_outer(bool dbl, void* rho, const void* psi, int n, hipStream_t s) {
  const int64_t total = int64_t(1) << (2 * n);
  const int grid = dens_grid(total, int64_t(kThreads) * 16);
  if (dbl)
    hipLaunchKernelGGL((k_outer<double>), dim3(grid), dim3(kThreads), 0, s, (double2*)rho, (const double2*)psi, n);
  else
    hipLaunchKernelGGL((k_outer<float>), dim3(grid), dim3(kThreads), 0, s, (float2*)rho, (const float2*)psi, n);
  return hipGetLastError();
}

hipError_t launch_dens_pauli(bool dbl, const void* rho, int n, const uint64_t* flips, const int32_t* goff,
                             const PauliTermDev* terms, int ngroups, double* partials, double* out,
                             hipStream_t s) {
  const int64_t D = int64_t(1) << n;
  const int grid = dens_grid(D, kThreads * 4);
  if (dbl)
    hipLaunchKernelGGL((k_dens_pauli<double>), dim3(grid), dim3(kThreads), 0, s, (const double2*)rho, n, flips,
                       goff, terms, ngroups, partials);
  else
    hipLaunchKernelGGL((k_dens_pauli<float>), dim3(grid), dim3(kThreads), 0, s, (const float2*)rho, n, flips,
                       goff, terms, ngroups, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_final_sum(partials, grid, out, s);
}

}  // namespace qs
