// Host linear algebra of the entanglement-entropy callback (linalg.cpp).
#pragma once
#include <complex>
#include <vector>

namespace qs {

// Eigenvalues (ascending) of an n x n Hermitian matrix given row-major.
std::vector<double> hermitian_eigenvalues(int n, std::vector<std::complex<double>> A);
// -sum l log l over the eigenvalues above 1e-15 (natural logarithm)
double entropy_of_eigenvalues(const std::vector<double>& ev);

}  // namespace qs
