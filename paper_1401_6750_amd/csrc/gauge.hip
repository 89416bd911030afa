// Synthetic gauge field on the host: U = exp(i eps H) per link, the ensemble
// the library is benchmarked on in place of the paper's 32^3 x 64 twisted-mass
// configurations (Section 2.1.1), which are not available.
//
//   H = sum_{a=1..8} h_a lambda_a / 2   (lambda_a the Gell-Mann matrices),
//   h_a ~ N(0, 1) by Box-Muller from a SplitMix64 counter stream
//   (Steele, Lea & Flood 2014): link l = 4 site + mu (site lexicographic,
//   x fastest) draws outputs 8 l .. 8 l + 7 of the stream `seed`; output i is
//   mix(seed + (i + 1) 0x9E3779B97F4A7C15), turned into a double in (0, 1) from
//   its top 53 bits; pairs (u_{2k}, u_{2k+1}) give
//   h_{2k} = sqrt(-2 ln u_{2k}) cos(2 pi u_{2k+1}), h_{2k+1} = ... sin(...).
//
// exp(i eps H) is taken by scaling and squaring of its Taylor series: the
// argument is halved until its Frobenius norm is below 1/4, the series summed
// to order 20 (truncation far below double rounding) and squared back.  Any
// accurate evaluation gives the same unitary matrix up to rounding.
#include <cmath>
#include <complex>
#include <cstdint>
#include <thread>
#include <vector>

#include "runtime.h"

namespace dl {

namespace {

using cd = std::complex<double>;

inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline double uniform_open(uint64_t w) { return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

void mat_mul(const cd (&a)[9], const cd (&b)[9], cd (&c)[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// exp(A) for a 3x3 complex matrix of modest norm
void mat_exp(const cd (&a_in)[9], cd (&out)[9]) {
  cd a[9];
  double nrm = 0.0;
  for (int k = 0; k < 9; ++k) {
    a[k] = a_in[k];
    nrm += std::norm(a[k]);
  }
  nrm = std::sqrt(nrm);
  int sq = 0;
  while (nrm > 0.25) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = std::ldexp(1.0, -sq);
  for (cd& v : a) v *= sc;
  // Horner form of sum_k A^k / k!: T = I + A T / k for k = 20 .. 1
  cd t[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int k = 20; k >= 1; --k) {
    cd p[9];
    mat_mul(a, t, p);
    for (int e = 0; e < 9; ++e) t[e] = p[e] / (double)k + ((e % 4 == 0) ? 1.0 : 0.0);
  }
  for (int s = 0; s < sq; ++s) {
    cd p[9];
    mat_mul(t, t, p);
    for (int e = 0; e < 9; ++e) t[e] = p[e];
  }
  for (int e = 0; e < 9; ++e) out[e] = t[e];
}

// i eps H for the eight Gaussian coefficients, H = sum_a h_a lambda_a / 2
void generator(const double (&h)[8], double eps, cd (&a)[9]) {
  const double r3 = 1.0 / std::sqrt(3.0);
  cd H[9];
  H[0] = 0.5 * (h[2] + r3 * h[7]);
  H[4] = 0.5 * (-h[2] + r3 * h[7]);
  H[8] = 0.5 * (-2.0 * r3 * h[7]);
  H[1] = 0.5 * cd(h[0], -h[1]);   // lambda_1 (1 at (0,1)) and lambda_2 (-i at (0,1))
  H[3] = std::conj(H[1]);
  H[2] = 0.5 * cd(h[3], -h[4]);   // lambda_4, lambda_5
  H[6] = std::conj(H[2]);
  H[5] = 0.5 * cd(h[5], -h[6]);   // lambda_6, lambda_7
  H[7] = std::conj(H[5]);
  for (int k = 0; k < 9; ++k) a[k] = cd(0.0, eps) * H[k];
}

}  // namespace

void random_gauge_host(const int dims[4], uint64_t seed, double eps, double* links) {
  const long long nlink = 4ll * dims[0] * dims[1] * dims[2] * dims[3];
  auto work = [&](long long l0, long long l1) {
    for (long long l = l0; l < l1; ++l) {
      double h[8];
      for (int k = 0; k < 4; ++k) {
        const double u0 = uniform_open(splitmix64_at(seed, (uint64_t)(8 * l + 2 * k)));
        const double u1 = uniform_open(splitmix64_at(seed, (uint64_t)(8 * l + 2 * k + 1)));
        const double rad = std::sqrt(-2.0 * std::log(u0));
        const double ang = 2.0 * M_PI * u1;
        h[2 * k] = rad * std::cos(ang);
        h[2 * k + 1] = rad * std::sin(ang);
      }
      cd a[9], u[9];
      generator(h, eps, a);
      mat_exp(a, u);
      double* o = links + 18 * l;
      for (int e = 0; e < 9; ++e) {
        o[2 * e] = u[e].real();
        o[2 * e + 1] = u[e].imag();
      }
    }
  };
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if (nlink < 4096) nt = 1;
  std::vector<std::thread> th;
  const long long per = (nlink + nt - 1) / nt;
  for (unsigned k = 1; k < nt; ++k) {
    const long long a = k * per, b = std::min(nlink, a + per);
    if (a < b) th.emplace_back(work, a, b);
  }
  work(0, std::min(nlink, per));
  for (auto& t : th) t.join();
}

}  // namespace dl
