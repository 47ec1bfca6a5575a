// mci_host_util.h -- FP64 host helpers used at plan time to build device tables.
#pragma once
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

namespace mci {

// e^{-2 pi i k / L}; the angle is reduced through the exact integer k mod L
inline std::complex<double> root_of_unity(int64_t k, int64_t L) {
  k %= L;
  if (k < 0) k += L;
  const double a = -2.0 * M_PI * ((double)k / (double)L);
  return {std::cos(a), std::sin(a)};
}

// Host FP64 Stockham FFT with sign S over radices of x.size() (each <= 8).
inline void host_fft(std::vector<std::complex<double>>& x, const std::vector<int>& radices, int S) {
  const int64_t L = (int64_t)x.size();
  std::vector<std::complex<double>> y(L);
  int64_t Ns = 1;
  for (int R : radices) {
    const int64_t nb = L / R;
    for (int64_t j = 0; j < nb; ++j) {
      const int64_t k = j % Ns;
      std::complex<double> v[8], o[8];
      for (int r = 0; r < R; ++r) {
        std::complex<double> w = root_of_unity(k * r * (L / (Ns * R)), L);
        if (S > 0) w = std::conj(w);
        v[r] = x[j + r * nb] * w;
      }
      for (int s = 0; s < R; ++s) {
        std::complex<double> acc = 0;
        for (int q = 0; q < R; ++q) {
          std::complex<double> w = root_of_unity((int64_t)((q * s) % R), R);
          if (S > 0) w = std::conj(w);
          acc += v[q] * w;
        }
        o[s] = acc;
      }
      const int64_t base = (j / Ns) * Ns * R + k;
      for (int r = 0; r < R; ++r) y[base + r * Ns] = o[r];
    }
    x.swap(y);
    Ns *= R;
  }
}

// Bluestein chirp c[k] = e^{sign i pi k^2 / len}, with k^2 reduced modulo 2 len exactly.
inline std::complex<double> chirp_value(int64_t k, int64_t len, int sign) {
  const int64_t q = (int64_t)(((__int128)k * k) % (2 * len));
  const double a = (double)sign * M_PI * ((double)q / (double)len);
  return {std::cos(a), std::sin(a)};
}

}  // namespace mci
