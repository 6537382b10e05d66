// Host-side construction of the per-pass twiddle tables.
//
// Pass k of the forward decimation-in-frequency transform multiplies output b
// of the butterfly at offset l by W_L^(l*b) = exp(-2 pi i l b / L), L = len(k).
// Tables are stored as T_k[(b-1)*strd(k) + l] so that lanes with consecutive l
// read consecutive entries.  Values are evaluated in float64 from the exact
// reduced integer angle (l*b mod L) and rounded once to float32; the paper does
// not discuss twiddles.
#pragma once

#include <cmath>
#include <vector>

#include "ols_fft.hpp"

namespace ols {

template <int N>
std::vector<float2> build_twiddles() {
  using GE = Geo<N>;
  std::vector<float2> t(GE::TW_TOTAL > 0 ? GE::TW_TOTAL : 1, make_float2(1.f, 0.f));
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < GE::P - 1; ++k) {
    const int L = GE::len(k), RK = GE::radix(k), S = GE::strd(k);
    for (int b = 1; b < RK; ++b) {
      for (int l = 0; l < S; ++l) {
        const long m = ((long)l * b) % L;
        const double ang = two_pi * (double)m / (double)L;
        t[GE::tw_offset(k) + (b - 1) * S + l] = make_float2((float)std::cos(ang), (float)(-std::sin(ang)));
      }
    }
  }
  return t;
}

}  // namespace ols
