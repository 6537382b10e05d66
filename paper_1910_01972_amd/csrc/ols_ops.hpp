// Per-lane steps of the fused overlap-and-save kernel (sec. 3.2, Alg. 2):
// segment load with zero fill, spectrum product, discard-and-store.  Shared by
// the device kernels and by the host emulator used in CPU tests.
#pragma once

#include "ols_fft.hpp"

namespace ols {

// Segment j covers signal samples start .. start + N - 1 with
// start = j*H - D (D >= M-1 samples of history, sec. 3.2); samples outside
// [0, N_s) read as zero.  Register reg of lane g receives the sample at
// position g + time_pos_const(reg) of the segment.
template <int N>
OLS_HD void load_segment(float2 (&x)[16], const float2* __restrict__ s, int64_t Ns, int64_t start, int g) {
  // valid positions p satisfy lo <= p < hi (clamped into [0, N])
  const int64_t lo64 = -start, hi64 = Ns - start;
  const int lo = lo64 <= 0 ? 0 : (lo64 >= N ? N : (int)lo64);
  const int hi = hi64 <= 0 ? 0 : (hi64 >= N ? N : (int)hi64);
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    x[reg] = (p >= lo && p < hi) ? s[start + p] : make_float2(0.f, 0.f);
  }
}

// Filter r zero padded to N (plan step, Fig. 1 / Alg. 2): register reg of
// lane g receives tap g + time_pos_const(reg) if it is < M.
template <int N>
OLS_HD void load_filter(float2 (&x)[16], const float2* __restrict__ h, int M, bool valid, int g) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    x[reg] = (valid && p < M) ? h[p] : make_float2(0.f, 0.f);
  }
}

// Spectra are stored in the order the forward transform leaves them in
// registers: F[r][reg][g] (coalesced for every reg).
template <int N>
OLS_HD void load_spectrum(float2 (&f)[16], const float2* __restrict__ F, int r, int g) {
  const float2* Fr = F + (int64_t)r * N;
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) f[reg] = Fr[reg * Geo<N>::G + g];
}

template <int N>
OLS_HD void store_spectrum(const float2 (&x)[16], float2* __restrict__ F, int r, int g, float scale) {
  float2* Fr = F + (int64_t)r * N;
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) Fr[reg * Geo<N>::G + g] = cscale(x[reg], scale);
}

// x = A * f (point-wise product in the permuted frequency order, sec. 3.4)
OLS_HD void spectrum_product(float2 (&x)[16], const float2 (&A)[16], const float2 (&f)[16]) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) x[reg] = cmul(A[reg], f[reg]);
}

// After the inverse transform register reg of lane g holds circular position
// p = g + time_pos_const(reg).  Positions D .. D+H-1 are unaliased
// (D >= M-1, sec. 3.2) and go to outputs out0 + p - D, out0 = j*H; outputs
// >= N_s are not written.  (Per-lane predicates: variants that made the
// full/empty decision per register in scalar code measured slower.)
template <int N>
OLS_HD void store_valid(const float2 (&x)[16], float2* __restrict__ yrow, int64_t Ns, int64_t out0, int D, int H,
                        int g) {
  const int64_t lim64 = Ns - out0 + D;  // p < lim  <=>  out0 + p - D < N_s
  const int lim_n = lim64 >= D + H ? D + H : (int)(lim64 < 0 ? 0 : lim64);
  float2* base = yrow + (out0 - D);
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    if (p >= D && p < lim_n) base[p] = x[reg];
  }
}


// ---------------------------------------------------------------------------
// Adjoint (gradient) helpers.  For the adjoint, segment j's window starts at
// j*H (no delay): the correlation with conj(h) uses future samples, so the
// aliased positions are at the end of the window and positions 0 .. H-1 are
// exact for H <= N - M + 1 (footnote to eq. 2).
// ---------------------------------------------------------------------------

// x[reg] = src[start + p] for p = g + time_pos_const(reg) < lim and
// start + p < N_s (start >= 0); zero elsewhere.
template <int N>
OLS_HD void load_window(float2 (&x)[16], const float2* __restrict__ src, int64_t Ns, int64_t start, int lim, int g) {
  const int64_t rem = Ns - start;
  const int hi = rem <= 0 ? 0 : (rem >= lim ? lim : (int)rem);
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    x[reg] = p < hi ? src[start + p] : make_float2(0.f, 0.f);
  }
}

// A = conj(x) * scale
OLS_HD void conj_scaled(float2 (&A)[16], const float2 (&x)[16], float scale) {
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = make_float2(x[i].x * scale, -x[i].y * scale);
}

// acc += G * conj(F)
OLS_HD void acc_conj_product(float2 (&acc)[16], const float2 (&G)[16], const float2 (&F)[16]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = cfma<true>(G[i], F[i], acc[i]);
}

// Lags 0 .. M-1 of a time-domain result: part[p] += x[reg] for p < M.  Every
// lag is always owned by the same lane, so the read-modify-write needs no
// synchronisation.
template <int N>
OLS_HD void add_lags(float2* __restrict__ part, const float2 (&x)[16], int M, int g) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    if (p < M) part[p] = cadd(part[p], x[reg]);
  }
}

template <int N>
OLS_HD void zero_lags(float2* __restrict__ part, int M, int g) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    if (p < M) part[p] = make_float2(0.f, 0.f);
  }
}

// Filters per work unit of the forward kernels: two interleaved transforms when
// registers allow it (N <= 4096) and the filter count wastes little on a
// padded last group; the batched kernel allows two only up to N = 2048.
constexpr int BATCH_NF2_MAX_N = 2048;
OLS_HD int choose_nf(int N, int K) { return (N <= 4096 && (K % 2 == 0 || K >= 9)) ? 2 : 1; }
OLS_HD int choose_nf_batched(int N, int K) { return N <= BATCH_NF2_MAX_N ? choose_nf(N, K) : 1; }

// Partition arithmetic shared by the persistent kernels: workgroup b of P
// owns units [first_unit(b), first_unit(b+1)); owner(u) inverts it.
OLS_HD int64_t first_unit(int64_t U, int64_t P, int64_t b) { return U * b / P; }
OLS_HD int64_t owner_of_unit(int64_t U, int64_t P, int64_t u) { return ((u + 1) * P + U - 1) / U - 1; }

}  // namespace ols
