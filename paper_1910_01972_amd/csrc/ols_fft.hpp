// Register/LDS FFT building blocks for the fused overlap-and-save kernel.
//
// The method (sec. 3.4, Alg. 2): every segment is forward transformed once,
// the spectrum is kept on chip and reused for all filters, and for every filter
// the point-wise product is inverse transformed and the aliased samples are
// dropped.  As in the paper's C2C variant (sec. 3.4), the forward transform is
// a Cooley-Tukey decimation-in-frequency FFT whose output stays in digit-
// reversed order; the filter spectra are produced by the very same transform so
// they share that order, and the inverse is the exact mirror (decimation in
// time) that takes the permuted spectrum back to natural order.  No reordering
// pass is ever executed.
//
// gfx950 mapping (our design, not the paper's):
//   * every lane holds R = 16 complex samples in VGPRs; an N-point FFT is
//     spread over G = N/16 lanes;
//   * passes are radix r0 = N / 16^(P-1) first, then radix 16; each pass is
//     done entirely in registers;
//   * between passes the data is exchanged through LDS, with an additive
//     padding per exchange that makes every ds_write_b64 / ds_read_b64 free of
//     bank conflicts (checked for 32 and 64 banks by the host emulator test);
//     the padding is linear in the position bits, so every LDS address is a
//     per-lane base plus a compile-time immediate;
//   * twiddles between passes come from per-pass tables T_k[b][l] computed in
//     float64 on the host and rounded once to float32.
//
// This header is included by the device kernels and by the host emulator that
// runs the same per-lane code on the CPU for tests.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define OLS_HD __host__ __device__ __forceinline__

namespace ols {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

// ---------------------------------------------------------------------------
// Compile-time geometry of one N-point transform.
// ---------------------------------------------------------------------------
template <int N_>
struct Geo {
  static constexpr int N = N_;
  static constexpr int R = 16;                       // complex samples per lane
  static constexpr int G = N / R;                    // lanes per transform
  static constexpr int LOG2N = ilog2(N);
  static constexpr int P = (LOG2N + 3) / 4;          // number of passes
  static constexpr int R0 = N >> (4 * (P - 1));      // radix of the first pass
  static constexpr int WG = G >= 256 ? G : 256;      // threads per workgroup
  static constexpr int SEGS = WG / G;                // transforms per workgroup

  static constexpr int radix(int k) { return k == 0 ? R0 : 16; }
  // length of the sub-transforms that pass k works on
  static constexpr int len(int k) { return k == 0 ? N : (N / R0) >> (4 * (k - 1)); }
  // distance between the inputs of one butterfly of pass k
  static constexpr int strd(int k) { return len(k) / radix(k); }
  // butterflies per lane in pass k
  static constexpr int slots(int k) { return R / radix(k); }
  // twiddles of pass k (applied after its butterflies in the forward direction)
  static constexpr int tw_count(int k) { return k >= P - 1 ? 0 : (radix(k) - 1) * strd(k); }
  static constexpr int tw_offset(int k) { return k <= 0 ? 0 : tw_offset(k - 1) + tw_count(k - 1); }
  static constexpr int TW_TOTAL = tw_offset(P - 1);
  // twiddles one lane keeps in registers
  static constexpr int lane_tw(int k) { return k >= P - 1 ? 0 : slots(k) * (radix(k) - 1); }
  static constexpr int lane_tw_offset(int k) { return k <= 0 ? 0 : lane_tw_offset(k - 1) + lane_tw(k - 1); }
  static constexpr int TWR = lane_tw_offset(P - 1) > 0 ? lane_tw_offset(P - 1) : 1;

  // LDS padding of exchange e (between pass e and e+1), chosen per stride of
  // the destination pass; linear in the bits of the position.
  static constexpr int pad(int e, int q) {
    return strd(e + 1) == 1 ? q + (q >> 4)
         : strd(e + 1) == 16 ? q + (q >> 5) + 2 * (q >> 6)
         : strd(e + 1) == 256 ? q + (q >> 10)
         : q;
  }
  static constexpr int lds_size_e(int e) { return pad(e, SEGS * N - 1) + 1; }
  static constexpr int lds_max(int e) {
    return e < 0 ? 1 : (lds_size_e(e) > lds_max(e - 1) ? lds_size_e(e) : lds_max(e - 1));
  }
  static constexpr int LDS = lds_max(P - 2);  // float2 elements

  // Position (within one transform) of element a of butterfly slot j of lane g
  // in pass k: pos = beta*len + l + strd*a with w = g + G*j, beta = w / strd,
  // l = w % strd.  Split into a lane part and a constant part with disjoint bits.
  static OLS_HD int lane_pos(int k, int g) {
    if (k == 0) return g;
    const int S = strd(k);
    return (g / S) * len(k) + (g % S);
  }
  static constexpr int const_pos(int k, int j, int a) {
    return k == 0 ? G * j + strd(0) * a : strd(k) * a;
  }
  // offset l of the butterfly (j) of lane g in pass k: selects its twiddles
  static OLS_HD int tw_index(int k, int g, int j) {
    return k == 0 ? g + G * j : (g % strd(k));
  }

  static_assert(N >= 256 && N <= 8192 && (N & (N - 1)) == 0, "N must be a power of two in [256, 8192]");
  static_assert(P >= 2, "at least two passes");
};

// ---------------------------------------------------------------------------
// Complex helpers (float2 = {re, im}).
// ---------------------------------------------------------------------------
OLS_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
OLS_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
OLS_HD float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
OLS_HD float2 cmulc(float2 a, float2 b) { return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
OLS_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
OLS_HD float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// multiply by W16^e = exp(-2 pi i e / 16) (forward) or its conjugate (inverse),
// e a compile-time constant in [0, 16)
template <int E, bool INV>
OLS_HD float2 mul_w16(float2 v) {
  constexpr float C1 = 0.92387953251128674f;   // cos(pi/8)
  constexpr float S1 = 0.38268343236508978f;   // sin(pi/8)
  constexpr float H = 0.70710678118654752f;    // sqrt(1/2)
  constexpr int e = E & 15;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (e == 4) {
    return mul_mi<INV>(v);
  } else if constexpr (e == 8) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (e == 12) {
    return mul_mi<!INV>(v);
  } else if constexpr (e == 2) {  // (1 - i)/sqrt2
    return INV ? make_float2((v.x - v.y) * H, (v.x + v.y) * H) : make_float2((v.x + v.y) * H, (v.y - v.x) * H);
  } else if constexpr (e == 6) {  // (-1 - i)/sqrt2
    return INV ? make_float2((-v.x - v.y) * H, (v.x - v.y) * H) : make_float2((v.y - v.x) * H, (-v.x - v.y) * H);
  } else {
    constexpr float tc[16] = {1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1, 0.f, S1, H, C1};
    constexpr float ts[16] = {0.f, S1, H, C1, 1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1};
    // W16^e = (cos, -sin)
    const float2 w = make_float2(tc[e], -ts[e]);
    return INV ? cmulc(v, w) : cmul(v, w);
  }
}

// ---------------------------------------------------------------------------
// In-register DFTs of radix 2, 4, 8, 16 on v[0 .. RADIX-1] (stride ST in the
// array), natural order in and out.  Forward kernel exp(-2 pi i ab / RADIX);
// INV uses the conjugate kernel (no 1/RADIX factor).
// ---------------------------------------------------------------------------
template <bool INV, int ST = 1>
OLS_HD void dft2(float2* v) {
  const float2 a = v[0], b = v[ST];
  v[0] = cadd(a, b);
  v[ST] = csub(a, b);
}

template <bool INV>
OLS_HD void dft4v(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  const float2 t2 = cadd(x1, x3), t3 = mul_mi<INV>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

template <bool INV, int ST = 1>
OLS_HD void dft4(float2* v) { dft4v<INV>(v[0], v[ST], v[2 * ST], v[3 * ST]); }

template <bool INV, int ST = 1>
OLS_HD void dft8(float2* v) {
  // a = a1 + 2 a2, b = b2 + 4 b1
  float2 e0 = v[0], e1 = v[2 * ST], e2 = v[4 * ST], e3 = v[6 * ST];
  float2 o0 = v[ST], o1 = v[3 * ST], o2 = v[5 * ST], o3 = v[7 * ST];
  dft4v<INV>(e0, e1, e2, e3);
  dft4v<INV>(o0, o1, o2, o3);
  o1 = mul_w16<2, INV>(o1);
  o2 = mul_w16<4, INV>(o2);
  o3 = mul_w16<6, INV>(o3);
  v[0] = cadd(e0, o0); v[4 * ST] = csub(e0, o0);
  v[ST] = cadd(e1, o1); v[5 * ST] = csub(e1, o1);
  v[2 * ST] = cadd(e2, o2); v[6 * ST] = csub(e2, o2);
  v[3 * ST] = cadd(e3, o3); v[7 * ST] = csub(e3, o3);
}

template <bool INV, int ST = 1>
OLS_HD void dft16(float2* v) {
  // a = a1 + 4 a2, b = b2 + 4 b1:
  //   y[a1][b2] = DFT4_{a2} v[a1 + 4 a2];  y[a1][b2] *= W16^(a1 b2);
  //   X[b2 + 4 b1] = DFT4_{a1} y[a1][b2]
  float2 y[4][4];
#pragma unroll
  for (int a1 = 0; a1 < 4; ++a1) {
    y[a1][0] = v[(a1) * ST];
    y[a1][1] = v[(a1 + 4) * ST];
    y[a1][2] = v[(a1 + 8) * ST];
    y[a1][3] = v[(a1 + 12) * ST];
    dft4v<INV>(y[a1][0], y[a1][1], y[a1][2], y[a1][3]);
  }
  y[1][1] = mul_w16<1, INV>(y[1][1]);
  y[1][2] = mul_w16<2, INV>(y[1][2]);
  y[1][3] = mul_w16<3, INV>(y[1][3]);
  y[2][1] = mul_w16<2, INV>(y[2][1]);
  y[2][2] = mul_w16<4, INV>(y[2][2]);
  y[2][3] = mul_w16<6, INV>(y[2][3]);
  y[3][1] = mul_w16<3, INV>(y[3][1]);
  y[3][2] = mul_w16<6, INV>(y[3][2]);
  y[3][3] = mul_w16<9, INV>(y[3][3]);
#pragma unroll
  for (int b2 = 0; b2 < 4; ++b2) {
    dft4v<INV>(y[0][b2], y[1][b2], y[2][b2], y[3][b2]);
    v[(b2) * ST] = y[0][b2];
    v[(b2 + 4) * ST] = y[1][b2];
    v[(b2 + 8) * ST] = y[2][b2];
    v[(b2 + 12) * ST] = y[3][b2];
  }
}

template <int RADIX, bool INV>
OLS_HD void dft(float2* v) {
  if constexpr (RADIX == 2) dft2<INV>(v);
  else if constexpr (RADIX == 4) dft4<INV>(v);
  else if constexpr (RADIX == 8) dft8<INV>(v);
  else if constexpr (RADIX == 16) dft16<INV>(v);
  else static_assert(RADIX == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// One pass of the transform on one lane's 16 registers.
// Register j*radix + a holds element a of butterfly slot j.
// Forward: butterflies, then twiddles W_len^(l*b) on output b (b >= 1).
// Inverse: conjugate twiddles first, then inverse butterflies.
// tw points at this lane's twiddles of this pass: [slot][b-1].
// ---------------------------------------------------------------------------
template <int N, int K, bool INV>
OLS_HD void run_pass(float2 (&x)[16], const float2* tw) {
  using GE = Geo<N>;
  constexpr int RK = GE::radix(K);
  constexpr int SL = GE::slots(K);
  constexpr bool HAS_TW = K < GE::P - 1;
#pragma unroll
  for (int j = 0; j < SL; ++j) {
    if constexpr (INV && HAS_TW) {
#pragma unroll
      for (int b = 1; b < RK; ++b) x[j * RK + b] = cmulc(x[j * RK + b], tw[j * (RK - 1) + b - 1]);
    }
    dft<RK, INV>(&x[j * RK]);
    if constexpr (!INV && HAS_TW) {
#pragma unroll
      for (int b = 1; b < RK; ++b) x[j * RK + b] = cmul(x[j * RK + b], tw[j * (RK - 1) + b - 1]);
    }
  }
}

// Loads the twiddles lane g needs in every pass (registers for the whole kernel).
template <int N>
OLS_HD void load_lane_twiddles(float2 (&tw)[Geo<N>::TWR], const float2* table, int g) {
  using GE = Geo<N>;
#pragma unroll
  for (int k = 0; k < GE::P - 1; ++k) {
    const int RK = GE::radix(k), S = GE::strd(k);
#pragma unroll
    for (int j = 0; j < GE::slots(k); ++j) {
      const int l = GE::tw_index(k, g, j);
#pragma unroll
      for (int b = 1; b < RK; ++b)
        tw[GE::lane_tw_offset(k) + j * (RK - 1) + b - 1] = table[GE::tw_offset(k) + (b - 1) * S + l];
    }
  }
}

// LDS address of element a of slot j in pass K's pattern, for exchange E,
// of transform grp (within the workgroup) on lane g.
template <int N, int E, int K>
OLS_HD int lds_base(int grp, int g) {
  return Geo<N>::pad(E, grp * N + Geo<N>::lane_pos(K, g));
}
template <int N, int E, int K>
constexpr int lds_off(int j, int a) {
  return Geo<N>::pad(E, Geo<N>::const_pos(K, j, a));
}

// Write the registers of lane g (pass K pattern) into LDS for exchange E.
template <int N, int E, int K>
OLS_HD void lds_store(float2* lds, const float2 (&x)[16], int grp, int g) {
  using GE = Geo<N>;
  constexpr int RK = GE::radix(K);
  const int base = lds_base<N, E, K>(grp, g);
#pragma unroll
  for (int j = 0; j < GE::slots(K); ++j)
#pragma unroll
    for (int a = 0; a < RK; ++a) lds[base + lds_off<N, E, K>(j, a)] = x[j * RK + a];
}

template <int N, int E, int K>
OLS_HD void lds_load(const float2* lds, float2 (&x)[16], int grp, int g) {
  using GE = Geo<N>;
  constexpr int RK = GE::radix(K);
  const int base = lds_base<N, E, K>(grp, g);
#pragma unroll
  for (int j = 0; j < GE::slots(K); ++j)
#pragma unroll
    for (int a = 0; a < RK; ++a) x[j * RK + a] = lds[base + lds_off<N, E, K>(j, a)];
}

// Time-domain position held by register reg = j*r0 + a after the last inverse
// pass (equivalently, before the first forward pass): g + G*(j + slots0*a).
template <int N>
constexpr int time_pos_const(int reg) {
  using GE = Geo<N>;
  return GE::G * (reg / GE::R0 + GE::slots(0) * (reg % GE::R0));
}

// Frequency index held by register b of lane g after the last forward pass
// (digit-reversed order of the decimation-in-frequency recursion).
template <int N>
OLS_HD int spectrum_index(int g, int b) {
  using GE = Geo<N>;
  int q = 16 * g + b;  // position after the last pass (stride 1, radix 16)
  int k = 0, mult = 1;
#pragma unroll
  for (int p = 0; p < GE::P; ++p) {
    const int L1 = GE::len(p) / GE::radix(p);  // length of the sub-transforms after pass p
    const int digit = q / L1;
    q -= digit * L1;
    k += digit * mult;
    mult *= GE::radix(p);
  }
  return k;
}

}  // namespace ols
