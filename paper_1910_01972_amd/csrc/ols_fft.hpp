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

// Declares a value that is equal in every lane of the wave as uniform, so the
// compiler keeps it (and what is derived from it) in scalar registers.  Only
// call it on values that really are wave-uniform.
OLS_HD int64_t wave_uniform64(int64_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
#else
  return v;
#endif
}

// A pointer that is the same in every lane of the wave, kept in scalar
// registers: accesses become scalar base + per-lane 32-bit offset.
template <class T>
OLS_HD T* wave_uniform_ptr(T* p) {
  return (T*)(intptr_t)wave_uniform64((int64_t)(intptr_t)p);
}

// Pointers into device global memory.  In device code gptr<T> is a pointer in
// the global address space: loads and stores through it compile to global and
// buffer instructions even where the compiler cannot see that a pointer
// points to global memory (a pointer read from a table inside a function that
// is not inlined would otherwise give flat instructions, which also hold up
// every LDS wait).  In host code (the emulator) it is a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;
#endif
template <class T>
OLS_HD gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}
// reinterpret_cast that keeps the pointer's address space
template <class T, class U>
OLS_HD T* rebind_ptr(U* p) {
  return reinterpret_cast<T*>(p);
}
#if defined(__HIP_DEVICE_COMPILE__)
template <class T, class U>
OLS_HD gptr<T> rebind_ptr(__attribute__((address_space(1))) U* p) {
  return reinterpret_cast<gptr<T>>(p);
}
#endif

// Loads of complex values through plain or global pointers: as builtin
// vectors (a class type such as float2 cannot be copied out of another
// address space).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class P>
OLS_HD float2 load_c64(P p, int64_t i) {
  const f32x2 v = rebind_ptr<const f32x2>(p)[i];
  return make_float2(v.x, v.y);
}

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
// Inverse DFTs whose inputs are first multiplied by per-input factors c[i]
// (the conjugate twiddles of an inverse pass, or the filter spectrum in the
// point-wise product).  Each multiplication is fused into the first radix-2
// level with FMAs: t0 = p0 + v2*c2 (two FMAs per component) and
// t1 = 2*p0 - t0 (one FMA per component), instead of a separate complex
// multiply followed by an add and a subtract.  CJ selects v*conj(c).
// ---------------------------------------------------------------------------
template <bool CJ>
OLS_HD float2 cmul_k(float2 v, float2 c) { return CJ ? cmulc(v, c) : cmul(v, c); }

// p + v*c (CJ: p + v*conj(c))
template <bool CJ>
OLS_HD float2 cfma(float2 v, float2 c, float2 p) {
  return CJ ? make_float2(fmaf(v.x, c.x, fmaf(v.y, c.y, p.x)), fmaf(v.y, c.x, fmaf(-v.x, c.y, p.y)))
            : make_float2(fmaf(v.x, c.x, fmaf(-v.y, c.y, p.x)), fmaf(v.x, c.y, fmaf(v.y, c.x, p.y)));
}

// 2a - b
OLS_HD float2 twice_minus(float2 a, float2 b) { return make_float2(fmaf(2.f, a.x, -b.x), fmaf(2.f, a.y, -b.y)); }

// Inverse DFT4 of (x0*c0, x1*c1, x2*c2, x3*c3); ONE0: c0 = 1.
template <bool CJ, bool ONE0>
OLS_HD void idft4_premul(float2& x0, float2& x1, float2& x2, float2& x3, float2 c0, float2 c1, float2 c2, float2 c3) {
  const float2 p0 = ONE0 ? x0 : cmul_k<CJ>(x0, c0);
  const float2 t0 = cfma<CJ>(x2, c2, p0);
  const float2 t1 = twice_minus(p0, t0);
  const float2 p1 = cmul_k<CJ>(x1, c1);
  const float2 t2 = cfma<CJ>(x3, c3, p1);
  const float2 t3 = mul_mi<true>(twice_minus(p1, t2));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// conj(W16^e) as a float2 (inverse-direction constant)
template <int E>
OLS_HD float2 w16c() {
  constexpr float C1 = 0.92387953251128674f, S1 = 0.38268343236508978f, H = 0.70710678118654752f;
  constexpr float tc[16] = {1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1, 0.f, S1, H, C1};
  constexpr float ts[16] = {0.f, S1, H, C1, 1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1};
  return make_float2(tc[E & 15], ts[E & 15]);
}

// Second radix-4 level of the inverse DFT16 for column b2: inverse DFT4 over
// a1 of y[a1] * conj(W16^(a1*b2)), with the constant factors fused.
template <int B2>
OLS_HD void idft16_col(float2& y0, float2& y1, float2& y2, float2& y3) {
  if constexpr (B2 == 0) {
    dft4v<true>(y0, y1, y2, y3);
  } else if constexpr (B2 == 2) {
    // factors 1, conj W^2, conj W^4 = +i, conj W^6
    const float2 t0 = cadd(y0, mul_mi<true>(y2));
    const float2 t1 = csub(y0, mul_mi<true>(y2));
    const float2 p1 = mul_w16<2, true>(y1);
    const float2 t2 = cfma<false>(y3, w16c<6>(), p1);
    const float2 t3 = mul_mi<true>(twice_minus(p1, t2));
    y0 = cadd(t0, t2);
    y2 = csub(t0, t2);
    y1 = cadd(t1, t3);
    y3 = csub(t1, t3);
  } else {
    // factors 1, conj W^B2, conj W^2B2, conj W^3B2 (none trivial for B2 = 1, 3)
    const float2 t0 = cfma<false>(y2, w16c<2 * B2>(), y0);
    const float2 t1 = twice_minus(y0, t0);
    const float2 p1 = mul_w16<B2, true>(y1);
    const float2 t2 = cfma<false>(y3, w16c<3 * B2>(), p1);
    const float2 t3 = mul_mi<true>(twice_minus(p1, t2));
    y0 = cadd(t0, t2);
    y2 = csub(t0, t2);
    y1 = cadd(t1, t3);
    y3 = csub(t1, t3);
  }
}

// Inverse DFT16 of v[i]*c[i] (CJ: v[i]*conj(c[i])); ONE0: c[0] = 1.
template <bool CJ, bool ONE0>
OLS_HD void idft16_premul(float2* v, const float2* c) {
  float2 y[4][4];
#pragma unroll
  for (int a1 = 0; a1 < 4; ++a1) {
    y[a1][0] = v[a1];
    y[a1][1] = v[a1 + 4];
    y[a1][2] = v[a1 + 8];
    y[a1][3] = v[a1 + 12];
  }
  idft4_premul<CJ, ONE0>(y[0][0], y[0][1], y[0][2], y[0][3], c[0], c[4], c[8], c[12]);
  idft4_premul<CJ, false>(y[1][0], y[1][1], y[1][2], y[1][3], c[1], c[5], c[9], c[13]);
  idft4_premul<CJ, false>(y[2][0], y[2][1], y[2][2], y[2][3], c[2], c[6], c[10], c[14]);
  idft4_premul<CJ, false>(y[3][0], y[3][1], y[3][2], y[3][3], c[3], c[7], c[11], c[15]);
  idft16_col<0>(y[0][0], y[1][0], y[2][0], y[3][0]);
  idft16_col<1>(y[0][1], y[1][1], y[2][1], y[3][1]);
  idft16_col<2>(y[0][2], y[1][2], y[2][2], y[3][2]);
  idft16_col<3>(y[0][3], y[1][3], y[2][3], y[3][3]);
#pragma unroll
  for (int b2 = 0; b2 < 4; ++b2) {
    v[b2] = y[0][b2];
    v[b2 + 4] = y[1][b2];
    v[b2 + 8] = y[2][b2];
    v[b2 + 12] = y[3][b2];
  }
}

// Inverse DFT8 of v[i]*c[i]; a = a1 + 2 a2, b = b2 + 4 b1.
template <bool CJ, bool ONE0>
OLS_HD void idft8_premul(float2* v, const float2* c) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  idft4_premul<CJ, ONE0>(e0, e1, e2, e3, c[0], c[2], c[4], c[6]);
  idft4_premul<CJ, false>(o0, o1, o2, o3, c[1], c[3], c[5], c[7]);
  // X[b2] = e[b2] + o[b2] conj(W8^b2), X[b2+4] = e[b2] - o[b2] conj(W8^b2)
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cfma<false>(o1, w16c<2>(), e1);
  v[5] = twice_minus(e1, v[1]);
  const float2 o2t = mul_mi<true>(o2);
  v[2] = cadd(e2, o2t);
  v[6] = csub(e2, o2t);
  v[3] = cfma<false>(o3, w16c<6>(), e3);
  v[7] = twice_minus(e3, v[3]);
}

template <bool CJ, bool ONE0>
OLS_HD void idft4_premul_arr(float2* v, const float2* c) {
  idft4_premul<CJ, ONE0>(v[0], v[1], v[2], v[3], c[0], c[1], c[2], c[3]);
}

template <bool CJ, bool ONE0>
OLS_HD void idft2_premul(float2* v, const float2* c) {
  const float2 p0 = ONE0 ? v[0] : cmul_k<CJ>(v[0], c[0]);
  v[0] = cfma<CJ>(v[1], c[1], p0);
  v[1] = twice_minus(p0, v[0]);
}

template <int RADIX, bool CJ, bool ONE0>
OLS_HD void idft_premul(float2* v, const float2* c) {
  if constexpr (RADIX == 2) idft2_premul<CJ, ONE0>(v, c);
  else if constexpr (RADIX == 4) idft4_premul_arr<CJ, ONE0>(v, c);
  else if constexpr (RADIX == 8) idft8_premul<CJ, ONE0>(v, c);
  else if constexpr (RADIX == 16) idft16_premul<CJ, ONE0>(v, c);
  else static_assert(RADIX == 2, "unsupported radix");
}

// Inverse pass K with its conjugate twiddles fused into the butterflies.
template <int N, int K>
OLS_HD void inverse_pass(float2 (&x)[16], const float2* tw) {
  using GE = Geo<N>;
  constexpr int RK = GE::radix(K);
  if constexpr (K < GE::P - 1) {
#pragma unroll
    for (int j = 0; j < GE::slots(K); ++j) {
      float2 c[RK];
      c[0] = make_float2(1.f, 0.f);
#pragma unroll
      for (int b = 1; b < RK; ++b) c[b] = tw[j * (RK - 1) + b - 1];
      idft_premul<RK, true, true>(&x[j * RK], c);
    }
  } else {
#pragma unroll
    for (int j = 0; j < GE::slots(K); ++j) dft<RK, true>(&x[j * RK]);
  }
}

// Point-wise product with the filter spectrum fused into the first inverse
// pass (the last forward pass, radix 16, has no twiddles).  x holds the
// filter spectrum on entry (the product commutes) and the pass output on exit.
template <int N>
OLS_HD void product_pass(float2 (&x)[16], const float2 (&A)[16]) {
  static_assert(Geo<N>::radix(Geo<N>::P - 1) == 16, "last pass is radix 16");
  idft16_premul<false, false>(x, A);
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
template <int N, class P>
OLS_HD void load_lane_twiddles(float2 (&tw)[Geo<N>::TWR], P table, int g) {
  using GE = Geo<N>;
#pragma unroll
  for (int k = 0; k < GE::P - 1; ++k) {
    const int RK = GE::radix(k), S = GE::strd(k);
#pragma unroll
    for (int j = 0; j < GE::slots(k); ++j) {
      const int l = GE::tw_index(k, g, j);
#pragma unroll
      for (int b = 1; b < RK; ++b)
        tw[GE::lane_tw_offset(k) + j * (RK - 1) + b - 1] = load_c64(table, GE::tw_offset(k) + (b - 1) * S + l);
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
