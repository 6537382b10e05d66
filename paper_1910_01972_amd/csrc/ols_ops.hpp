// Per-lane steps of the fused overlap-and-save kernel (sec. 3.2, Alg. 2):
// segment load with zero fill, spectrum product, discard-and-store.  Shared by
// the device kernels and by the host emulator used in CPU tests.
#pragma once

#include <type_traits>

#include "ols_fft.hpp"

namespace ols {

// Segment j covers signal samples start .. start + N - 1 with
// start = j*H - D (D >= M-1 samples of history, sec. 3.2); samples outside
// [0, N_s) read as zero.  Register reg of lane g receives the sample at
// position g + time_pos_const(reg) of the segment.
template <int N, class P>
OLS_HD void load_segment(float2 (&x)[16], P __restrict__ s, int64_t Ns, int64_t start, int g) {
  // valid positions p satisfy lo <= p < hi (clamped into [0, N])
  const int64_t lo64 = -start, hi64 = Ns - start;
  const int lo = lo64 <= 0 ? 0 : (lo64 >= N ? N : (int)lo64);
  const int hi = hi64 <= 0 ? 0 : (hi64 >= N ? N : (int)hi64);
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    x[reg] = (p >= lo && p < hi) ? load_c64(s, start + p) : make_float2(0.f, 0.f);
  }
}

// Filter r zero padded to N (plan step, Fig. 1 / Alg. 2): register reg of
// lane g receives tap g + time_pos_const(reg) - shift if that is in [0, M)
// (shift > 0 delays the filter by that many samples; see row_shift).
template <int N>
OLS_HD void load_filter(float2 (&x)[16], const float2* __restrict__ h, int M, bool valid, int g, int shift = 0) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg) - shift;
    x[reg] = (valid && p >= 0 && p < M) ? h[p] : make_float2(0.f, 0.f);
  }
}

// Filter r followed by a first difference, h'[k] = h[k] - h[k-1] for
// k = 0 .. M (h[-1] = h[M] = 0): y' = y * [1, -1] is the derivative of the
// convolved signal (sec. 4, non-local post-processing) and, being a
// convolution, it folds into the filter spectrum at no cost per segment.
template <int N>
OLS_HD void load_filter_diff(float2 (&x)[16], const float2* __restrict__ h, int M, bool valid, int g, int shift = 0) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg) - shift;
    const float2 a = (valid && p >= 0 && p < M) ? h[p] : make_float2(0.f, 0.f);
    const float2 b = (valid && p >= 1 && p <= M) ? h[p - 1] : make_float2(0.f, 0.f);
    x[reg] = csub(a, b);
  }
}

// Real filter r (R2R plans) as complex taps with zero imaginary part,
// optionally followed by the first difference of load_filter_diff.
template <int N>
OLS_HD void load_filter_real(float2 (&x)[16], const float* __restrict__ h, int M, bool valid, bool diff, int g,
                             int shift = 0) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg) - shift;
    float a = (valid && p >= 0 && p < M) ? h[p] : 0.f;
    if (diff) a -= (valid && p >= 1 && p <= M) ? h[p - 1] : 0.f;
    x[reg] = make_float2(a, 0.f);
  }
}

// Two real segments in one complex transform (R2R): segment 2q in the real
// part, segment 2q+1 in the imaginary part.  With real filters the product
// of their joint spectrum with a filter spectrum transforms back to the two
// real convolutions in the real and imaginary parts, so the pair costs one
// complex FFT of length N and needs no split of the spectra.  start is the
// window start of segment 2q; segment 2q+1 starts H samples later.
template <int N, class P>
OLS_HD void load_segment_pair(float2 (&x)[16], P __restrict__ s, int64_t Ns, int64_t start, int H, int g) {
  const int64_t lo0 = -start, hi0 = Ns - start;
  const int lo_a = lo0 <= 0 ? 0 : (lo0 >= N ? N : (int)lo0);
  const int hi_a = hi0 <= 0 ? 0 : (hi0 >= N ? N : (int)hi0);
  const int64_t lo1 = lo0 - H, hi1 = hi0 - H;
  const int lo_b = lo1 <= 0 ? 0 : (lo1 >= N ? N : (int)lo1);
  const int hi_b = hi1 <= 0 ? 0 : (hi1 >= N ? N : (int)hi1);
  const P sa = s + start;
  const P sb = sa + H;
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    x[reg] = make_float2((p >= lo_a && p < hi_a) ? sa[p] : 0.f, (p >= lo_b && p < hi_b) ? sb[p] : 0.f);
  }
}

// Spectra are stored in the order the forward transform leaves them in
// registers, two registers of a lane side by side: F[r][reg/2][g][reg%2].
// Each lane then loads its 16 values with 8 16-byte loads, and a wave reads
// 1 KB contiguous per load (half the load instructions of 8-byte loads;
// 3-6 % faster forward kernels).
template <int N>
OLS_HD int spectrum_offset(int reg, int g) { return (((reg >> 1) * Geo<N>::G + g) << 1) + (reg & 1); }

template <int N, class P>
OLS_HD void load_spectrum(float2 (&f)[16], P __restrict__ F, int r, int g) {
  const auto Fr = rebind_ptr<const f32x4>(F + (int64_t)r * N);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const f32x4 v = Fr[j * Geo<N>::G + g];
    f[2 * j] = make_float2(v.x, v.y);
    f[2 * j + 1] = make_float2(v.z, v.w);
  }
}

template <int N>
OLS_HD void store_spectrum(const float2 (&x)[16], float2* __restrict__ F, int r, int g, float scale) {
  float2* Fr = F + (int64_t)r * N;
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) Fr[spectrum_offset<N>(reg, g)] = cscale(x[reg], scale);
}

// x = A * f (point-wise product in the permuted frequency order, sec. 3.4)
OLS_HD void spectrum_product(float2 (&x)[16], const float2 (&A)[16], const float2 (&f)[16]) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) x[reg] = cmul(A[reg], f[reg]);
}

// Output stores.  Forward outputs are written once and never read back by
// the kernel, so they take the non-temporal (streaming) cache policy, which
// measured ~7 % faster than default stores on the filter-bank benchmark.
// When a transform spans whole waves (G >= 64) a wave's segment and output
// row are wave-uniform, so the stores go through a buffer resource covering
// exactly the kept outputs: the hardware range check drops the aliased and
// past-the-end positions (a negative offset wraps to a huge unsigned one),
// with no per-lane compare or branch.  Smaller transforms share a wave
// between segments and use per-lane predicates.
//
// Non-temporal stores only pay for whole 64-byte granules.  A granule that
// one store instruction covers only in part (rows of complex outputs whose
// length N_s is not a multiple of 8 start off the 64-byte grid; so can a
// segment edge) is written with the default policy instead, so that its two
// partial writes can merge in L2 before they go to HBM: with non-temporal
// partial writes the forward kernel ran 1.5-1.75x slower when its rows were
// off the grid, with the split policy 1.15x.  The batched kernel uses the
// split policy too (its rows, of arbitrary length, are mostly off the grid;
// the uneven batch ran 13 % faster with every row on the grid).
// How a kernel writes its outputs: plain per-lane predicated stores,
// non-temporal predicated stores, or non-temporal stores for whole granules
// only (buffer stores when G >= 64, predicated ones otherwise).  Kernels
// near the register limit keep the cheaper forms.
enum StoreMode { STORE_PLAIN = 0, STORE_NT = 1, STORE_NT_WHOLE = 2 };

// P: float* or gptr<float> (float2* or gptr<float2> for the complex form)
template <int MODE, typename P>
OLS_HD void out_store(P p, float v) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (MODE != STORE_PLAIN) {
    __builtin_nontemporal_store(v, p);
    return;
  }
#endif
  *p = v;
}

template <int MODE, typename P>
OLS_HD void out_store(P p, float2 v) {
  out_store<MODE>(&p->x, v.x);
  out_store<MODE>(&p->y, v.y);
}

// Vector elements (packed stencil phases): one store of the whole vector.
template <int MODE, typename P>
OLS_HD void out_store(P p, f32x2 v) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (MODE != STORE_PLAIN) {
    __builtin_nontemporal_store(v, p);
    return;
  }
#endif
  *p = v;
}

template <int MODE, typename P>
OLS_HD void out_store(P p, f32x4 v) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (MODE != STORE_PLAIN) {
    __builtin_nontemporal_store(v, p);
    return;
  }
#endif
  *p = v;
}

#if defined(__HIP_DEVICE_COMPILE__)
constexpr int CPOL_NT = 2;  // cache-policy operand of the buffer builtins: nt

// Raw buffer over [base, base + bytes): accesses at offsets >= bytes are
// dropped by the range check.
template <class P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(P base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, 0x00020000);
}

template <int CPOL>
__device__ __forceinline__ void buffer_store(float2 v, __amdgpu_buffer_rsrc_t rs, int off) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  u32x2 d;
  d.x = __float_as_uint(v.x);
  d.y = __float_as_uint(v.y);
  __builtin_amdgcn_raw_buffer_store_b64(d, rs, off, 0, CPOL);
}

template <int CPOL>
__device__ __forceinline__ void buffer_store(float v, __amdgpu_buffer_rsrc_t rs, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, off, 0, CPOL);
}

template <int CPOL>
__device__ __forceinline__ void buffer_store(f32x2 v, __amdgpu_buffer_rsrc_t rs, int off) {
  buffer_store<CPOL>(make_float2(v.x, v.y), rs, off);
}

template <int CPOL>
__device__ __forceinline__ void buffer_store(f32x4 v, __amdgpu_buffer_rsrc_t rs, int off) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  u32x4 d;
  d.x = __float_as_uint(v.x);
  d.y = __float_as_uint(v.y);
  d.z = __float_as_uint(v.z);
  d.w = __float_as_uint(v.w);
  __builtin_amdgcn_raw_buffer_store_b128(d, rs, off, 0, CPOL);
}
#endif

// Number of outputs a segment whose first output is out0 keeps: min(H, N_s - out0), >= 0.
OLS_HD int kept_count(int64_t Ns, int64_t out0, int H) {
  const int64_t rem = Ns - out0;
  return rem >= H ? H : (rem < 0 ? 0 : (int)rem);
}

// Position of an element inside its 64-byte granule, in elements.
template <typename T>
OLS_HD int granule_phase(const T* p) {
  return (int)(((uintptr_t)p / sizeof(T)) & (64 / sizeof(T) - 1));
}

// Stores of one segment's kept outputs.  After the inverse transform register
// reg of lane g holds circular position p = g + time_pos_const(reg); positions
// D .. D+H-1 are unaliased (D >= M-1, sec. 3.2) and go to outputs
// out0 + p - D, out0 = j*H; outputs >= N_s are not written.  val(reg) gives
// the value stored from register reg.
//
// STORE_NT_WHOLE: one store instruction writes C = min(G, 64) consecutive
// positions of a segment (lane l = g mod C of a chunk that starts on a
// multiple of C; time_pos_const is a multiple of G, and of LS, the outputs
// per 64-byte granule).  The phase c of a lane's output inside its granule
// is therefore the same in every register, so whether the chunk holds the
// lane's whole granule (l - c >= 0 and l - c + LS <= C) is a property of the
// lane: those lanes store non-temporally, the others (the partial granules
// at the two ends of each chunk when the row is off the 64-byte grid) with
// the default policy.  The first and last granule of a segment are partial
// when they share a granule with the neighbouring segment; the chunk test
// sees that exactly when the segment's kept positions start and end on chunk
// boundaries (D a multiple of C, and D + H = N as with the default hop),
// otherwise its head and tail granules may go non-temporal, two granules in
// H / LS.  The choice of policy never changes what is written.
// Registers R0 .. R0 + NR - 1 only (callers that produce the values in parts).
template <int N, int MODE, int R0 = 0, int NR = 16, typename T, typename V>
OLS_HD void store_segment(T* __restrict__ yrow, int64_t Ns, int64_t out0, int D, int H, int g, V val) {
  // T is float2 or float, with the pointer's address space (gptr) if any
  constexpr int LS = 64 / (int)sizeof(T);                // outputs per 64-byte granule
  constexpr int C = Geo<N>::G < 64 ? Geo<N>::G : 64;     // positions per store instruction
  static_assert(C % LS == 0, "chunks hold whole granules");
  const int cnt = kept_count(Ns, out0, H);
  const int l = g & (C - 1);
  const int c = (granule_phase(yrow + out0) + g - D) & (LS - 1);
  const bool whole = l >= c && l - c + LS <= C;
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (MODE == STORE_NT_WHOLE && Geo<N>::G >= 64) {
    // a wave holds one segment here, so its row, first output and count are
    // wave-uniform; saying so keeps the descriptor in scalar registers (the
    // compiler cannot always prove it, and would loop over the lanes)
    const __amdgpu_buffer_rsrc_t rs =
        out_rsrc(wave_uniform_ptr(yrow + out0), __builtin_amdgcn_readfirstlane(cnt * (int)sizeof(T)));
    if (whole) {
#pragma unroll
      for (int reg = R0; reg < R0 + NR; ++reg)
        buffer_store<CPOL_NT>(val(reg), rs, (g + time_pos_const<N>(reg) - D) * (int)sizeof(T));
    } else {
#pragma unroll
      for (int reg = R0; reg < R0 + NR; ++reg)
        buffer_store<0>(val(reg), rs, (g + time_pos_const<N>(reg) - D) * (int)sizeof(T));
    }
    return;
  }
#endif
  T* base = yrow + (out0 - D);
  if (MODE == STORE_NT || (MODE == STORE_NT_WHOLE && whole)) {
#pragma unroll
    for (int reg = R0; reg < R0 + NR; ++reg) {
      const int p = g + time_pos_const<N>(reg);
      if (p >= D && p < D + cnt) out_store<STORE_NT>(base + p, val(reg));
    }
  } else {
#pragma unroll
    for (int reg = R0; reg < R0 + NR; ++reg) {
      const int p = g + time_pos_const<N>(reg);
      if (p >= D && p < D + cnt) out_store<STORE_PLAIN>(base + p, val(reg));
    }
  }
}

// F maps the transform value to the stored one (the identity, or the power
// epilogue of sec. 4 with a float output).
template <int N, int MODE, typename T, typename F>
OLS_HD void store_kept(const float2 (&x)[16], T* __restrict__ yrow, int64_t Ns, int64_t out0, int D, int H, int g,
                       F f) {
  store_segment<N, MODE>(yrow, Ns, out0, D, H, g, [&](int reg) { return f(x[reg]); });
}

struct Identity {
  OLS_HD float2 operator()(float2 v) const { return v; }
};
// Per-element post-processing at the store (sec. 4): the power |y|^2 as
// float32, half the output bytes of complex64.
struct Power {
  OLS_HD float operator()(float2 v) const { return fmaf(v.x, v.x, v.y * v.y); }
};

template <int N, int MODE = STORE_PLAIN, class P>
OLS_HD void store_valid(const float2 (&x)[16], P yrow, int64_t Ns, int64_t out0, int D, int H, int g) {
  store_kept<N, MODE>(x, yrow, Ns, out0, D, H, g, Identity());
}

template <int N, int MODE = STORE_PLAIN, class P>
OLS_HD void store_valid_power(const float2 (&x)[16], P yrow, int64_t Ns, int64_t out0, int D, int H, int g) {
  store_kept<N, MODE>(x, yrow, Ns, out0, D, H, g, Power());
}

// ---------------------------------------------------------------------------
// Non-local post-processing (sec. 4: an output may depend on its neighbours,
// the paper's examples being the numerical derivative and interpolation).
// After the inverse transform the segment's outputs are written to LDS in
// natural order; each kept position p then combines the outputs at p - L ..
// p + R into J values by a stencil with real weights and J outputs (phases) per sample,
//     z[J n + j] = sum_{d=-L}^{R} w[j][d + L] * y[n + d],   n = out0 + p - D,
// optionally followed by the power.  The kept positions must see unaliased
// neighbours: D >= M - 1 + L and D + H + R <= N (stencil_delay), so the last
// segment also reads samples past N_s, which the zero-filled segment load
// makes eq. (1)'s tail.  Any hop up to N - D - R gives the same result.
// ---------------------------------------------------------------------------
constexpr int STENCIL_MAX_PHASES = 4;  // J: outputs per sample
constexpr int STENCIL_MAX_TAPS = 8;    // T = L + 1 + R
constexpr int STENCIL_PAD = 8;         // staged slots before and after a segment (>= max L, R)

struct Stencil {
  int J;       // phases, 1 .. STENCIL_MAX_PHASES
  int L;       // taps before the sample
  int T;       // taps, L + 1 + R
  int packed;  // the output is aligned to J elements: J <= 2 takes stage_store_packed
  float w[STENCIL_MAX_PHASES][STENCIL_MAX_TAPS];  // w[j][d + L]; zero past T and J
};

// LDS slots of one staged segment: position p at STENCIL_PAD + p, so every
// tap of every position of the transform stays inside its own segment slots.
template <int N>
constexpr int stage_stride() { return N + 2 * STENCIL_PAD; }

// First kept position of a plan whose stencil reaches L back and R ahead
// (Meff: taps of the filter as applied): the default_delay rounding when
// D + R <= N - 1 still holds, else exactly Meff - 1 + L.  The hop may reach
// N - D - R.
OLS_HD int stencil_delay(int N, int Meff, int L, int R) {
  const int lo = Meff - 1 + L;
  const int d = (lo + 15) / 16 * 16;
  return d + R <= N - 1 ? d : lo;
}

// Default hop with a stencil: N - D - R, rounded down to a multiple of 16
// samples when it is at least 16, so that segments keep starting on the
// 128-byte output grid (as the plain default hop does).
OLS_HD int stencil_hop(int N, int D, int R) {
  const int h = N - D - R;
  return h >= 16 ? h & ~15 : h;
}

// The transform output of lane g (register reg = circular position
// g + time_pos_const(reg)) into the segment's LDS slots.
template <int N>
OLS_HD void stage_write(float2* __restrict__ region, const float2 (&x)[16], int g) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) region[STENCIL_PAD + g + time_pos_const<N>(reg)] = x[reg];
}

// Phase j of the stencil at the 16 positions of lane g.  The tap loop runs T
// times (wave-uniform); position p + d - L is read for tap d, inside the
// segment's slots for every p (|d - L| <= STENCIL_PAD), from staged outputs
// for every kept p.
template <int N, class S>
OLS_HD void stage_phase(float2 (&acc)[16], const float2* __restrict__ region, const S& st, int j, int g) {
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) acc[reg] = make_float2(0.f, 0.f);
  const float2* src = region + STENCIL_PAD + g - st.L;
  for (int d = 0; d < st.T; ++d) {
    const float wd = st.w[j][d];
#pragma unroll
    for (int reg = 0; reg < 16; ++reg) {
      const float2 v = src[d + time_pos_const<N>(reg)];
      acc[reg].x = fmaf(wd, v.x, acc[reg].x);
      acc[reg].y = fmaf(wd, v.y, acc[reg].y);
    }
  }
}

// Store of phase j of a segment's kept positions: position p (D <= p <
// D + cnt) goes to element J * (out0 + p - D) + j of the row.  Rows with
// J > 1 are written J elements apart by each instruction, so the default
// cache policy lets the phases of a granule merge in L2.  A wave-wide
// transform (G >= 64) stores through a buffer resource over exactly the
// segment's J * cnt elements, whose range check drops the other positions.
template <int N, typename T, typename V>
OLS_HD void store_phase(T* __restrict__ yrow, int64_t Ns, int64_t out0, int D, int H, int g, int J, int j, V val) {
  const int cnt = kept_count(Ns, out0, H);
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (Geo<N>::G >= 64) {
    const __amdgpu_buffer_rsrc_t rs = out_rsrc(wave_uniform_ptr(yrow + (int64_t)J * out0),
                                               __builtin_amdgcn_readfirstlane(J * cnt * (int)sizeof(T)));
#pragma unroll
    for (int reg = 0; reg < 16; ++reg)
      buffer_store<0>(val(reg), rs, ((g + time_pos_const<N>(reg) - D) * J + j) * (int)sizeof(T));
    return;
  }
#endif
  T* base = yrow + (int64_t)J * out0;
#pragma unroll
  for (int reg = 0; reg < 16; ++reg) {
    const int p = g + time_pos_const<N>(reg);
    if (p >= D && p < D + cnt) out_store<STORE_PLAIN>(base + (p - D) * J + j, val(reg));
  }
}

// All JC phases at positions R0 .. R0 + NR - 1 of lane g (acc[j][reg - R0]),
// each tap read from LDS once.
template <int N, int JC, int R0, int NR, class S>
OLS_HD void stage_phases(float2 (&acc)[JC][NR], const float2* __restrict__ region, const S& st, int g) {
#pragma unroll
  for (int j = 0; j < JC; ++j)
#pragma unroll
    for (int i = 0; i < NR; ++i) acc[j][i] = make_float2(0.f, 0.f);
  const float2* src = region + STENCIL_PAD + g - st.L;
  for (int d = 0; d < st.T; ++d) {
    float wd[JC];
#pragma unroll
    for (int j = 0; j < JC; ++j) wd[j] = st.w[j][d];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const float2 v = src[d + time_pos_const<N>(R0 + i)];
#pragma unroll
      for (int j = 0; j < JC; ++j) {
        acc[j][i].x = fmaf(wd[j], v.x, acc[j][i].x);
        acc[j][i].y = fmaf(wd[j], v.y, acc[j][i].y);
      }
    }
  }
}

// One (JC = 1) or two phases per position written as one element: a float2,
// float or the vector of the two phases, so that each store instruction
// covers consecutive positions whole and the store policy of store_segment
// (non-temporal for whole 64-byte granules) applies as to a plain row.
// yrow must be aligned to the element (Stencil::packed).
// The positions go in parts of STAGE_PART registers, which bounds the live
// accumulators.
constexpr int STAGE_PART = 4;
template <int N, int JC, bool POWER, bool REAL, int SMODE, int R0, class S, class P>
OLS_HD void stage_store_packed_part(const float2* __restrict__ region, const S& st, P yrow, int64_t Ns, int64_t out0,
                                    int D, int H, int g) {
  constexpr int NR = STAGE_PART;
  float2 acc[JC][NR];
  stage_phases<N, JC, R0, NR>(acc, region, st, g);
  if constexpr (REAL || POWER) {
    // float rows: component c of each phase (REAL) or the power (POWER)
    auto val = [&](int reg, int c) {
      float v[JC];
#pragma unroll
      for (int j = 0; j < JC; ++j) {
        const float2 a = acc[j][reg - R0];
        v[j] = REAL ? (c == 0 ? (POWER ? a.x * a.x : a.x) : (POWER ? a.y * a.y : a.y)) : Power()(a);
      }
      if constexpr (JC == 1) return v[0];
      else return f32x2{v[0], v[1]};
    };
    using V = typename std::conditional<JC == 1, float, f32x2>::type;
    const auto yv = rebind_ptr<V>(yrow);
    store_segment<N, SMODE, R0, NR>(yv, Ns, out0, D, H, g, [&](int reg) { return val(reg, 0); });
    if constexpr (REAL)
      store_segment<N, SMODE, R0, NR>(yv, Ns, out0 + H, D, H, g, [&](int reg) { return val(reg, 1); });
  } else if constexpr (JC == 1) {
    store_segment<N, SMODE, R0, NR>(yrow, Ns, out0, D, H, g, [&](int reg) { return acc[0][reg - R0]; });
  } else {
    const auto yv = rebind_ptr<f32x4>(yrow);
    store_segment<N, SMODE, R0, NR>(yv, Ns, out0, D, H, g, [&](int reg) {
      const float2 a = acc[0][reg - R0], b = acc[1][reg - R0];
      return f32x4{a.x, a.y, b.x, b.y};
    });
  }
}

template <int N, int JC, bool POWER, bool REAL, int SMODE, class S, class P>
OLS_HD void stage_store_packed(const float2* __restrict__ region, const S& st, P yrow, int64_t Ns, int64_t out0,
                               int D, int H, int g) {
  static_assert(JC == 1 || JC == 2, "one or two phases per element");
  stage_store_packed_part<N, JC, POWER, REAL, SMODE, 0>(region, st, yrow, Ns, out0, D, H, g);
  stage_store_packed_part<N, JC, POWER, REAL, SMODE, STAGE_PART>(region, st, yrow, Ns, out0, D, H, g);
  if constexpr (STAGE_PART < 8) {
    stage_store_packed_part<N, JC, POWER, REAL, SMODE, 2 * STAGE_PART>(region, st, yrow, Ns, out0, D, H, g);
    stage_store_packed_part<N, JC, POWER, REAL, SMODE, 3 * STAGE_PART>(region, st, yrow, Ns, out0, D, H, g);
  }
}

// Every phase of the stencil for one filter's staged segment, stored to row
// yrow (J * N_s elements; float for POWER or REAL).  REAL: the staged values
// hold segment 2q in the real part and 2q + 1 in the imaginary part (R2R
// pairs), stored from out0 and out0 + H.  J <= 2 with an aligned output takes
// the packed form; otherwise each phase is computed and stored on its own,
// J elements apart.
template <int N, bool POWER, bool REAL, int SMODE = STORE_PLAIN, class S, class P>
OLS_HD void stage_store(const float2* __restrict__ region, const S& st, P yrow, int64_t Ns, int64_t out0, int D,
                        int H, int g) {
  if (st.packed && st.J == 1) {
    stage_store_packed<N, 1, POWER, REAL, SMODE>(region, st, yrow, Ns, out0, D, H, g);
    return;
  }
  if (st.packed && st.J == 2) {
    stage_store_packed<N, 2, POWER, REAL, SMODE>(region, st, yrow, Ns, out0, D, H, g);
    return;
  }
  for (int j = 0; j < st.J; ++j) {
    float2 acc[16];
    stage_phase<N>(acc, region, st, j, g);
    if constexpr (REAL) {
      store_phase<N>(yrow, Ns, out0, D, H, g, st.J, j,
                     [&](int reg) { return POWER ? acc[reg].x * acc[reg].x : acc[reg].x; });
      store_phase<N>(yrow, Ns, out0 + H, D, H, g, st.J, j,
                     [&](int reg) { return POWER ? acc[reg].y * acc[reg].y : acc[reg].y; });
    } else if constexpr (POWER) {
      store_phase<N>(yrow, Ns, out0, D, H, g, st.J, j, [&](int reg) { return Power()(acc[reg]); });
    } else {
      store_phase<N>(yrow, Ns, out0, D, H, g, st.J, j, [&](int reg) { return acc[reg]; });
    }
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

// Store of a segment pair (R2R): the real part holds segment 2q's output,
// written from out0 = 2q*H, the imaginary part segment 2q+1's, written from
// out0 + H; each with its own end bound.  POWER squares each sample.
template <int N, bool POWER, int MODE = STORE_PLAIN, class P>
OLS_HD void store_valid_pair(const float2 (&x)[16], P yrow, int64_t Ns, int64_t out0, int D, int H, int g) {
  store_segment<N, MODE>(yrow, Ns, out0, D, H, g,
                         [&](int reg) { return POWER ? x[reg].x * x[reg].x : x[reg].x; });
  store_segment<N, MODE>(yrow, Ns, out0 + H, D, H, g,
                         [&](int reg) { return POWER ? x[reg].y * x[reg].y : x[reg].y; });
}

// Filters per work unit of the forward kernels: two interleaved transforms
// when a transform spans several waves (N = 2048, 4096: the pair shares each
// exchange's barriers), registers allow it and the filter count wastes little
// on a padded last group.  Single-wave transforms (N <= 1024) exchange
// without barriers and measured as fast or faster with one filter per unit.
constexpr int BATCH_NF2_MAX_N = 2048;
OLS_HD int choose_nf(int N, int K) { return (N >= 2048 && N <= 4096 && (K % 2 == 0 || K >= 9)) ? 2 : 1; }
// The batched kernel's registers are set by its largest branch, so one filter
// per unit saves nothing there and two measured faster at every N <= 2048.
OLS_HD int choose_nf_batched(int N, int K) { return (N <= BATCH_NF2_MAX_N && (K % 2 == 0 || K >= 9)) ? 2 : 1; }
// R2R (segment pairs) needs a few more registers per transform: two filters
// per unit only up to N = 2048 as well.
OLS_HD int choose_nf_real(int N, int K) { return N <= BATCH_NF2_MAX_N ? choose_nf(N, K) : 1; }

// ---------------------------------------------------------------------------
// Segment geometry and FFT-length choice, shared by the host plan code and the
// device-side batch setup so that both always reach the same answer.
// ---------------------------------------------------------------------------
// First kept circular position: M - 1 rounded up to a multiple of 16 samples
// (128-byte aligned output windows) when that still leaves room, else M - 1.
OLS_HD int default_delay(int N, int M) {
  const int d = ((M - 1) + 15) / 16 * 16;
  return d <= N - 1 ? d : M - 1;
}

// Cost model for N = 0: transform work per kept output sample, about
// (K + 1) * 3.2 N log2 N + K * 4 N flops per segment over K * H kept samples,
// among N >= cost_model_min_n(K).  Compared as exact integers (5x the work,
// cross-multiplied by the hops) so that the host and the device pick the same
// N.  Lengths whose measured time per output is worse than their flop count
// says are left out:
//   * N = 256 and 512: their transforms are narrower than a wave and measured
//     10-24 % slower per output than N = 1024 on every cell of the
//     2^25-sample sweep where both fit, although they need up to ~10 % fewer
//     flops;
//   * N = 1024 for K >= COST_MODEL_WIDE_K filters: with the inverse
//     transforms dominating, N = 2048 measured 1-12 % faster per output
//     (K = 24 .. 64, M = 32, 128, 256, 2^25 samples) although it needs ~7 %
//     more flops; at K = 8 N = 1024 is 6-7 % faster, as the flops say.
// Returns 0 if no length in [cost_model_min_n(K), max_n] holds M taps.
constexpr int COST_MODEL_MIN_N = 1024;
constexpr int COST_MODEL_WIDE_K = 24;
OLS_HD int cost_model_min_n(int K) { return K >= COST_MODEL_WIDE_K ? 2 * COST_MODEL_MIN_N : COST_MODEL_MIN_N; }
OLS_HD int cost_model_fft_length(int K, int M, int max_n) {
  int best = 0;
  unsigned __int128 best_w = 0, best_h = 1;
  for (int n = cost_model_min_n(K); n <= max_n; n *= 2) {
    if (n < M) continue;
    const int h = n - default_delay(n, M);
    if (h < 1) continue;
    const unsigned __int128 w = (unsigned __int128)(K + 1) * 16u * (unsigned)n * (unsigned)ilog2(n) +
                                (unsigned __int128)K * 20u * (unsigned)n;
    if (best == 0 || w * best_h < best_w * (unsigned)h) {
      best = n;
      best_w = w;
      best_h = (unsigned)h;
    }
  }
  return best;
}

// Batched items: validation of one item (the checks ols_batch_plan and the
// workspace sizing do on the host, repeated by the device-side setup of
// ols_batched) and its FFT length.  Returns an ols_status_t value (0 = valid).
constexpr int BATCH_MIN_N = 256, BATCH_MAX_N = 4096;
OLS_HD int batch_item_check(const void* s, int64_t Ns, const void* h, int K, int M, int N, const void* y,
                            int* N_out) {
  if (K < 1 || M < 1 || Ns < 0) return 1;
  if (!h || (Ns > 0 && (!s || !y))) return 1;
  if (((uintptr_t)s | (uintptr_t)y | (uintptr_t)h) % 8) return 1;
  if (Ns > ((int64_t)1 << 56) / 8 / K) return 1;
  if (Ns > 0) {
    const uintptr_t s0 = (uintptr_t)s, s1 = s0 + (uintptr_t)Ns * 8;
    const uintptr_t y0 = (uintptr_t)y, y1 = y0 + (uintptr_t)Ns * 8 * (uintptr_t)K;
    if (s0 < y1 && y0 < s1) return 1;  // y overlaps s
  }
  int n = N;
  if (n == 0) {
    n = cost_model_fft_length(K, M, BATCH_MAX_N);
    if (n == 0) return 2;  // filter longer than the largest batched length
  }
  if (n < BATCH_MIN_N || n > BATCH_MAX_N || (n & (n - 1))) return 2;
  if (M > n) return 1;
  *N_out = n;
  return 0;
}

// Output rows off the 128-byte grid (the L2 line).  A row that starts off
// the grid (y not 128-byte aligned, or N_s not a multiple of LS, the outputs
// per line: 16 complex64 or 32 float32) would have every store
// instruction's run of consecutive outputs straddle two partly written
// lines.  For such a call each filter r is delayed by row_delay samples in
// its spectrum, which moves row r's outputs that many circular positions
// later: with the hop a multiple of LS, every store instruction then starts
// on a line (runs start at circular positions that are multiples of 64, or
// of the transform's G lanes), and only the two ends of each segment's kept
// window are partial.  The kept positions move with the filter (D + delay),
// so the hop must leave room for a delay of LS - 1.
struct RowShift {
  int H;     // hop the call runs with
  int mask;  // LS - 1 when the rows are shifted, else 0
};
constexpr int SHIFT_LINE = 128;  // bytes
// H: the plan's hop; el: bytes per output; allowed: the kernel supports it.
// The hop the call runs with is H rounded down to a multiple of LS, and no
// more than the room the delay leaves (N - D - (LS - 1), rounded down too);
// below LS the rows stay as they are.
OLS_HD RowShift row_shift_geometry(const void* y, int64_t Ns, int N, int D, int H, int el, bool allowed) {
  const int LS = SHIFT_LINE / el;
  const bool off = ((uintptr_t)y & (SHIFT_LINE - 1)) != 0 || (Ns & (LS - 1)) != 0;
  if (!allowed || !off) return RowShift{H, 0};
  const int room = (N - D - (LS - 1)) & ~(LS - 1);
  const int hs = (H & ~(LS - 1)) < room ? (H & ~(LS - 1)) : room;
  return hs >= LS ? RowShift{hs, LS - 1} : RowShift{H, 0};
}
// Delay of row r (0 .. mask): output n of row r is element r*N_s + n of y
// (el bytes each), and circular position p of segment j holds
// n = j*H - D + p - delay, so the line phase of a position p on the LS-sample
// grid is (y/el + r*N_s - D - delay) mod LS, which this delay makes 0.
OLS_HD int row_delay(const void* y, int el, int64_t Ns, int D, int r, int mask) {
  return (int)((((uintptr_t)y / (uintptr_t)el) + (uint64_t)r * (uint64_t)Ns - (uint64_t)D) & (uint64_t)mask);
}
// Batched items (complex64 rows, the default hop).
OLS_HD RowShift batch_row_shift(const void* y, int64_t Ns, int N, int D) {
  return row_shift_geometry(y, Ns, N, D, N - D, 8, true);
}

// Classes of batched items, (N, filters per unit): the kernel takes the items
// class by class (stable within a class), so that each workgroup meets each
// class in one run of tiles.
constexpr int BATCH_CLASSES = 10;
OLS_HD int batch_class(int N, int nf) { return 2 * (ilog2(N) - 8) + (nf - 1); }

// Schedule of the batched kernel (the device kernel and the host emulator
// both walk it through these functions).  Tiles of all items, numbered in the
// kernel's item order, are dealt to the P persistent workgroups round-robin:
// workgroup b takes tiles b, b + P, b + 2P, ..., so the grid as a whole works
// on a window of neighbouring tiles of one or two items (whose filter spectra
// then stay in L2).  Dealing chunks of 2-8 consecutive tiles instead measured
// 4-18 % slower on the uneven batch.
OLS_HD int64_t first_batch_tile(int64_t b) { return b; }
OLS_HD int64_t next_batch_tile(int64_t t, int64_t P) { return t + P; }
// Workgroup index b of launch index blk: the hardware deals workgroups to the
// 8 XCDs round-robin by launch index, so consecutive b (consecutive chunks of
// a round, which share overlap samples and spectra) are put on one XCD and
// its L2.  A permutation of [0, P).
OLS_HD int64_t batch_workgroup_order(int64_t blk, int64_t P) {
  return P % 8 == 0 ? (blk % 8) * (P / 8) + blk / 8 : blk;
}

// dh reduction order: the per-slot partial lags are summed in chunks of
// DH_CHUNK consecutive slots (each chunk in slot order, one thread per lag
// and chunk), then the chunk sums in chunk order.  Fixed order, no atomics.
constexpr int DH_CHUNK = 16;
OLS_HD int64_t dh_chunks(int64_t nslots) { return (nslots + DH_CHUNK - 1) / DH_CHUNK; }

// Walk of one workgroup over its units [u0, u1) of a single signal: unit u is
// filter group u mod KG of tile u / KG (a tile's groups in order, then the
// next tile).  The forward kernels and the host emulator both walk with it.
struct UnitWalk {
  int64_t tile;
  int rg;  // filter group within the tile; KG once the tile is done
  OLS_HD UnitWalk(int64_t u0, int KG) : tile(u0 / KG), rg((int)(u0 - (u0 / KG) * KG)) {}
  // At the start of a unit: past the tile's last group the unit starts the
  // next tile (new segments to transform).
  OLS_HD bool tile_done(int KG) const { return rg == KG; }
  OLS_HD void next_tile() {
    rg = 0;
    ++tile;
  }
  OLS_HD int next_group(int KG) const { return rg + 1 == KG ? 0 : rg + 1; }  // group of the unit after this one
  OLS_HD void leave() { ++rg; }
};

// Partition arithmetic shared by the persistent kernels: workgroup b of P
// owns units [first_unit(b), first_unit(b+1)); owner(u) inverts it.
OLS_HD int64_t first_unit(int64_t U, int64_t P, int64_t b) { return U * b / P; }
OLS_HD int64_t owner_of_unit(int64_t U, int64_t P, int64_t u) { return ((u + 1) * P + U - 1) / U - 1; }

}  // namespace ols
