// Device-side helpers: matrix-core (MFMA) wrappers for gfx950, precision
// traits, activation functions and wavefront utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpse {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// MFMA operand layouts on gfx950 (wave64; measured):
//   f64 16x16x4 : A[m][k] at lane m + 16k;  B[k][n] at lane n + 16k;
//                 D[m][n] at lane n + 16*(m%4), element m/4.
//   16x16x32 bf16/f16 : A[m][k] at lane m + 16*(k/8), element k%8;
//                 B[k][n] at lane n + 16*(k/8), element k%8;
//                 D[m][n] (f32) at lane n + 16*(m/4), element m%4.
//   16x16x16 f16 : A[m][k] at lane m + 16*(k/4), element k%4;
//                 B[k][n] at lane n + 16*(k/4), element k%4; D as above.
// A D-layout tile (m = feature, n = row) therefore serves unchanged as the
// B operand of the next product (k = feature, n = row) and as the A operand
// of a product with rows as m, once the k index is permuted as below.
//   f64 k-step (t, v)   : lane group g supplies feature 16t + 4v + g
//   16x16x32 k-step t, element j : lane group g supplies
//                         feature 32t + 16(j/4) + 4g + (j%4)
// Operands read from memory may use any k order that A and B share; the
// FP64 fitting GEMM uses 16t + 4g + v there (4 contiguous values per lane).
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));

// 16x16x16 FP16 product with FP32 accumulation (4 elements per lane).
__device__ __forceinline__ f4 mfma_f16k16(h16x4 a, h16x4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// Rounds 4 floats to FP16 (round to nearest even).
__device__ __forceinline__ h16x4 pack4_f16(const float* x) {
  return h16x4{(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
}

// Precision traits of the mixed forms.  vec8 is the 8-element operand of
// one 16x16x32 product; store_t the element type operands are kept in (in
// HBM and LDS), raw8 / raw4 vectors of 8 / 4 of them.  kind: 1 BF16, 2 FP16,
// 3 FP32 (the FP32 form issues the same 16x16x32 product as eight 16x16x4
// FP32 products, element j of both operands in product j: lane group g
// holds k = 8g + j in both layouts, so the sum over j is the full product).
struct PrecBF16 {
  typedef bf16x8 vec8;
  typedef uint16_t store_t;
  typedef u16x8 raw8;
  typedef u16x4 raw4;
  static constexpr int kind = 1;
  static __device__ __forceinline__ f4 mfma(vec8 a, vec8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t bits(float x) {
    __bf16 h = (__bf16)x;
    return __builtin_bit_cast(uint16_t, h);
  }
  static __device__ __forceinline__ float tof(uint16_t b) {
    return __builtin_bit_cast(float, ((uint32_t)b) << 16);
  }
};

struct PrecF16 {
  typedef h16x8 vec8;
  typedef uint16_t store_t;
  typedef u16x8 raw8;
  typedef u16x4 raw4;
  static constexpr int kind = 2;
  static __device__ __forceinline__ f4 mfma(vec8 a, vec8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t bits(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
  }
  static __device__ __forceinline__ float tof(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
  }
};

struct PrecF32 {
  typedef f32x8 vec8;
  typedef float store_t;
  typedef f32x8 raw8;
  typedef f4 raw4;
  static constexpr int kind = 3;
  static __device__ __forceinline__ f4 mfma(vec8 a, vec8 b, f4 c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
    return c;
  }
  static __device__ __forceinline__ float bits(float x) { return x; }
  static __device__ __forceinline__ float tof(float b) { return b; }
};

// Packs 8 floats into the 8-element operand of a 16x16x32 MFMA.
template <class P>
__device__ __forceinline__ typename P::vec8 pack8(const float* x) {
  if constexpr (P::kind == 3) {
    return f32x8{x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]};
  } else {
    u16x8 u;
#pragma unroll
    for (int j = 0; j < 8; ++j) u[j] = P::bits(x[j]);
    return __builtin_bit_cast(typename P::vec8, u);
  }
}

template <class P>
__device__ __forceinline__ typename P::vec8 load8(const typename P::store_t* p) {
  typename P::raw8 u = *reinterpret_cast<const typename P::raw8*>(p);
  return __builtin_bit_cast(typename P::vec8, u);
}

template <class P>
__device__ __forceinline__ typename P::raw8 zero8() {
  typename P::raw8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = 0;
  return z;
}

template <class P>
__device__ __forceinline__ typename P::raw8 join8(typename P::raw4 lo, typename P::raw4 hi) {
  typename P::raw8 z;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    z[j] = lo[j];
    z[4 + j] = hi[j];
  }
  return z;
}

// Stores 4 floats in the trait's element type.
template <class P>
__device__ __forceinline__ void store4(typename P::store_t* p, const float* v) {
  typename P::raw4 u;
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = P::bits(v[j]);
  *reinterpret_cast<typename P::raw4*>(p) = u;
}

// Per-net kernels on a one-row grid (the embedding nets, forward and
// backward, and their tabulated form): every net gets one work-group and
// the other G - nnets are split in proportion to the nets' work (a net's
// columns times its section's row tiles), the nets' shares laid out in
// decreasing order of work.  Work-group b serves the net
// whose share holds b, as the j-th of gk work-groups.  A grid of the
// work-groups the CUs hold at once then finishes every net in one round:
// with one net per grid row, the light nets' work-groups would wait for the
// heavy nets' slots and each work-group would get a few columns only, its
// waves idling at its end for up to one column each.  Returns -1 for b past
// the shares (none when G >= nnets and some net has work).
__device__ __forceinline__ int net_of_group(const int32_t* meta, const int* sec, int ntypes, int G, int b, int* j,
                                            int* gk) {
  const int nnets = ntypes * ntypes;
  auto wt = [&](int k) -> int64_t {
    const int kti = k / ntypes, ktj = k - kti * ntypes;
    return (int64_t)meta[2 * kti] * ((sec[ktj + 1] - sec[ktj] + 15) / 16);
  };
  int64_t total = 0;
  for (int k = 0; k < nnets; ++k) total += wt(k);
  const int64_t spare = G - nnets;
  for (int k = 0; k < nnets; ++k) {
    const int64_t wk = wt(k);
    int rank = 0;
    int64_t before = 0;  // work of the nets ranked before k
    for (int q = 0; q < nnets; ++q) {
      const int64_t wq = wt(q);
      if (wq > wk || (wq == wk && q < k)) {
        ++rank;
        before += wq;
      }
    }
    const int64_t lo = rank + (total > 0 ? spare * before / total : 0);
    const int64_t hi = rank + 1 + (total > 0 ? spare * (before + wk) / total : 0);
    if (b >= lo && b < hi) {
      *j = (int)(b - lo);
      *gk = (int)(hi - lo);
      return k;
    }
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Activations.  FP32 (mixed forms): 1 - 2/(e^{2x}+1) with the hardware exp2
// and reciprocal; saturates correctly at +-inf.
// FP64 tanh.  With t = |x| and e = exp(-2t) in (0, 1], tanh(t) = 2/(1 + e) - 1;
// the sign of x is copied onto the result.  t is carried as u = t/32 clamped
// to [0, 1] (one scaled, clamped instruction; tanh(32) rounds to 1).  Range
// reduction -2t = n ln2 + 2w, |w| <= ln2/4, with ln 2 split in a 32-bit head
// (n*head/64 is exact) and a tail; exp(2w) is a degree-11 polynomial fitted
// to it in the Chebyshev (near-minimax) sense, fit error 3e-18 relative,
// evaluated in w/32 with the coefficients scaled by 32^k (exact, so the
// roundings are those of the unscaled form).  The reciprocal is the hardware
// estimate q (relative error below 5e-8 on gfx950) refined in one step to
// third order: with r = 1 - d q, 1/d = q (1 + r + r^2 + ...), and
// q + q (r + r^2) leaves r^3 ~ 1e-22 (two Newton steps would cost one more
// instruction and round twice).  Absolute error below 5e-16 (about 2 ulp
// of 1); relative accuracy is lost only for |x| below ~1e-3, where the
// absolute error still is ~1e-16.  A NaN argument gives +-0: every caller's
// arguments derive from coordinates checked by the wrap test and parameters
// checked finite when the model is created.
__device__ __forceinline__ double tanh_d(double x) {
  const double u = __builtin_fmin(__builtin_fmax(__builtin_fabs(x) * 0.03125, 0.0), 1.0);
  const double n = rint(u * -92.33248261689366);  // -64/ln2
  double w = fma(-n, 0.01083042469326756, -u);    // head(ln2)/64
  w = fma(-n, 2.9815858269852933e-12, w);         // tail(ln2)/64
  double p = 1852793749593.745;
  p = fma(p, w, 318582644689.01984);
  p = fma(p, w, 49642711972.90849);
  p = fma(p, w, 6980997548.528086);
  p = fma(p, w, 872628278.1579455);
  p = fma(p, w, 95443718.12474826);
  p = fma(p, w, 8947848.533318589);
  p = fma(p, w, 699050.6666636708);
  p = fma(p, w, 43690.6666666667);
  p = fma(p, w, 2048.0000000000077);
  p = fma(p, w, 64.0);
  p = fma(p, w, 1.0);
  const double e = __builtin_amdgcn_ldexp(p, (int)n);
  const double d = 1.0 + e;
  const double q0 = __builtin_amdgcn_rcp(d);
  const double r = fma(-d, q0, 1.0);
  const double q = fma(q0, fma(r, r, r), q0);
  return __builtin_copysign(fma(2.0, q, -1.0), x);
}

// FP64 tanh with a table tab[j] = 2^(j/32), j = 0..31 (kept in LDS by the
// caller).  As in tanh_d, t = |x| is carried as u = t/32 clamped to [0, 1];
// with a = -2t = -64u and k = rint(a 32/ln 2), a = k ln2/32 + f with
// |f| <= ln2/64 (ln 2/32 split in a 36-bit head, so k head is exact for
// |k| < 2^17, and a tail), and e^a = 2^(k >> 5) tab[k & 31] e^f with e^f by
// its Taylor polynomial of degree 6 (truncation below 4e-18 relative),
// evaluated in w = f/64 with the coefficients 64^k/k! (exact scalings).
// The reciprocal and the result as in tanh_d, with six FP64 operations
// fewer than its degree-11 polynomial.
__device__ __forceinline__ double tanh_d_tab(double x, const double* tab) {
  const double u = __builtin_fmin(__builtin_fmax(__builtin_fabs(x) * 0.03125, 0.0), 1.0);
  const double k = rint(u * -2954.639443740597);    // -2048/ln 2
  double w = fma(-k, 0.0003384507717569818, -u);  // head(ln 2/32)/64
  w = fma(-k, 8.040014444773966e-16, w);          // tail(ln 2/32)/64
  double p = 95443717.68888889;
  p = fma(p, w, 8947848.533333333);
  p = fma(p, w, 699050.6666666666);
  p = fma(p, w, 43690.666666666664);
  p = fma(p, w, 2048.0);
  p = fma(p, w, 64.0);
  p = fma(p, w, 1.0);
  const int ki = (int)k;
  const double e = __builtin_amdgcn_ldexp(p * tab[ki & 31], ki >> 5);
  const double d = 1.0 + e;
  const double q0 = __builtin_amdgcn_rcp(d);
  const double r = fma(-d, q0, 1.0);
  const double q = fma(q0, fma(r, r, r), q0);
  return __builtin_copysign(fma(2.0, q, -1.0), x);
}

constexpr float kTanhScale = 2.8853900817779268f;  // 2/ln 2
// tanh(x) from y = x * kTanhScale, for producers that fold the scale into
// their own multiply-add (a bias stored pre-scaled: y = fma(z, scale, b'))
__device__ __forceinline__ float tanh_f_pre(float y) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f);
}
__device__ __forceinline__ float tanh_f(float x) { return tanh_f_pre(x * kTanhScale); }

// Rows of an environment-matrix section through a buffer resource that
// spans its nn valid rows (32 bytes each): the hardware's range check returns
// zeros for rows past them, so a load needs no branch around it and no
// select on its value.  With either, the compiler waits for every
// outstanding load at that point, where these loads are meant to stay in
// flight until their values are used.  Rs and nn are wave-uniform.
typedef __amdgpu_buffer_rsrc_t env_rsrc_t;
// Resource word 3 of an untyped buffer on this family: 32-bit data format
// (a zero format makes every load return zero).
constexpr int kBufWord3 = 0x00020000;
__device__ __forceinline__ env_rsrc_t env_rsrc(const double* Rs, int nn) {
  // uniform by the caller's contract; read from lane 0 so that the resource
  // is formed once in scalar registers
  const unsigned long long a = reinterpret_cast<unsigned long long>(Rs);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  void* const base = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, __builtin_amdgcn_readfirstlane(nn) * 32, kBufWord3);
}
__device__ __forceinline__ d4 env_row(env_rsrc_t r, int q) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v a = __builtin_amdgcn_raw_buffer_load_b128(r, q * 32, 0, 0);
  const u4v b = __builtin_amdgcn_raw_buffer_load_b128(r, q * 32 + 16, 0, 0);
  d4 x;
  x[0] = __builtin_bit_cast(double, (unsigned long long)a[0] | ((unsigned long long)a[1] << 32));
  x[1] = __builtin_bit_cast(double, (unsigned long long)a[2] | ((unsigned long long)a[3] << 32));
  x[2] = __builtin_bit_cast(double, (unsigned long long)b[0] | ((unsigned long long)b[1] << 32));
  x[3] = __builtin_bit_cast(double, (unsigned long long)b[2] | ((unsigned long long)b[3] << 32));
  return x;
}
// Element c of row q (same rule).
__device__ __forceinline__ double env_elt(env_rsrc_t r, int q, int c) {
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  const u2v a = __builtin_amdgcn_raw_buffer_load_b64(r, q * 32 + c * 8, 0, 0);
  return __builtin_bit_cast(double, (unsigned long long)a[0] | ((unsigned long long)a[1] << 32));
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, 64); }

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Orders the LDS traffic of one wavefront (lanes exchange data through LDS
// inside a wave-private region without a work-group barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hides a pointer's value from the optimiser for one loop iteration so that
// loads through it are not hoisted out of the loop (the weight fragments are
// loop-invariant across neighbour tiles; keeping all of them in registers
// would exhaust the register file).
// The pointer itself is not passed through the asm (that would turn it into
// a generic pointer and its loads into flat loads, which also count against
// the LDS wait counter): an opaque zero offset is added instead, so loads
// stay global.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
  int z = 0;
  asm volatile("" : "+v"(z));
  return p + z;
}

__device__ __forceinline__ void set_flag(int32_t* flags, int32_t bit) { atomicOr(flags, bit); }

}  // namespace dpse
