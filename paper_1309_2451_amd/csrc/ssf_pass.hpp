// Pencil-pass kernels of the 3-D split-operator step for CDNA4 (gfx950).
//
// One launch applies a 1-D DFT of length N to every pencil along one axis of
// a (nz, ny, nx) complex field, optionally fused with the pointwise factors of
// the Fourier split-operator method (Morgan et al., arXiv:1309.2451, Sec. IV):
// the potential phase exp(-i V c) on the way in or out, and -- for a fused
// forward/inverse pass -- the kinetic phase exp(-i k^2 dt/2) (or the potential
// phase) between the two transforms, so the factors cost no extra HBM sweep.
//
// Transform: Stockham autosort, stage radices from Plan<N>.  Stage s with
// radix r and p = product of the earlier radices turns input i + m N/r
// (m < r) into output j + q p with k = i mod p, j = (i - k) r + k, after
// multiplying input m by exp(sign 2 pi i m k / (p r)).  The first stage reads
// global memory and the last one writes it, both coalesced; the stages in
// between exchange through LDS.  Arithmetic is FP64 in registers whatever the
// storage type, so complex64 storage is rounded once per pass, at the store.
//
// Thread layout: a workgroup owns P pencils and every thread owns E values
// (E/r butterflies per stage).  Contiguous (x) passes map consecutive threads
// to consecutive butterflies of one pencil; strided (y, z) passes map them to
// consecutive x columns of a px-wide tile, so each global access is a run of
// px * sizeof(storage) contiguous bytes.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "ssf_internal.hpp"

namespace ssf {

// ---------------------------------------------------------------------------
// Plans: stage radices (forward order) and values per thread E, a common
// multiple of the radices.
// ---------------------------------------------------------------------------
template <int N> struct Plan;
#define SSF_PLAN(NN, EE, ...)                                              \
  template <> struct Plan<NN> {                                            \
    static constexpr int E = EE;                                           \
    static constexpr int R[] = {__VA_ARGS__};                              \
    static constexpr int S = sizeof(R) / sizeof(int);                      \
  };
SSF_PLAN(1, 1, 1)
SSF_PLAN(2, 2, 2)
SSF_PLAN(4, 4, 4)
SSF_PLAN(8, 8, 8)
SSF_PLAN(16, 16, 16)
SSF_PLAN(32, 8, 4, 8)
SSF_PLAN(64, 8, 8, 8)
SSF_PLAN(128, 8, 4, 4, 8)
SSF_PLAN(256, 8, 4, 8, 8)
SSF_PLAN(512, 8, 8, 8, 8)
SSF_PLAN(1024, 8, 4, 4, 8, 8)
SSF_PLAN(12, 12, 3, 4)
SSF_PLAN(24, 12, 2, 3, 4)
SSF_PLAN(48, 12, 3, 4, 4)
SSF_PLAN(96, 12, 4, 4, 2, 3)
SSF_PLAN(192, 12, 3, 4, 4, 4)
SSF_PLAN(384, 24, 3, 4, 4, 8)
SSF_PLAN(768, 24, 3, 4, 8, 8)
SSF_PLAN(20, 20, 4, 5)
SSF_PLAN(40, 20, 2, 4, 5)
SSF_PLAN(80, 20, 4, 4, 5)
SSF_PLAN(160, 20, 2, 4, 4, 5)
SSF_PLAN(320, 20, 4, 4, 4, 5)
SSF_PLAN(640, 20, 2, 4, 4, 4, 5)
#undef SSF_PLAN

template <class PL, bool REV> struct Order {
  static constexpr bool rev = REV;
  static constexpr int r(int s) { return REV ? PL::R[PL::S - 1 - s] : PL::R[s]; }
  static constexpr int p(int s) {
    int q = 1;
    for (int t = 0; t < s; ++t) q *= r(t);
    return q;
  }
};

// Build-time tuning switches (defaults are the measured best).
#ifndef SSF_TW_FULL
#define SSF_TW_FULL 0          // 1: load every twiddle power from LDS
#endif
#ifndef SSF_CR_SHIFT
#define SSF_CR_SHIFT 0         // x-pass rows per workgroup scaled by 2^shift
#endif
#ifndef SSF_STRIDED_MAXWG
#define SSF_STRIDED_MAXWG 1024 // largest y/z workgroup
#endif
#ifndef SSF_TILE_INTERLEAVE
#define SSF_TILE_INTERLEAVE 1  // y/z workgroups take every gridDim-th tile (0: a contiguous range)
#endif
#ifndef SSF_X32
#define SSF_X32 1              // FP32 LDS exchanges in the fused passes of complex64 fields
#endif

// Tile shapes.  LDS holds P pencils of N FP64 complex values.
constexpr int LDS_CAP_ELEMS = 8192;       // 128 KiB of double2
template <int N> struct Shape {
  static constexpr int E = Plan<N>::E;
  static constexpr int sx0(int dt) {               // variant-0 tile width in x
    int px = dt == 0 ? 16 : 8;                      // 128 B of storage per row segment
    while (px > 1 && px * N > LDS_CAP_ELEMS) px /= 2;
    return px;
  }
  static constexpr int so(int dt, int /*var*/ = 0) {   // strided tile depth (outer pencils), both variants
    int po = 256 * E / (N * sx0(dt));
    if (po < 1) po = 1;
    while (po > 1 && sx0(dt) * po * N > LDS_CAP_ELEMS) po /= 2;
    while (po > 1 && sx0(dt) * po * N / E > 1024) po /= 2;
    return po;
  }
  // Variant-0 values-per-thread multiplier.  A 1024-thread workgroup leaves
  // 128 registers per thread: enough for the 8-value plans up to N = 512
  // (measured faster than 512 threads with 16 values), not for N = 1024.
  static constexpr int sm0(int dt) {
    const int maxwg = N >= 1024 && SSF_STRIDED_MAXWG > 512 ? 512 : SSF_STRIDED_MAXWG;
    int em = 1;
    while (sx0(dt) * so(dt) * N / (E * em) > maxwg) em *= 2;
    return em;
  }
  // variant 1: half-width tile with the same values per thread, i.e. half
  // the workgroup and half the LDS, so twice as many workgroups share a CU
  static constexpr bool v1(int dt) { return sx0(dt) > 1; }
  static constexpr int sx(int dt, int var = 0) { return (var == 1 && v1(dt)) ? sx0(dt) / 2 : sx0(dt); }
  // variant 2: the variant-0 tile with twice the values per thread (at most
  // 16), half the workgroup, no register prefetch and (complex64) an FP32
  // LDS buffer of half the bytes, so two workgroups share a CU and one's
  // arithmetic overlaps the other's memory traffic instead of a prefetch
  static constexpr int sm(int dt, int var = 0) {
    return (var == 2 && Plan<N>::E * sm0(dt) * 2 <= 16 && N % (Plan<N>::E * sm0(dt) * 2) == 0) ? 2 * sm0(dt)
                                                                                                : sm0(dt);
  }
  static constexpr int ldrow() { return N; }
  static constexpr int cr() {              // contiguous rows per workgroup
    int rows = 256 * E / N;
    if (SSF_CR_SHIFT > 0) rows <<= SSF_CR_SHIFT;
    if (SSF_CR_SHIFT < 0) rows >>= -SSF_CR_SHIFT;
    if (rows < 1) rows = 1;
    while (rows > 1 && rows * ldrow() > 4096) rows /= 2;
    while (rows > 1 && rows * N / E > 1024) rows /= 2;
    return rows;
  }
};

// ---------------------------------------------------------------------------
// Complex helpers, for the register type C of a pass: double2 (FP64
// arithmetic, the default for both storage types) or float2 (FP32
// arithmetic, a selectable mode for complex64 storage).
// ---------------------------------------------------------------------------
template <class C> struct Cx;
template <> struct Cx<double2> {
  using R = double;
  __device__ static __forceinline__ double2 mk(double x, double y) { return make_double2(x, y); }
};
template <> struct Cx<float2> {
  using R = float;
  __device__ static __forceinline__ float2 mk(float x, float y) { return make_float2(x, y); }
};
// a complex value formed in FP64 (a phase factor, a table entry) in register type C
template <class C> __device__ __forceinline__ C to_c(double2 d) {
  return Cx<C>::mk((typename Cx<C>::R)d.x, (typename Cx<C>::R)d.y);
}
template <class C> __device__ __forceinline__ double2 to_d(C v) { return make_double2((double)v.x, (double)v.y); }
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return Cx<C>::mk(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return Cx<C>::mk(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  return Cx<C>::mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// x K for a butterfly constant K.  In FP32 the constant is split into two
// FP32 terms and the product is rounded once from (nearly) the exact x K.  A
// one-term FP32 constant would scale by the same 1 + (relative error of K) in
// every butterfly of every step, a systematic drift of the norm (for sqrt(1/2),
// -1.7e-8 on the odd outputs of each radix-8 butterfly).
template <class R> __device__ __forceinline__ R kmul(R x, double K) {
  if constexpr (sizeof(R) == 4) {
    const float hi = (float)K, lo = (float)(K - (double)hi);
    return __builtin_fmaf(x, hi, x * lo);
  } else {
    return x * K;
  }
}
template <class C> __device__ __forceinline__ C kscale(C a, double K) {
  return Cx<C>::mk(kmul(a.x, K), kmul(a.y, K));
}
template <class C> __device__ __forceinline__ C cscale(C a, double s) {
  const typename Cx<C>::R t = (typename Cx<C>::R)s;
  return Cx<C>::mk(a.x * t, a.y * t);
}
template <class C> __device__ __forceinline__ C conj2(C a) { return Cx<C>::mk(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, class C> __device__ __forceinline__ C mul_mi(C a) {
  return INV ? Cx<C>::mk(-a.y, a.x) : Cx<C>::mk(a.y, -a.x);
}
// multiply by exp(-/+ i pi/4) * sqrt2 ... as rotation by w8 = exp(-/+ 2 pi i / 8)
constexpr double SQRT1_2 = 0.70710678118654752440084436210485;
template <bool INV, class C> __device__ __forceinline__ C mul_w8_1(C a) {
  // fwd: (1 - i)/sqrt2, inv: (1 + i)/sqrt2
  return INV ? Cx<C>::mk(kmul(a.x - a.y, SQRT1_2), kmul(a.x + a.y, SQRT1_2))
             : Cx<C>::mk(kmul(a.x + a.y, SQRT1_2), kmul(a.y - a.x, SQRT1_2));
}
template <bool INV, class C> __device__ __forceinline__ C mul_w8_3(C a) {
  // fwd: (-1 - i)/sqrt2, inv: (-1 + i)/sqrt2
  return INV ? Cx<C>::mk(kmul(-a.x - a.y, SQRT1_2), kmul(a.x - a.y, SQRT1_2))
             : Cx<C>::mk(kmul(a.y - a.x, SQRT1_2), kmul(-a.x - a.y, SQRT1_2));
}

// Storage conversions.  Field and table pointers may come from a batch
// descriptor in memory rather than from the kernel arguments; the accesses
// name the global address space explicitly so that they compile to global
// (not flat) memory instructions, which do not tie up the LDS counter.
#define SSF_GLOBAL __attribute__((address_space(1)))
#define SSF_CONST __attribute__((address_space(4)))
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef double d2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldraw(const float2* p) {
  const f2v_t t = *(const SSF_GLOBAL f2v_t*)p;
  return make_float2(t.x, t.y);
}
__device__ __forceinline__ double2 ldraw(const double2* p) {
  const d2v_t t = *(const SSF_GLOBAL d2v_t*)p;
  return make_double2(t.x, t.y);
}
__device__ __forceinline__ double ldg(const double* p) { return *(const SSF_GLOBAL double*)p; }
__device__ __forceinline__ double2 ld2(const float2* p) { const float2 f = ldraw(p); return make_double2(f.x, f.y); }
__device__ __forceinline__ double2 ld2(const double2* p) { return ldraw(p); }
__device__ __forceinline__ void st2(float2* p, double2 v) {
  const f2v_t t = {(float)v.x, (float)v.y};
  *(SSF_GLOBAL f2v_t*)p = t;
}
__device__ __forceinline__ void st2(double2* p, double2 v) {
  const d2v_t t = {v.x, v.y};
  *(SSF_GLOBAL d2v_t*)p = t;
}
__device__ __forceinline__ void st2(float2* p, float2 v) {
  const f2v_t t = {v.x, v.y};
  *(SSF_GLOBAL f2v_t*)p = t;
}
// Value as it is after rounding to storage (for reductions that must see the stored field), in FP64.
__device__ __forceinline__ double2 rounded(double2 v, const float2*) { return make_double2((double)(float)v.x, (double)(float)v.y); }
__device__ __forceinline__ double2 rounded(double2 v, const double2*) { return v; }
__device__ __forceinline__ double2 rounded(float2 v, const float2*) { return make_double2((double)v.x, (double)v.y); }

// ---------------------------------------------------------------------------
// Small DFTs: y_q = sum_m x_m exp(sign 2 pi i m q / r), in place, sign = -1
// forward and +1 inverse.
// ---------------------------------------------------------------------------
template <int R, bool INV> struct Bfly;

template <bool INV> struct Bfly<1, INV> {
  template <class C> __device__ static void run(C*) {}
};

template <bool INV> struct Bfly<2, INV> {
  template <class C> __device__ static void run(C* x) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV> struct Bfly<4, INV> {
  template <class C> __device__ static void run(C* x) {
    C t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    C t2 = cadd(x[1], x[3]), t3 = mul_mi<INV>(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
  }
};

template <bool INV> struct Bfly<8, INV> {
  template <class C> __device__ static void run(C* x) {
    C e[4] = {x[0], x[2], x[4], x[6]};
    C o[4] = {x[1], x[3], x[5], x[7]};
    Bfly<4, INV>::run(e);
    Bfly<4, INV>::run(o);
    o[1] = mul_w8_1<INV>(o[1]);
    o[2] = mul_mi<INV>(o[2]);
    o[3] = mul_w8_3<INV>(o[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = cadd(e[q], o[q]);
      x[q + 4] = csub(e[q], o[q]);
    }
  }
};

// cos and sin of 2 pi q / 16, q = 0..7
__device__ constexpr double C16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                      0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double S16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                      1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};

template <bool INV> struct Bfly<16, INV> {
  template <class C> __device__ static void run(C* x) {
    C e[8], o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) { e[q] = x[2 * q]; o[q] = x[2 * q + 1]; }
    Bfly<8, INV>::run(e);
    Bfly<8, INV>::run(o);
#pragma unroll
    for (int q = 1; q < 8; ++q) {
      const C w = to_c<C>(make_double2(C16[q], INV ? S16[q] : -S16[q]));
      o[q] = cmul(o[q], w);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      x[q] = cadd(e[q], o[q]);
      x[q + 8] = csub(e[q], o[q]);
    }
  }
};

constexpr double SIN_2PI_3 = 0.86602540378443864676372317075294;  // sqrt(3)/2
template <bool INV> struct Bfly<3, INV> {
  template <class C> __device__ static void run(C* x) {
    using R = typename Cx<C>::R;
    C t = cadd(x[1], x[2]);
    C s = csub(x[1], x[2]);
    C a = Cx<C>::mk(x[0].x - (R)0.5 * t.x, x[0].y - (R)0.5 * t.y);
    // fwd: y1 = a - i (sqrt3/2) s, y2 = a + i (sqrt3/2) s
    C b = mul_mi<INV>(kscale(s, SIN_2PI_3));
    x[0] = cadd(x[0], t);
    x[1] = cadd(a, b);
    x[2] = csub(a, b);
  }
};

constexpr double C1_5 = 0.30901699437494742410229341718282;   // cos(2 pi / 5)
constexpr double C2_5 = -0.80901699437494742410229341718282;  // cos(4 pi / 5)
constexpr double S1_5 = 0.95105651629515357211643933337938;   // sin(2 pi / 5)
constexpr double S2_5 = 0.58778525229247312916870595463907;   // sin(4 pi / 5)
template <bool INV> struct Bfly<5, INV> {
  template <class C> __device__ static void run(C* x) {
    C a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
    C b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
    C x0 = x[0];
    C r1 = Cx<C>::mk(x0.x + kmul(a1.x, C1_5) + kmul(a2.x, C2_5), x0.y + kmul(a1.y, C1_5) + kmul(a2.y, C2_5));
    C r2 = Cx<C>::mk(x0.x + kmul(a1.x, C2_5) + kmul(a2.x, C1_5), x0.y + kmul(a1.y, C2_5) + kmul(a2.y, C1_5));
    C i1 = Cx<C>::mk(kmul(b1.x, S1_5) + kmul(b2.x, S2_5), kmul(b1.y, S1_5) + kmul(b2.y, S2_5));
    C i2 = Cx<C>::mk(kmul(b1.x, S2_5) - kmul(b2.x, S1_5), kmul(b1.y, S2_5) - kmul(b2.y, S1_5));
    // fwd: y1 = r1 - i i1, y4 = r1 + i i1, y2 = r2 - i i2, y3 = r2 + i i2
    C j1 = mul_mi<INV>(i1), j2 = mul_mi<INV>(i2);
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(r1, j1);
    x[4] = csub(r1, j1);
    x[2] = cadd(r2, j2);
    x[3] = csub(r2, j2);
  }
};

// ---------------------------------------------------------------------------
// Phase factors.  theta = V * c.  Real time: exp(-i theta); imaginary time:
// exp(-theta).
//
// sincos: Cody-Waite reduction by pi/2 with a two-part constant (the product
// q * (pi/2)_hi is exact inside the fused multiply-add), then the Taylor
// series of sin to degree 17 and of cos to degree 18 on |r| <= pi/4, whose
// truncation error is below 5e-17; quadrant by q mod 4.  About 1 ulp for
// |theta| up to 1e5 (checked against long-double sin/cos on the host).
// ---------------------------------------------------------------------------
constexpr double TWO_OVER_PI = 0.63661977236758134308;
constexpr double PIO2_HI = 1.5707963267948966192;       // nearest double to pi/2
constexpr double PIO2_LO = 6.123233995736766036e-17;    // pi/2 - PIO2_HI
// Taylor coefficients (-1)^k / (2k+1)! for sin (k = 8..1) and (-1)^k / (2k)!
// for cos (k = 9..1), read from constant memory so that they stay in scalar
// registers instead of vector registers.
__constant__ double SINCOS_C[17] = {
    1.0 / 355687428096000.0, -1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0,
    1.0 / 362880.0, -1.0 / 5040.0, 1.0 / 120.0, -1.0 / 6.0,
    1.0 / 6402373705728000.0, -1.0 / 20922789888000.0, 1.0 / 87178291200.0, -1.0 / 479001600.0,
    1.0 / 3628800.0, -1.0 / 40320.0, 1.0 / 720.0, -1.0 / 24.0, 0.5};
//
// LOW (complex64 storage, whose values carry 6e-8 relative rounding): sin to
// degree 13 and cos to degree 14 after the reduction (truncation error below
// 3e-14), and degree 11/12 without it (below 7e-12).
template <bool LOW = false>
__device__ __forceinline__ void sincos_fast(double t, double* s, double* c) {
  const double q = rint(t * TWO_OVER_PI);
  double r = fma(-q, PIO2_HI, t);
  r = fma(-q, PIO2_LO, r);
  const double r2 = r * r;
  constexpr int S0 = LOW ? 2 : 0, C0 = LOW ? 10 : 8;
  double ps = SINCOS_C[S0];
#pragma unroll
  for (int k = S0 + 1; k < 8; ++k) ps = fma(ps, r2, SINCOS_C[k]);
  const double sr = fma(ps * r2, r, r);
  double pc = SINCOS_C[C0];
#pragma unroll
  for (int k = C0 + 1; k < 17; ++k) pc = fma(pc, r2, SINCOS_C[k]);
  const double cr = fma(-pc, r2, 1.0);
  // quadrant k = q mod 4: odd k swaps sin and cos; sin changes sign for
  // k = 2, 3 and cos for k = 1, 2
  const int k = (int)((long long)q & 3);
  const bool swap = (k & 1) != 0;
  const double sgn_s = (k & 2) ? -1.0 : 1.0;
  const double sgn_c = ((k + 1) & 2) ? -1.0 : 1.0;
  *s = sgn_s * (swap ? cr : sr);
  *c = sgn_c * (swap ? sr : cr);
}
// exp(-i theta) without argument reduction, Taylor series from the term
// index S0 of sin and C0 of cos (see SINCOS_C).
template <int S0, int C0>
__device__ __forceinline__ double2 phase_series(double r) {
  const double r2 = r * r;
  double ps = SINCOS_C[S0];
#pragma unroll
  for (int k = S0 + 1; k < 8; ++k) ps = fma(ps, r2, SINCOS_C[k]);
  const double sr = fma(ps * r2, r, r);
  double pc = SINCOS_C[C0];
#pragma unroll
  for (int k = C0 + 1; k < 17; ++k) pc = fma(pc, r2, SINCOS_C[k]);
  const double cr = fma(-pc, r2, 1.0);
  return make_double2(cr, -sr);
}
// |theta| <= pi/4: sin to degree 15 and cos to degree 16, truncation error
// below 5e-17 (LOW: degree 11 and 12, below 7e-12).
template <bool LOW = false>
__device__ __forceinline__ double2 phase_small(double r) {
  return phase_series<LOW ? 3 : 1, LOW ? 11 : 9>(r);
}
// |theta| <= 0.1: sin to degree 9 and cos to degree 10, truncation error
// below 3e-19 (LOW: degree 5 and 6, below 3e-11).
template <bool LOW = false>
__device__ __forceinline__ double2 phase_tiny(double r) {
  return phase_series<LOW ? 6 : 4, LOW ? 14 : 12>(r);
}
// exp(-i theta)
template <bool LOW = false>
__device__ __forceinline__ double2 phase_rt(double theta) {
  double s, c;
  sincos_fast<LOW>(theta, &s, &c);
  return make_double2(c, -s);
}
// exp(-i theta) in real time, exp(-theta) in imaginary time
template <bool LOW = false>
__device__ __forceinline__ double2 phase_factor(double theta, int imag) {
  if (imag) return make_double2(exp(-theta), 0.0);
  return phase_rt<LOW>(theta);
}

// Potential at grid point (x, y, z).  The guide tables always hold MAX_GUIDES
// guides; unused guides have zero depth.
__device__ __forceinline__ double potential_at(const PassArgs& a, int x, int y, int z) {
  switch (a.vkind) {
    case V_TAB64: return ((const double*)a.vtab)[((long long)z * a.ny + y) * a.nx + x];
    case V_TAB32: return (double)((const float*)a.vtab)[((long long)z * a.ny + y) * a.nx + x];
    case V_CTAP: {
      const long long pl = (long long)a.nz * a.nx, o = (long long)z * a.nx + x;
      return -(a.ctapA[o] * a.ctapB[y] + a.ctapA[pl + o] * a.ctapB[a.ny + y] +
               a.ctapA[2 * pl + o] * a.ctapB[2 * a.ny + y]);
    }
    default: return 0.0;
  }
}

// Workgroup sum of NV doubles per thread; thread 0 writes them to dst.
template <int WG, int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV], double* dst, double* red) {
  constexpr int NW = (WG + 63) / 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[q] = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w * NV + threadIdx.x];
    dst[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The pass kernel.
// ---------------------------------------------------------------------------
// Ordering of LDS writes and reads between Stockham stages: a workgroup
// barrier, or -- when every row lives in one wave -- a wavefront-scope
// release/acquire fence around a wave barrier (LDS operations of one wave
// complete in order; the fences also stop the compiler from moving them).
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename S, int N, int PX, int PO, bool CONTIG, int EM = 1>
struct PassGeom {
  using PL = Plan<N>;
  static constexpr int NN = N;
  static constexpr bool CONTIGUOUS = CONTIG;
  static constexpr int PXX = PX, POO = PO;
  static constexpr int P = PX * PO;
  static constexpr int E = PL::E * EM;
  static constexpr int WG = P * N / E;
  static constexpr int LDROW = Shape<N>::ldrow();
  static constexpr int LDS = PL::S > 1 ? (CONTIG ? P * LDROW : P * N) : 1;

  // x passes whose rows fit in a wave (64 E a multiple of N, whole waves per
  // workgroup): each wave owns PPW whole rows in every stage layout, so the
  // LDS exchanges between stages stay inside the wave and need no workgroup
  // barrier.
  static constexpr int PPW = CONTIG ? (64 * E) / N : 0;
  static constexpr bool WAVELOCAL = CONTIG && (64 * E) % N == 0 && PPW >= 1 && WG % 64 == 0 && P % PPW == 0;

  // butterfly u (0 <= u < E/r) of this thread in a radix-r stage ->
  // (pencil b of the tile, butterfly i within the pencil)
  template <int r> __device__ static __forceinline__ void map(int u, int& b, int& i) {
    if constexpr (WAVELOCAL) {
      // 3 * 2^k and 5 * 2^k rows: the lane index passes through an opaque
      // move, so the (division-heavy) stage indices are recomputed per tile
      // instead of being hoisted out of the tile loop into ~100 registers
      // (the 160-point fused x pass: 265 instead of 512 registers)
      int tx = threadIdx.x;
      if constexpr (N % 3 == 0 || N % 5 == 0) asm volatile("v_mov_b32 %0, %1" : "=v"(tx) : "v"(tx));
      const int q = (tx & 63) + 64 * u;
      i = q % (N / r);
      b = (tx >> 6) * PPW + q / (N / r);
    } else if constexpr (CONTIG) {
      const int g = threadIdx.x + WG * u;
      i = g % (N / r);
      b = g / (N / r);
    } else {
      const int g = threadIdx.x + WG * u;
      b = g % P;
      i = g / P;
    }
  }
  __device__ static __forceinline__ int lidx(int b, int n) {
    // rows are swizzled (n XOR bits 3..6 of n, a permutation of every
    // supported length) so that the strided stage writes of 16 lanes fall
    // into distinct bank sets
    if constexpr (CONTIG) return b * LDROW + (n ^ ((n >> 3) & 15));
    else return n * P + b;
  }
};

// TWF: every twiddle power from the (FP64) table, rounded once to the
// register type -- the FP32-arithmetic mode's table of exactly rounded FP32
// twiddles; otherwise the powers that are not a power of two are products.
// The x passes read a stage-major copy of the table (stage_twiddles), one
// block per radix order, so that the lanes of a read take consecutive
// entries.
template <class G, bool INV, class ORD, int s, bool TWF, class C>
__device__ __forceinline__ void compute_stage(C (&v)[G::E], const double2* __restrict__ tw) {
  constexpr int N = G::NN;
  constexpr int r = ORD::r(s), p = ORD::p(s);
  constexpr int E = G::E;
#pragma unroll
  for (int u = 0; u < E / r; ++u) {
    int b, i;
    G::template map<r>(u, b, i);
    C* x = &v[u * r];
    if constexpr (p > 1) {
      // input m is multiplied by w^m, w = exp(sign 2 pi i k / (p r)) = W[k N/(p r)].
      // w^1, w^2, w^4, w^8 come from the table (exactly rounded); every other
      // power is the product of its highest power-of-two part and the rest.
      const int k = i % p;
      constexpr int step = N / (p * r);
      C w[r];
      if constexpr (TWF && G::CONTIGUOUS) {
        const double2* ts = tw + (ORD::rev ? N : 0) + (p - ORD::p(1));
#pragma unroll
        for (int m = 1; m < r; ++m) {
          w[m] = to_c<C>(ts[(m - 1) * p + k]);
          if constexpr (INV) w[m].y = -w[m].y;
        }
      } else if constexpr (TWF) {
#pragma unroll
        for (int m = 1; m < r; ++m) {
          w[m] = to_c<C>(tw[m * k * step]);
          if constexpr (INV) w[m].y = -w[m].y;
        }
      } else {
#pragma unroll
        for (int m = 1; m < r; m <<= 1) {
          w[m] = to_c<C>(tw[m * k * step]);
          if constexpr (INV) w[m].y = -w[m].y;
        }
#pragma unroll
        for (int m = 3; m < r; ++m) {
          const int hp = 1 << (31 - __builtin_clz(m));
          if (hp != m) w[m] = cmul(w[hp], w[m - hp]);
        }
      }
#pragma unroll
      for (int m = 1; m < r; ++m) x[m] = cmul(x[m], w[m]);
    }
    Bfly<r, INV>::run(x);
  }
}

// Stage-major twiddle table of one radix order: for every stage s >= 1 the
// powers W^(m k N/(p r)), m = 1..r-1, k = 0..p-1, at (p_s - p_1) + (m-1) p + k,
// so that the lanes of a read take consecutive entries.
template <class ORD, int N>
__device__ void stage_twiddles(double2* dst, const double2* __restrict__ tw) {
  constexpr int S = Plan<N>::S;
  for (int s = 1; s < S; ++s) {
    const int p = ORD::p(s), r = ORD::r(s), off = p - ORD::p(1), step = N / (p * r);
    for (int j = threadIdx.x; j < (r - 1) * p; j += blockDim.x) {
      const int m = j / p + 1, k = j % p;
      dst[off + j] = tw[m * k * step];
    }
  }
}

// Write the outputs of stage s-1 to LDS and read the inputs of stage s.
//
// X32 (complex64 storage, fused strided passes): the values cross LDS
// rounded to FP32 -- half the LDS bytes -- in two buffers that alternate
// from one exchange to the next (xp counts the exchanges), so the barrier
// after the reads is not needed: the next exchange writes the other buffer,
// and the one after it comes after a barrier that every thread reaches only
// once its reads of this buffer are done.  The FP64 exchange uses one buffer
// and a barrier after the reads.
//
// XB: 0 = FP64, one buffer; 1 = FP32, two alternating buffers; 2 = FP32, one
// buffer (a barrier after the reads, as FP64).
template <class G, class ORD, int s, int XB, class C>
__device__ __forceinline__ void exchange(C (&v)[G::E], double2* lds, int& xp) {
  using R = typename Cx<C>::R;
  constexpr int N = G::NN;
  constexpr int r1 = ORD::r(s - 1), p1 = ORD::p(s - 1);
  constexpr int r2 = ORD::r(s);
  constexpr int E = G::E;
  constexpr bool X32 = XB != 0;
  float2* l32 = (float2*)lds + (XB == 1 && (xp & 1) ? G::P * N : 0);
#pragma unroll
  for (int u = 0; u < E / r1; ++u) {
    int b, i;
    G::template map<r1>(u, b, i);
    const int k = i % p1;
    const int j = (i - k) * r1 + k;
#pragma unroll
    for (int q = 0; q < r1; ++q) {
      const C w = v[u * r1 + q];
      if constexpr (X32) l32[G::lidx(b, j + q * p1)] = make_float2((float)w.x, (float)w.y);
      else lds[G::lidx(b, j + q * p1)] = to_d(w);
    }
  }
  lds_sync<G::WAVELOCAL>();
#pragma unroll
  for (int u = 0; u < E / r2; ++u) {
    int b, i;
    G::template map<r2>(u, b, i);
#pragma unroll
    for (int m = 0; m < r2; ++m) {
      if constexpr (X32) {
        const float2 w = l32[G::lidx(b, i + m * (N / r2))];
        v[u * r2 + m] = Cx<C>::mk((R)w.x, (R)w.y);
      } else {
        v[u * r2 + m] = to_c<C>(lds[G::lidx(b, i + m * (N / r2))]);
      }
    }
  }
  if constexpr (XB == 1) ++xp;
  else lds_sync<G::WAVELOCAL>();
}

// All stages of one transform direction; v holds the inputs of stage 0 on
// entry and the outputs of the last stage on exit.
template <class G, bool INV, bool REV, int XB, bool TWF, class C>
__device__ __forceinline__ void transform(C (&v)[G::E], double2* lds, const double2* __restrict__ tw, int& xp) {
  using ORD = Order<Plan<G::NN>, REV>;
  constexpr int NS = Plan<G::NN>::S;
  static_assert(NS <= 5, "at most 5 stages");
  compute_stage<G, INV, ORD, 0, TWF>(v, tw);
  if constexpr (NS > 1) {
    exchange<G, ORD, 1, XB>(v, lds, xp);
    compute_stage<G, INV, ORD, 1, TWF>(v, tw);
  }
  if constexpr (NS > 2) {
    exchange<G, ORD, 2, XB>(v, lds, xp);
    compute_stage<G, INV, ORD, 2, TWF>(v, tw);
  }
  if constexpr (NS > 3) {
    exchange<G, ORD, 3, XB>(v, lds, xp);
    compute_stage<G, INV, ORD, 3, TWF>(v, tw);
  }
  if constexpr (NS > 4) {
    exchange<G, ORD, 4, XB>(v, lds, xp);
    compute_stage<G, INV, ORD, 4, TWF>(v, tw);
  }
}

// The pencils a thread's values belong to in the layout of a radix-r stage:
// value (u, m) is element n = i[u] + m N/r of pencil u, whose first element
// sits at offset off[u] (32-bit: fields have fewer than 2^31 points).
//   x passes:    row y = c0 of plane z = c1;
//   y, z passes: column x = c0 of outer pencil c1 (z for y passes, y for z passes).
// Ragged tiles clamp c0/c1 into range and clear ok: such lanes load, transform
// and store a copy of the last pencil of the same tile (identical inputs give
// identical values, so the duplicate stores are harmless), and reductions
// give them weight zero.  Every lane then issues the same number of memory
// operations, which lets the compiler wait for the prefetched loads alone.
template <class G, int r> struct Pen {
  static constexpr int U = G::E / r;
  int i[U], c0[U], c1[U];
  bool ok[U];
  unsigned off[U];
};

template <class G, int r>
__device__ __forceinline__ void pencils(Pen<G, r>& p, const PassArgs& a, int t) {
  const int t0 = t % a.tiles_x, t1 = t / a.tiles_x;
#pragma unroll
  for (int u = 0; u < Pen<G, r>::U; ++u) {
    int b, i;
    G::template map<r>(u, b, i);
    p.i[u] = i;
    if constexpr (G::CONTIGUOUS) {
      const int y = t0 * G::P + b;
      p.ok[u] = y < a.ny;
      p.c0[u] = p.ok[u] ? y : a.ny - 1;
      p.c1[u] = t1;
      p.off[u] = ((unsigned)t1 * (unsigned)a.ny + (unsigned)p.c0[u]) * (unsigned)a.nx;
    } else {
      const int x = t0 * G::PXX + (b % G::PXX), o = t1 * G::POO + (b / G::PXX);
      p.ok[u] = x < a.nx && o < a.nouter;
      p.c0[u] = x < a.nx ? x : a.nx - 1;
      p.c1[u] = o < a.nouter ? o : a.nouter - 1;
      p.off[u] = (unsigned)p.c1[u] * (unsigned)a.ostride + (unsigned)p.c0[u];
    }
  }
}

template <class G>
__device__ __forceinline__ unsigned elem_off(unsigned off, int n, const PassArgs& a) {
  if constexpr (G::CONTIGUOUS) return off + (unsigned)n;
  else return off + (unsigned)n * (unsigned)a.nstride;
}

// Potentials at a thread's values of an x pass (plane z).  Guide potential:
// sA = A_g(x, z) for g < MAX_GUIDES, x < N and sB = B_g(y), both in LDS.
// Tables: read from global memory.
template <class G, int r>
__device__ __forceinline__ void potentials(const PassArgs& a, const double* sA, const double* sB, const void* vtab,
                                           const Pen<G, r>& p, double (&V)[G::E]) {
  constexpr int N = G::NN, U = Pen<G, r>::U;
  if (a.vkind == V_CTAP) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int y = p.c0[u];
      const double b0 = sB[y], b1 = sB[a.ny + y], b2 = sB[2 * a.ny + y];
#pragma unroll
      for (int m = 0; m < r; ++m) {
        const int x = p.i[u] + m * (N / r);
        V[u * r + m] = -(sA[x] * b0 + sA[N + x] * b1 + sA[2 * N + x] * b2);
      }
    }
  } else if (a.vkind == V_TAB64) {
    const double* __restrict__ T = (const double*)vtab;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < r; ++m) V[u * r + m] = T[p.off[u] + p.i[u] + m * (N / r)];
  } else if (a.vkind == V_TAB32) {
    const float* __restrict__ T = (const float*)vtab;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < r; ++m) V[u * r + m] = (double)T[p.off[u] + p.i[u] + m * (N / r)];
  } else {
#pragma unroll
    for (int e = 0; e < G::E; ++e) V[e] = 0.0;
  }
}

// acc[g] += sum over the thread's values of dV/dxc_g Im(conj(lambda) psi),
// dV/dxc_g = -D_g(x, z) B_g(y); psi is read from a.aux at the same offset.
template <class G, int r, typename S, class C>
__device__ __forceinline__ void adj_accumulate(const PassArgs& a, const C (&lam)[G::E], const Pen<G, r>& p,
                                               int z, double* acc) {
  constexpr int N = G::NN, U = Pen<G, r>::U;
  const S* __restrict__ aux = (const S*)a.aux;
  const long long pl = (long long)a.nz * a.nx;
  const double* __restrict__ D = a.ctapD + (long long)z * a.nx;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!p.ok[u]) continue;
    const int y = p.c0[u];
    const double b0 = a.ctapB[y], b1 = a.ctapB[a.ny + y], b2 = a.ctapB[2 * a.ny + y];
#pragma unroll
    for (int m = 0; m < r; ++m) {
      const int x = p.i[u] + m * (N / r);
      const double2 l = to_d(lam[u * r + m]);
      const double2 w = ld2(aux + p.off[u] + x);
      const double im = l.x * w.y - l.y * w.x;  // Im(conj(lambda) psi)
      acc[0] -= D[x] * b0 * im;
      acc[1] -= D[pl + x] * b1 * im;
      acc[2] -= D[2 * pl + x] * b2 * im;
    }
  }
}

// Pass kernel.  FUSED: transform (direction INV1) - mid op - transform
// (opposite direction, reversed radix order).  Not FUSED: one transform in
// direction INV1.  Pointwise ops (potential phase, scale, reductions) exist
// for x passes (CONTIG); strided passes carry the kinetic factor and the
// kinetic-energy sum of z pencils.
//
// LEAN: only the mid op (potential phase from the guide tables in LDS, or
// the kinetic factor); no pre/post ops, no reductions, no global tables.
//
// BATCH: the launch covers a.ninst fields of the same grid, each with its own
// guide tables (a.inst); tiles are numbered instance-major.
//
// Persistent, tile t = (t % tiles_x, t / tiles_x).  x passes: workgroup w
// owns the contiguous tile range [w C, (w+1) C), C = ceil(tiles / gridDim.x),
// so it refills its guide tables only when the plane changes.  y and z
// passes: workgroup w takes tiles w, w + gridDim.x, ..., so the workgroups
// in flight together cover whole rows of consecutive outer pencils (one
// contiguous stretch of memory per plane) instead of one 128-byte segment
// each from rows far apart (measured faster for both).  Twiddles, the z
// kinetic table and (x passes) the guide tables live in LDS, so while a tile
// is transformed the only vector-memory reads in flight are the prefetch of
// the next tile's values (and of its per-pencil kinetic factors), which
// therefore overlap the arithmetic.
//
// VT (with LEAN, fused x pass): the potential comes from an FP64 table in
// global memory; each tile's values at the mid-op positions are prefetched
// with the tile, so the table read overlaps the arithmetic like the field's.
//
// SV (strided passes): tile variant; variant 2 loads each tile when it gets
// to it (no register prefetch) and, with complex64 storage, exchanges
// through one FP32 buffer (XB = 2).
//
// Variant 2 kernels are built for four waves per SIMD (at most 128 VGPRs),
// so that two of their half-size workgroups fit a CU.
//
// F32M (complex64 storage only): FP32 arithmetic in registers -- butterflies,
// twiddle products and exchanges in FP32 with every twiddle power an exactly
// rounded FP32 value of the FP64 table; the phase arguments, the phase and
// kinetic factors themselves and every reduction stay FP64, each factor
// rounded to FP32 once before it multiplies the field.
//
// Launch bounds: variant-2 tiles are built for four waves per SIMD; the lean
// fused x pass of the 3 * 2^k and 5 * 2^k rows for two (the 160-point pass
// then spills 6 registers and runs 8 % faster than at one wave per SIMD).
template <typename S, int N, int PX, int PO, bool CONTIG, bool FUSED, bool INV1, int EM, bool LEAN, bool BATCH,
          bool VT = false, int SV = 0, bool F32M = false>
__global__ void __launch_bounds__(PX * PO * N / (Plan<N>::E * EM),
                                  SV == 2 ? 4 : ((CONTIG && FUSED && LEAN && (N % 3 == 0 || N % 5 == 0)) ? 2 : 1))
pass_kernel(PassArgs a) {
  static_assert(!F32M || sizeof(S) == 8, "FP32 arithmetic only with complex64 storage");
  using C = typename std::conditional<F32M, float2, double2>::type;
  using G = PassGeom<S, N, PX, PO, CONTIG, EM>;
  using PL = Plan<N>;
  constexpr int E = G::E, WG = G::WG;
  constexpr int r0 = PL::R[0];                                     // first stage of the first transform
  constexpr int rm = PL::R[PL::S - 1];                             // last stage of the first transform
  constexpr int rl = FUSED ? PL::R[0] : PL::R[PL::S - 1];          // last stage of the last transform
  constexpr bool KZ = !CONTIG && FUSED;                            // z pass with the kinetic factor
  constexpr int UM = E / rm;
  constexpr bool LOWP = sizeof(S) == 8;                            // complex64 storage: shorter phase series

  // LDS exchanges of complex64 passes: strided variant 2 and the lean fused
  // x pass through one FP32 buffer (half the bytes); other fused strided
  // passes through two alternating FP32 buffers (the bytes of one FP64
  // buffer); everything else FP64.  The single-transform passes of the
  // 3 * 2^k-point plans exchange in FP64 in every variant: at 96
  // points FP32 rounding at their stage boundaries lost norm steadily, 2e-9
  // per step (the same with FP64 exchanges rounded to FP32 precision), where
  // the fused passes and the other plans show no such loss.
  constexpr bool C64S = !CONTIG && sizeof(S) == 8 && PL::S > 1;
  constexpr bool V2X = SV == 2 && (FUSED || N % 3 != 0);
  constexpr bool C64X = CONTIG && FUSED && LEAN && sizeof(S) == 8 && PL::S > 1 && SSF_X32;
  constexpr int XB = F32M ? ((C64S && FUSED && SV != 2 && SSF_X32) ? 1 : 2)
                          : ((C64S && V2X) || C64X ? 2 : ((C64S && FUSED && SSF_X32) ? 1 : 0));
  constexpr bool PF = SV != 2;                                     // register prefetch of the next tile
  int xpar = 0;
  __shared__ double2 lds[XB == 2 ? (G::LDS + 1) / 2 : G::LDS];
  // Power-of-two plans read twiddle powers W^t only for t < N/2 (the
  // products of lower powers are formed in registers), so half the table.
  // (FP32 arithmetic and the x passes read every power from the table, so
  // all of it: in the x passes that trades four complex products per radix-8
  // butterfly for four LDS reads, measured faster there and slower in y/z.
  // The x passes keep it stage-major, one block of N per radix order: fewer
  // bank conflicts and index registers, 3-4 % off the fused x pass.)
  constexpr bool TWF = SSF_TW_FULL || F32M || CONTIG;
  constexpr int TWN = CONTIG ? (FUSED ? 2 * N : N) : ((!TWF && N > 1 && (N & (N - 1)) == 0) ? N / 2 : N);
  __shared__ double2 s_tw[TWN];
  __shared__ double2 s_kz[KZ ? N : 1];
  // Lean fused x pass whose waves own one row each (64 E = N): the guide
  // factors B_g(y) of the wave's row are read with scalar loads, so the B
  // table takes no LDS (at N = 512 that lets a third workgroup onto a CU).
  constexpr bool BSC = CONTIG && LEAN && !VT && G::WAVELOCAL && G::PPW == 1;
  __shared__ double s_A[(CONTIG && !VT) ? MAX_GUIDES * N : 1];
  __shared__ double red[((WG + 63) / 64) * NRED_OBS];
  extern __shared__ double s_dyn[];                                // x passes: B_g(y), MAX_GUIDES * ny

  // tiles of one field; a batched launch covers ninst fields of this grid,
  // instance-major (global tile tg = instance * tpi + local tile)
  const int tpi = a.tiles_x * a.tiles_y;
  const int ntiles = tpi * (BATCH ? a.ninst : 1);
  constexpr bool ILV = !CONTIG && SSF_TILE_INTERLEAVE;
  const int chunk = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int tbeg = ILV ? (int)blockIdx.x : (int)blockIdx.x * chunk;
  const int tend = ILV ? ntiles : min(ntiles, tbeg + chunk);
  const int tstep = ILV ? (int)gridDim.x : 1;
  if (tbeg >= tend) return;                                        // whole workgroup

  const bool ctap = CONTIG && a.vkind == V_CTAP;
  const long long gplane = (long long)MAX_GUIDES * a.nz * a.nx;    // one guide table (A or D)
  // Batch descriptors are read with scalar loads (uniform index, constant
  // address space) and only when the instance changes, so the field pointers
  // stay in scalar registers and no vector-memory wait is tied to them.
  const InstDesc SSF_CONST* idesc = (const InstDesc SSF_CONST*)a.inst;
  const S* in_k = (const S*)a.in;                                  // field read by load_tile
  S* out_k = (S*)a.out;                                            // field written by the tile loop
  const void* vt_in = a.vtab;                                      // potential table of the prefetched tile
  const void* vt_k = a.vtab;                                       // potential table of the current tile
  int k_in = -1, k_out = -1;
  // tables into LDS (once per workgroup; the guide B table again when the instance changes)
  if constexpr (CONTIG) {
    stage_twiddles<Order<PL, false>, N>(s_tw, a.tw);
    if constexpr (FUSED) stage_twiddles<Order<PL, true>, N>(s_tw + N, a.tw);
  }
  for (int j = threadIdx.x; j < N; j += WG) {
    if (!CONTIG && j < TWN) s_tw[j] = a.tw[j];
    if constexpr (KZ) s_kz[j] = a.kt[2][j];
  }
  const double pre_scale = (CONTIG && (a.pre & PRE_SCALE)) ? *a.scale : 1.0;
  __syncthreads();

  // raw stage-0 inputs (storage type) and, for the z pass, the per-pencil
  // kinetic factors of the mid layout
  // In y/z passes a thread always owns pencil b = threadIdx.x % P (the
  // workgroup size is a multiple of P), so the z pass needs one per-pencil
  // kinetic factor kx(x) ky(y) per thread and tile.
  S raw[E];
  double vraw[VT ? E : 1];                                         // VT: potential at the mid-op positions
  double2 kx_n, ky_n;
  auto load_tile = [&](int tg) {
    const int k = BATCH ? __builtin_amdgcn_readfirstlane(tg / tpi) : 0;
    const int t = tg - k * tpi;
    if (BATCH && k != k_in) {
      in_k = (const S*)idesc[k].in;
      if constexpr (VT) vt_in = idesc[k].vtab;
      k_in = k;
    }
    const S* __restrict__ in = in_k;
    Pen<G, r0> p;
    pencils(p, a, t);
#pragma unroll
    for (int u = 0; u < E / r0; ++u)
#pragma unroll
      for (int m = 0; m < r0; ++m) {
        raw[u * r0 + m] = ldraw(in + elem_off<G>(p.off[u], p.i[u] + m * (N / r0), a));
      }
    if constexpr (KZ) {
      static_assert(G::WG % G::P == 0, "one pencil per thread");
      kx_n = a.kt[0][p.c0[0]];
      ky_n = a.kt[1][p.c1[0]];
    }
    if constexpr (VT) {
      Pen<G, rm> pm;
      pencils(pm, a, t);
      const double* T = (const double*)vt_in;
#pragma unroll
      for (int u = 0; u < UM; ++u)
#pragma unroll
        for (int m = 0; m < rm; ++m) vraw[u * rm + m] = ldg(T + pm.off[u] + pm.i[u] + m * (N / rm));
    }
  };
  // the adjoint and global potential tables read global memory inside the
  // tile, so those passes load each tile when they reach it
  const bool prefetch = PF && (LEAN || !(CONTIG && ((a.pre & PRE_ADJ) || (a.post & POST_ADJ) ||
                                                   (!ctap && a.vkind != V_NONE))));

  int plane = -1, binst = -1;
  if (prefetch) {
    load_tile(tbeg);
    // x passes wait for the first tile here.  Otherwise the loop head merges
    // this path (its loads the newest memory operations) with the back edge
    // (prefetched loads, then the previous tile's stores), and the counter
    // waits it derives for the prefetched registers also drain those stores
    // before every tile.  (vmcnt(0), expcnt and lgkmcnt at their maxima.)
    // The strided passes measured faster with the drain, so they keep it.
    if constexpr (CONTIG) __builtin_amdgcn_s_waitcnt(0x0F70);
  }
  for (int tg = tbeg; tg < tend; tg += tstep) {
    const int k = BATCH ? __builtin_amdgcn_readfirstlane(tg / tpi) : 0;
    const int t = tg - k * tpi;
    const int t1 = t / a.tiles_x;
    if (BATCH && k != k_out) {
      out_k = (S*)idesc[k].out;
      vt_k = idesc[k].vtab;
      k_out = k;
    }
    S* __restrict__ out = out_k;
    if constexpr (CONTIG) {
      if (ctap && (k != binst || t1 != plane)) {
        // guide tables of this plane (A_g(x, z)) and instance (B_g(y)) into LDS
        __syncthreads();
        const long long pl = (long long)a.nz * a.nx;
        const double* A = BATCH ? idesc[k].ctap : a.ctapA;
        for (int j = threadIdx.x; j < MAX_GUIDES * N; j += WG)
          s_A[j] = ldg(A + (j / N) * pl + (long long)t1 * a.nx + (j % N));
        if (!BSC && k != binst) {
          const double* B = BATCH ? idesc[k].ctap + 2 * gplane : a.ctapB;
          for (int j = threadIdx.x; j < MAX_GUIDES * a.ny; j += WG) s_dyn[j] = ldg(B + j);
        }
        __syncthreads();
        plane = t1;
        binst = k;
      }
    }
    if (!prefetch) load_tile(tg);
    C v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = Cx<C>::mk((typename Cx<C>::R)raw[e].x, (typename Cx<C>::R)raw[e].y);
    double2 kxy = make_double2(1.0, 0.0);
    if constexpr (KZ) kxy = cmul(kx_n, ky_n);
    double vcur[VT ? E : 1];
    if constexpr (VT) {
#pragma unroll
      for (int e = 0; e < E; ++e) vcur[e] = vraw[e];
    }
    if (prefetch && tg + tstep < tend) load_tile(tg + tstep);

    double acc[NRED_OBS];
#pragma unroll
    for (int q = 0; q < NRED_OBS; ++q) acc[q] = 0.0;

    // ---- pre ops on the stage-0 inputs of the first transform ----
    if constexpr (CONTIG && !LEAN) {
      if (a.pre & (PRE_ADJ | PRE_SCALE | PRE_VPHASE)) {
        Pen<G, r0> p;
        pencils(p, a, t);
        if (a.pre & PRE_ADJ) adj_accumulate<G, r0, S>(a, v, p, t1, acc);
        if (a.pre & PRE_SCALE) {
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = cscale(v[e], pre_scale);
        }
        if (a.pre & PRE_VPHASE) {
          double V[E];
          potentials<G, r0>(a, s_A, s_dyn, vt_k, p, V);
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_factor<LOWP>(V[e] * a.cpre, a.imag)));
        }
      }
    }

    transform<G, INV1, false, XB, TWF>(v, lds, s_tw, xpar);

    if constexpr (FUSED) {
      // outputs of the last stage sit at n = i + q N / rm
      if constexpr (CONTIG) {
        if (a.mid == MID_VPHASE || (!LEAN && a.mid == MID_VNORM)) {
          Pen<G, rm> p;
          pencils(p, a, t);
          double V[E];
          if constexpr (LEAN && VT) {
            // table potential, prefetched with the tile
#pragma unroll
            for (int e = 0; e < E; ++e) V[e] = vcur[e];
          } else if constexpr (LEAN) {
            // guide potential from LDS (the host selects LEAN only for it or for V = 0)
            const double SSF_CONST* Bs =
                (const double SSF_CONST*)(BATCH ? idesc[k].ctap + 2 * gplane : a.ctapB);
#pragma unroll
            for (int u = 0; u < UM; ++u) {
              double b0 = 0.0, b1 = 0.0, b2 = 0.0;
              if constexpr (BSC) {
                // one row per wave: y is uniform, the loads are scalar
                const int y = __builtin_amdgcn_readfirstlane(p.c0[u]);
                if (ctap) {
                  b0 = Bs[y];
                  b1 = Bs[a.ny + y];
                  b2 = Bs[2 * a.ny + y];
                }
              } else {
                const int y = p.c0[u];
                b0 = s_dyn[y];
                b1 = s_dyn[a.ny + y];
                b2 = s_dyn[2 * a.ny + y];
              }
#pragma unroll
              for (int m = 0; m < rm; ++m) {
                const int x = p.i[u] + m * (N / rm);
                V[u * rm + m] = ctap ? -(s_A[x] * b0 + s_A[N + x] * b1 + s_A[2 * N + x] * b2) : 0.0;
              }
            }
          }
          if constexpr (LEAN) {
            if (a.small_phase == 2) {
#pragma unroll
              for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_tiny<LOWP>(V[e] * a.cmid)));
            } else if (a.small_phase == 1) {
#pragma unroll
              for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_small<LOWP>(V[e] * a.cmid)));
            } else {
#pragma unroll
              for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_rt<LOWP>(V[e] * a.cmid)));
            }
          } else if (a.mid == MID_VNORM) {
            // end of one step (half-step factor), the norm of that step's
            // field (FP64, ragged rows weighted zero), start of the next
            potentials<G, rm>(a, s_A, s_dyn, vt_k, p, V);
#pragma unroll
            for (int u = 0; u < UM; ++u) {
              const double w = p.ok[u] ? 1.0 : 0.0;
#pragma unroll
              for (int q = 0; q < rm; ++q) {
                const int e = u * rm + q;
                const C f = to_c<C>(phase_factor<LOWP>(V[e] * a.cmid, a.imag));
                v[e] = cmul(v[e], f);
                const double2 dv = to_d(v[e]);
                acc[0] += w * (dv.x * dv.x + dv.y * dv.y);
                v[e] = cmul(v[e], f);
              }
            }
          } else {
            potentials<G, rm>(a, s_A, s_dyn, vt_k, p, V);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_factor<LOWP>(V[e] * a.cmid, a.imag)));
          }
        }
      } else {
        if (a.mid == MID_KINETIC) {
#pragma unroll
          for (int u = 0; u < UM; ++u) {
            int b, i;
            G::template map<rm>(u, b, i);
#pragma unroll
            for (int q = 0; q < rm; ++q)
              v[u * rm + q] = cmul(v[u * rm + q], to_c<C>(cmul(kxy, s_kz[i + q * (N / rm)])));
          }
        }
      }
      transform<G, !INV1, true, XB, TWF>(v, lds, s_tw, xpar);
    }

    // ---- post ops + store (outputs of the last stage at n = i + q N / rl) ----
    {
      constexpr int r = rl;
      Pen<G, r> p;
      pencils(p, a, t);
      if constexpr (LEAN) {
      } else if constexpr (CONTIG) {
        double V[E];
        if (a.post & (POST_VPHASE | POST_OBS)) potentials<G, r>(a, s_A, s_dyn, vt_k, p, V);
        if (a.post & POST_VPHASE) {
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = cmul(v[e], to_c<C>(phase_factor<LOWP>(V[e] * a.cpost, a.imag)));
        }
        if (a.post & POST_OBS) {
          const double zc = a.lo[2] + t1 * a.d[2];
          const int ilo = a.ixz ? a.ixz[2 * t1] : a.ix_lo;
          const int ihi = a.ixz ? a.ixz[2 * t1 + 1] : a.ix_hi;
#pragma unroll
          for (int u = 0; u < E / r; ++u) {
            const double w = p.ok[u] ? 1.0 : 0.0;
            const double yc = a.lo[1] + p.c0[u] * a.d[1];
#pragma unroll
            for (int q = 0; q < r; ++q) {
              const int n = p.i[u] + q * (N / r);
              const double2 sv = rounded(v[u * r + q], out);
              const double rho = w * (sv.x * sv.x + sv.y * sv.y);
              acc[0] += rho;
              acc[1] += (a.lo[0] + n * a.d[0]) * rho;
              acc[2] += yc * rho;
              acc[3] += zc * rho;
              acc[4] += n < ilo ? rho : 0.0;
              acc[6] += n > ihi ? rho : 0.0;
              acc[5] += (n >= ilo && n <= ihi) ? rho : 0.0;
              acc[7] += V[u * r + q] * rho;
            }
          }
        }
        if (a.post & POST_ADJ) {
          double2 sv[E];
#pragma unroll
          for (int e = 0; e < E; ++e) sv[e] = rounded(v[e], out);
          adj_accumulate<G, r, S>(a, sv, p, t1, acc);
        }
      } else {
        if (a.post & POST_KIN) {
          // z pencils of a field transformed along x and y: bins (c0, c1, n)
#pragma unroll
          for (int u = 0; u < E / r; ++u) {
            const double w = p.ok[u] ? 0.5 : 0.0;
            const int mx = 2 * p.c0[u] < a.nx ? p.c0[u] : p.c0[u] - a.nx;
            const int my = 2 * p.c1[u] < a.ny ? p.c1[u] : p.c1[u] - a.ny;
            const double kx = a.kfac[0] * mx, ky = a.kfac[1] * my;
#pragma unroll
            for (int q = 0; q < r; ++q) {
              const int n = p.i[u] + q * (N / r);
              const int mz = 2 * n < a.nz ? n : n - a.nz;
              const double kz = a.kfac[2] * mz;
              const double2 val = to_d(v[u * r + q]);
              acc[0] += w * (kx * kx + ky * ky + kz * kz) * (val.x * val.x + val.y * val.y);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < E / r; ++u) {
#pragma unroll
        for (int q = 0; q < r; ++q) st2(out + elem_off<G>(p.off[u], p.i[u] + q * (N / r), a), v[u * r + q]);
      }
    }

    if constexpr (!LEAN) {
      if ((a.post & (POST_OBS | POST_ADJ | POST_KIN)) || (a.pre & PRE_ADJ) || (CONTIG && a.mid == MID_VNORM))
        block_sum<WG, NRED_OBS>(acc, a.partials + (long long)tg * NRED_OBS, red);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.  `tiles` is the tile grid (tiles_x, tiles_y); the launch uses as
// many persistent workgroups as fit on the device at once (at most one per
// tile).
// ---------------------------------------------------------------------------
inline int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cus = v > 0 ? v : 1;
    else
      cus = 1;
  }
  return cus;
}

// Workgroups per compute unit of one kernel, cached per dynamic LDS size (the
// x passes hold 3 Ny doubles of guide table in dynamic LDS, so grids with
// another Ny can fit a different number of workgroups).  A full cache is
// bypassed, not evicted.
struct OccCache {
  static constexpr int SLOTS = 8;
  size_t dyn[SLOTS] = {};
  int occ[SLOTS] = {};
  int used = 0;
};

template <typename K>
int occupancy(K kernel, int wg, size_t dyn, OccCache& c) {
  for (int i = 0; i < c.used; ++i)
    if (c.dyn[i] == dyn) return c.occ[i];
  int o = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kernel, wg, dyn) != hipSuccess || o < 1) o = 1;
  if (c.used < OccCache::SLOTS) {
    c.dyn[c.used] = dyn;
    c.occ[c.used] = o;
    ++c.used;
  }
  return o;
}

template <typename K>
hipError_t launch_persistent(K kernel, int wg, size_t dyn, PassArgs a, dim3 tiles, hipStream_t st, OccCache& oc) {
  const int occ = occupancy(kernel, wg, dyn, oc);
  a.tiles_x = (int)tiles.x;
  a.tiles_y = (int)tiles.y;
  const long long ntiles = (long long)tiles.x * tiles.y * (a.ninst > 0 ? a.ninst : 1);
  long long grid = (long long)occ * device_cus();
  if (grid > ntiles) grid = ntiles;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(wg), dyn, st, a);
  return hipGetLastError();
}

// y/z passes of one tile variant (B: batched launch; F: FP32 arithmetic).
template <typename S, int N, int DT, int VAR, bool B, bool F>
hipError_t launch_strided(int kind, const PassArgs& a, dim3 tiles, hipStream_t st) {
  constexpr int SX = Shape<N>::sx(DT, VAR), SO = Shape<N>::so(DT, VAR), SM = Shape<N>::sm(DT, VAR);
  constexpr int WGS = PassGeom<S, N, SX, SO, false, SM>::WG;
  static OccCache occ[4];
  switch (kind) {
    case STRIDED_FWD:
      if (a.post == 0)
        return launch_persistent(pass_kernel<S, N, SX, SO, false, false, false, SM, true, B, false, VAR, F>, WGS, 0, a,
                                 tiles, st, occ[0]);
      if constexpr (B) return hipErrorInvalidValue;
      else
        return launch_persistent(pass_kernel<S, N, SX, SO, false, false, false, SM, false, false, false, VAR, F>, WGS,
                                 0, a, tiles, st, occ[1]);
    case STRIDED_INV:
      return launch_persistent(pass_kernel<S, N, SX, SO, false, false, true, SM, true, B, false, VAR, F>, WGS, 0, a,
                               tiles, st, occ[2]);
    case STRIDED_FUSED:
      return launch_persistent(pass_kernel<S, N, SX, SO, false, true, false, SM, true, B, false, VAR, F>, WGS, 0, a,
                               tiles, st, occ[3]);
    default:
      return hipErrorInvalidValue;
  }
}

// The lean x kernel serves the fused x pass of the steady-state steps (only
// the potential phase, real time): guide potential or none, or (VT) an FP64
// potential table read with the tile; lean y/z kernels
// serve every strided pass without a reduction.  Batched launches (B) exist
// for the passes of a real-time step: x forward with a pre phase, x inverse
// with a post phase, the lean fused x pass and the lean y/z passes.
template <typename S, int N, int DT, bool B, bool F>
hipError_t launch_pass(int kind, int variant, const PassArgs& a, dim3 tiles, hipStream_t st) {
  constexpr int CR = Shape<N>::cr();
  constexpr int WGC = PassGeom<S, N, CR, 1, true, 1>::WG;
  const size_t dync = sizeof(double) * MAX_GUIDES * (size_t)a.ny;
  static OccCache occ[5];
  using GX = PassGeom<S, N, CR, 1, true, 1>;
  // the lean kernels that keep no B_g(y) table in LDS (scalar loads, or a potential table)
  const size_t dyn_bsc = (GX::WAVELOCAL && GX::PPW == 1) ? 0 : dync;
  const bool lean_x = a.pre == 0 && a.post == 0 && !a.imag && (a.vkind == V_CTAP || a.vkind == V_NONE);
  const bool lean_t = a.pre == 0 && a.post == 0 && !a.imag && a.vkind == V_TAB64 && a.mid == MID_VPHASE;
  switch (kind) {
    case CONTIG_FWD:
      return launch_persistent(pass_kernel<S, N, CR, 1, true, false, false, 1, false, B, false, 0, F>, WGC, dync, a,
                               tiles, st, occ[0]);
    case CONTIG_INV:
      return launch_persistent(pass_kernel<S, N, CR, 1, true, false, true, 1, false, B, false, 0, F>, WGC, dync, a,
                               tiles, st, occ[1]);
    case CONTIG_FUSED:
      if (lean_x)
        return launch_persistent(pass_kernel<S, N, CR, 1, true, true, true, 1, true, B, false, 0, F>, WGC, dyn_bsc, a,
                                 tiles, st, occ[2]);
      if (lean_t)
        return launch_persistent(pass_kernel<S, N, CR, 1, true, true, true, 1, true, B, true, 0, F>, WGC, 0, a, tiles,
                                 st, occ[4]);
      if constexpr (B) return hipErrorInvalidValue;
      else
        return launch_persistent(pass_kernel<S, N, CR, 1, true, true, true, 1, false, false, false, 0, F>, WGC, dync, a,
                                 tiles, st, occ[3]);
    default:
      return variant == 2   ? launch_strided<S, N, DT, 2, B, F>(kind, a, tiles, st)
             : variant == 1 ? launch_strided<S, N, DT, 1, B, F>(kind, a, tiles, st)
                            : launch_strided<S, N, DT, 0, B, F>(kind, a, tiles, st);
  }
}

// Kernel-type index: 0 = complex64 storage with FP64 arithmetic, 1 =
// complex128, 2 = complex64 storage with FP32 arithmetic (single fields only).
template <int N>
hipError_t launch_any(int kind, int kt_index, int variant, const PassArgs& a, dim3 grid, hipStream_t st) {
  if (a.ninst > 0) {
    if (kt_index == 2) return hipErrorInvalidValue;
    return kt_index == 0 ? launch_pass<float2, N, 0, true, false>(kind, variant, a, grid, st)
                         : launch_pass<double2, N, 1, true, false>(kind, variant, a, grid, st);
  }
  if (kt_index == 2) return launch_pass<float2, N, 0, false, true>(kind, variant, a, grid, st);
  return kt_index == 0 ? launch_pass<float2, N, 0, false, false>(kind, variant, a, grid, st)
                       : launch_pass<double2, N, 1, false, false>(kind, variant, a, grid, st);
}

template <int N, int DT, int VAR>
constexpr PassShape strided_shape() {
  using S = typename std::conditional<DT == 0, float2, double2>::type;
  return PassShape{Shape<N>::sx(DT, VAR), Shape<N>::so(DT, VAR),
                   PassGeom<S, N, Shape<N>::sx(DT, VAR), Shape<N>::so(DT, VAR), false, Shape<N>::sm(DT, VAR)>::WG};
}

template <int N>
constexpr KernelSet make_kernel_set() {
  return KernelSet{
      N,
      {PassShape{Shape<N>::cr(), 1, PassGeom<float2, N, Shape<N>::cr(), 1, true, 1>::WG},
       PassShape{Shape<N>::cr(), 1, PassGeom<double2, N, Shape<N>::cr(), 1, true, 1>::WG}},
      {{strided_shape<N, 0, 0>(), strided_shape<N, 0, 1>(), strided_shape<N, 0, 2>()},
       {strided_shape<N, 1, 0>(), strided_shape<N, 1, 1>(), strided_shape<N, 1, 2>()}},
      &launch_any<N>};
}

}  // namespace ssf
