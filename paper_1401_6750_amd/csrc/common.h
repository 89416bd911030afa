// Internal definitions shared by the HIP kernels and the host runtime.
//
// Device data layout (one lattice, one right-hand side):
//   spinor half field, parity p:  [chunk][site]   16-byte chunks, site = even-odd
//                                                index within the parity
//       FP64: 12 chunks of 1 complex, FP32: 6 chunks of 2 complex,
//       bf16 / fp16: 3 chunks of 4 complex.  Component k = 3 * spin + colour.
//   gauge field:                  [mu][parity][chunk][site]  16-byte chunks in rows
//                                                of the padded half volume, so a wave's
//                                                link loads are contiguous like its
//                                                spinor loads.  FP64: 9 chunks of 1
//                                                complex, FP32: 5 of 2 (one padding),
//                                                bf16 / fp16: 3 of 4 (three padding)
//   loop accumulators (FP64):     [component q][full e/o site = parity * Vh + site]
//
// A "batch" interleaves several lattices and right-hand sides: rhs r of slot i
// starts at site offset fo_i + r * Vh_i of every batch field.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dl {

enum Prec : int { P64 = 0, P32 = 1, PB16 = 2, PH16 = 3 };

// Tag types of the two 16-bit storage formats.
struct bf16s {};
struct f16s {};

template <class S> struct Traits;
template <> struct Traits<double> { using R = double; static constexpr int NC = 12; static constexpr int prec = P64; };
template <> struct Traits<float> { using R = float; static constexpr int NC = 6; static constexpr int prec = P32; };
template <> struct Traits<bf16s> { using R = float; static constexpr int NC = 3; static constexpr int prec = PB16; };
template <> struct Traits<f16s> { using R = float; static constexpr int NC = 3; static constexpr int prec = PH16; };

inline int chunks_of(int prec) { return prec == P64 ? 12 : (prec == P32 ? 6 : 3); }

constexpr int TILE = 64;        // sites per unit (one wavefront)

// ---------------------------------------------------------------------------
// complex numbers in the compute precision
// ---------------------------------------------------------------------------
template <class R> struct cx { R re, im; };

// Products are written as explicit fused multiply-adds: without reassociation
// the compiler cannot turn  a += b*c - d*e  into two FMAs on its own.
__device__ inline float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class R> __host__ __device__ inline cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <class R> __device__ inline cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ inline cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
  return {fmadd(a.re, b.re, -(a.im * b.im)), fmadd(a.re, b.im, a.im * b.re)};
}
template <class R> __device__ inline cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> __device__ inline cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <class R> __device__ inline cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <class R> __device__ inline cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
// a += conj(b) * c
template <class R> __device__ inline void cjmac(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fmadd(b.im, c.im, fmadd(b.re, c.re, a.re));
  a.im = fmadd(-b.im, c.re, fmadd(b.re, c.im, a.im));
}
// a += b * c
template <class R> __device__ inline void cmac(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fmadd(-b.im, c.im, fmadd(b.re, c.re, a.re));
  a.im = fmadd(b.im, c.re, fmadd(b.re, c.im, a.im));
}

// ---------------------------------------------------------------------------
// 16-bit conversions (round to nearest even)
// ---------------------------------------------------------------------------
__device__ inline float f16_to_f(uint32_t h) {
  _Float16 v = __builtin_bit_cast(_Float16, (uint16_t)h);
  return (float)v;
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

template <class S> __device__ inline cx<float> unpack2(uint32_t w);
template <> __device__ inline cx<float> unpack2<bf16s>(uint32_t w) {
  return {__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
}
template <> __device__ inline cx<float> unpack2<f16s>(uint32_t w) { return {f16_to_f(w & 0xffffu), f16_to_f(w >> 16)}; }
// (re, im) -> one dword with two 16-bit values, hardware round-to-nearest-even
// conversion of both halves in one instruction
template <class S> __device__ inline uint32_t pack2(cx<float> v);
template <> __device__ inline uint32_t pack2<bf16s>(cx<float> v) {
  const f32x2_t x = {v.re, v.im};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2_t));
}
template <> __device__ inline uint32_t pack2<f16s>(cx<float> v) {
  const f32x2_t x = {v.re, v.im};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, f16x2_t));
}

// ---------------------------------------------------------------------------
// packed 16-bit colour products
// ---------------------------------------------------------------------------
// 16-bit storage: FP32 dot product of two packed (re, im) pairs, c + a.lo b.lo
// + a.hi b.hi.  The products of 16-bit values are exact in FP32, so this is
// FP32 arithmetic on the stored values without unpacking them.
template <class S> __device__ inline float dot2(uint32_t a, uint32_t b, float c);
template <> __device__ inline float dot2<bf16s>(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}
template <> __device__ inline float dot2<f16s>(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, a), __builtin_bit_cast(f16x2_t, b), c, false);
}
// First product of a chain: the three-operand form with an inline zero
// accumulator (the two-operand form accumulates into its destination and
// would need the register cleared first).  The compiler cannot see that the
// asm holds a dot2, whose result a different vector instruction (the
// accumulating two-operand form included) may read only after three wait
// states, so the asm supplies them.
template <class S> __device__ inline float dot2_first(uint32_t a, uint32_t b);
template <> __device__ inline float dot2_first<bf16s>(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_bf16 %0, %1, %2, 0\n\ts_nop 2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
template <> __device__ inline float dot2_first<f16s>(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0\n\ts_nop 2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// Six chained dot2 products in one asm block, x = sum_k a_k . b_k, the first
// three with the input modifiers (L1, H1) on a_k, the last three with (L2, H2):
// neg_lo / neg_hi flip the sign of the low / high half of a_k, the same
// products as a_k with those sign bits XOR-ed, without the XOR.  Inside the
// block each product takes the previous sum as its accumulator, which the
// hardware forwards between dot2 instructions of one opcode; the block ends
// with three wait states, because a dot2 result must not be read sooner by a
// different vector instruction and the compiler cannot see what the block
// holds.
#define DL_NEG00 ""
#define DL_NEG10 " neg_lo:[1,0,0]"
#define DL_NEG01 " neg_hi:[1,0,0]"
#define DL_NEG11 " neg_lo:[1,0,0] neg_hi:[1,0,0]"
template <class S, int L1, int H1, int L2, int H2> struct Chain6;
#define DL_CHAIN6(S, INSTR, L1, H1, L2, H2)                                                                  \
  template <> struct Chain6<S, L1, H1, L2, H2> {                                                             \
    __device__ static inline float run(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,      \
                                       uint32_t a5, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3,      \
                                       uint32_t b4, uint32_t b5) {                                           \
      float x;                                                                                               \
      asm(INSTR " %0, %1, %7, 0" DL_NEG##L1##H1 "\n\t"                                                       \
          INSTR " %0, %2, %8, %0" DL_NEG##L1##H1 "\n\t"                                                      \
          INSTR " %0, %3, %9, %0" DL_NEG##L1##H1 "\n\t"                                                      \
          INSTR " %0, %4, %10, %0" DL_NEG##L2##H2 "\n\t"                                                     \
          INSTR " %0, %5, %11, %0" DL_NEG##L2##H2 "\n\t"                                                     \
          INSTR " %0, %6, %12, %0" DL_NEG##L2##H2 "\n\t"                                                     \
          "s_nop 2"                                                                                          \
          : "=&v"(x)                                                                                         \
          : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(b0), "v"(b1), "v"(b2), "v"(b3),        \
            "v"(b4), "v"(b5));                                                                               \
      return x;                                                                                              \
    }                                                                                                        \
  };
#define DL_CHAIN6_H2(S, INSTR, L1, H1, L2) DL_CHAIN6(S, INSTR, L1, H1, L2, 0) DL_CHAIN6(S, INSTR, L1, H1, L2, 1)
#define DL_CHAIN6_L2(S, INSTR, L1, H1) DL_CHAIN6_H2(S, INSTR, L1, H1, 0) DL_CHAIN6_H2(S, INSTR, L1, H1, 1)
#define DL_CHAIN6_H1(S, INSTR, L1) DL_CHAIN6_L2(S, INSTR, L1, 0) DL_CHAIN6_L2(S, INSTR, L1, 1)
#define DL_CHAIN6_ALL(S, INSTR) DL_CHAIN6_H1(S, INSTR, 0) DL_CHAIN6_H1(S, INSTR, 1)
DL_CHAIN6_ALL(bf16s, "v_dot2_f32_bf16")
DL_CHAIN6_ALL(f16s, "v_dot2_f32_f16")
// Two chained products, x = a0 . b0 + a1 . b1, modifiers (L0, H0) on a0 and
// (L1, H1) on a1, the same wait states at the end.
template <class S, int L0, int H0, int L1, int H1> struct Chain2;
#define DL_CHAIN2(S, INSTR, L0, H0, L1, H1)                                                                  \
  template <> struct Chain2<S, L0, H0, L1, H1> {                                                             \
    __device__ static inline float run(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {                 \
      float x;                                                                                               \
      asm(INSTR " %0, %1, %3, 0" DL_NEG##L0##H0 "\n\t"                                                        \
          INSTR " %0, %2, %4, %0" DL_NEG##L1##H1 "\n\t"                                                       \
          "s_nop 2"                                                                                          \
          : "=&v"(x)                                                                                         \
          : "v"(a0), "v"(a1), "v"(b0), "v"(b1));                                                             \
      return x;                                                                                              \
    }                                                                                                        \
  };
DL_CHAIN2(bf16s, "v_dot2_f32_bf16", 0, 1, 1, 0)
DL_CHAIN2(bf16s, "v_dot2_f32_bf16", 0, 0, 1, 1)
DL_CHAIN2(f16s, "v_dot2_f32_f16", 0, 1, 1, 0)
DL_CHAIN2(f16s, "v_dot2_f32_f16", 0, 0, 1, 1)
#undef DL_CHAIN2
#undef DL_CHAIN6_ALL
#undef DL_CHAIN6_H1
#undef DL_CHAIN6_L2
#undef DL_CHAIN6_H2
#undef DL_CHAIN6
#undef DL_NEG00
#undef DL_NEG10
#undef DL_NEG01
#undef DL_NEG11

__device__ inline uint32_t swap16(uint32_t w) { return (w >> 16) | (w << 16); }

// Colour-product coefficients of one link for the packed path: row a of
// M = U (forward) or U^dag (backward) contributes Re += dot2(cr[3a+b], psi_b),
// Im += dot2(ci[3a+b], psi_b), with
//   forward:  cr = (Re U_ab, -Im U_ab), ci = (Im U_ab, Re U_ab)
//   backward: cr = (Re U_ba,  Im U_ba), ci = (-Im U_ba, Re U_ba).
// `neg` flips the sign of every entry (a -1 boundary factor of the link).
template <bool FWD>
__device__ inline void link_coef16(const uint32_t (&e)[9], bool neg, uint32_t (&cr)[9], uint32_t (&ci)[9]) {
  const uint32_t m = neg ? 0x80008000u : 0u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (FWD) {
        const uint32_t w = e[3 * a + b] ^ m;
        cr[3 * a + b] = w ^ 0x80000000u;
        ci[3 * a + b] = swap16(w);
      } else {
        const uint32_t w = e[3 * b + a] ^ m;
        cr[3 * a + b] = w;
        ci[3 * a + b] = swap16(w) ^ 0x00008000u;
      }
    }
}

// out[3 s + a] = sum_b M_ab psi[3 s + b] for the four spins, psi packed words.
template <class S>
__device__ inline void colour_mul16(const uint32_t (&cr)[9], const uint32_t (&ci)[9], const uint32_t (&v)[12],
                                    cx<float> (&out)[12]) {
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float re = dot2_first<S>(cr[3 * a], v[3 * s4]);
      re = dot2<S>(cr[3 * a + 1], v[3 * s4 + 1], re);
      re = dot2<S>(cr[3 * a + 2], v[3 * s4 + 2], re);
      float im = dot2_first<S>(ci[3 * a], v[3 * s4]);
      im = dot2<S>(ci[3 * a + 1], v[3 * s4 + 1], im);
      im = dot2<S>(ci[3 * a + 2], v[3 * s4 + 2], im);
      out[3 * s4 + a] = mk<float>(re, im);
    }
}

// ---------------------------------------------------------------------------
// spinor loads / stores: base points at chunk 0 of one (rhs, parity) half
// field; stride is Vh (chunks between consecutive chunk rows).
// ---------------------------------------------------------------------------
template <class S> struct Spinor {
  using R = typename Traits<S>::R;
  cx<R> c[12];
};

// Element i (per lane) of an array of 16-byte values in device memory that
// starts at `row` (wave-uniform): a scalar base plus a 32-bit lane offset, the
// form the vector memory instructions take directly, so no 64-bit address is
// formed and held per lane.  Every array here has fewer than 2^28 elements per
// row.  The access goes through a global-address-space pointer: a pointer read
// from a descriptor (the links of a slot) is otherwise generic, and generic
// (flat) loads make every later wait for any load also wait for all of them.
// (The access is made on a native vector type: copying the HIP vector struct
// would go through a generic reference again.)
template <class T> struct Vec16;
template <> struct Vec16<uint4> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<float4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double2> { typedef double type __attribute__((ext_vector_type(2))); };
#define DL_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ inline T at16(const void* row, long long i) {
  using V = typename Vec16<T>::type;
  const V v = *(const V DL_GLOBAL*)((const char*)row + ((uint32_t)i << 4));
  return __builtin_bit_cast(T, v);
}
template <class T>
__device__ inline void st16(void* row, long long i, const T& x) {
  using V = typename Vec16<T>::type;
  *(V DL_GLOBAL*)((char*)row + ((uint32_t)i << 4)) = __builtin_bit_cast(V, x);
}
#undef DL_GLOBAL
// Row k of a family of rows `stride` elements apart.
__device__ inline const void* row16(const void* base, long long k, long long stride) {
  return (const char*)base + k * stride * 16;
}
__device__ inline void* row16(void* base, long long k, long long stride) {
  return (char*)base + k * stride * 16;
}

template <class S>
__device__ inline void load_spinor(const void* base, long stride, long s, cx<typename Traits<S>::R> (&v)[12]);

template <>
__device__ inline void load_spinor<double>(const void* base, long stride, long s, cx<double> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 w = at16<double2>(row16(base, k, stride), s);
    v[k] = {w.x, w.y};
  }
}
template <>
__device__ inline void load_spinor<float>(const void* base, long stride, long s, cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 w = at16<float4>(row16(base, k, stride), s);
    v[2 * k] = {w.x, w.y};
    v[2 * k + 1] = {w.z, w.w};
  }
}
template <class S16>
__device__ inline void load_spinor16(const void* base, long stride, long s, cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 w = at16<uint4>(row16(base, k, stride), s);
    v[4 * k + 0] = unpack2<S16>(w.x);
    v[4 * k + 1] = unpack2<S16>(w.y);
    v[4 * k + 2] = unpack2<S16>(w.z);
    v[4 * k + 3] = unpack2<S16>(w.w);
  }
}
template <>
__device__ inline void load_spinor<bf16s>(const void* base, long stride, long s, cx<float> (&v)[12]) {
  load_spinor16<bf16s>(base, stride, s, v);
}
template <>
__device__ inline void load_spinor<f16s>(const void* base, long stride, long s, cx<float> (&v)[12]) {
  load_spinor16<f16s>(base, stride, s, v);
}

template <class S>
__device__ inline void store_spinor(void* base, long stride, long s, const cx<typename Traits<S>::R> (&v)[12]);

template <>
__device__ inline void store_spinor<double>(void* base, long stride, long s, const cx<double> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) st16<double2>(row16(base, k, stride), s, make_double2(v[k].re, v[k].im));
}
template <>
__device__ inline void store_spinor<float>(void* base, long stride, long s, const cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k)
    st16<float4>(row16(base, k, stride), s, make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
}
template <class S16>
__device__ inline void store_spinor16(void* base, long stride, long s, const cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint4 w;
    w.x = pack2<S16>(v[4 * k + 0]);
    w.y = pack2<S16>(v[4 * k + 1]);
    w.z = pack2<S16>(v[4 * k + 2]);
    w.w = pack2<S16>(v[4 * k + 3]);
    st16<uint4>(row16(base, k, stride), s, w);
  }
}
template <>
__device__ inline void store_spinor<bf16s>(void* base, long stride, long s, const cx<float> (&v)[12]) {
  store_spinor16<bf16s>(base, stride, s, v);
}
template <>
__device__ inline void store_spinor<f16s>(void* base, long stride, long s, const cx<float> (&v)[12]) {
  store_spinor16<f16s>(base, stride, s, v);
}

// Round a spinor held in the compute precision to the storage precision.
template <class S> __device__ inline void quantize(cx<typename Traits<S>::R> (&)[12]) {}
template <class S16> __device__ inline void quantize16(cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = unpack2<S16>(pack2<S16>(v[k]));
}
template <> __device__ inline void quantize<bf16s>(cx<float> (&v)[12]) { quantize16<bf16s>(v); }
template <> __device__ inline void quantize<f16s>(cx<float> (&v)[12]) { quantize16<f16s>(v); }

// |v|^2 summed in FP64
template <class R> __device__ inline double norm2(const cx<R> (&v)[12]) {
  double n = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) n += (double)v[k].re * (double)v[k].re + (double)v[k].im * (double)v[k].im;
  return n;
}

// Address of (rhs field) chunk row 0 for site offset `off` (in sites) of a
// batch field with NC chunks per site.
template <class S> __device__ inline const void* field_at(const void* base, long long off) {
  return (const char*)base + off * (long long)Traits<S>::NC * 16;
}
template <class S> __device__ inline void* field_at(void* base, long long off) {
  return (char*)base + off * (long long)Traits<S>::NC * 16;
}

// ---------------------------------------------------------------------------
// gauge links: the 9 complex entries of each 3x3 matrix, row-major, padded to
// whole 16-byte chunks (FP64 9 chunks, FP32 5, 16-bit 3); chunk k of the link
// (mu, parity, site) sits at row (mu * 2 + parity) * nchunks + k, column site,
// rows Vp apart, so the lanes of a wave load one chunk of their 64 links as
// 1 KiB contiguous.
// ---------------------------------------------------------------------------
inline int link_chunks(int prec) { return prec == P64 ? 9 : (prec == P32 ? 5 : 3); }
// Rows of Vp chunks per precision: 8 (mu, parity) x link_chunks; 16-bit links
// add, per parity, one row with the ninth entries of the four links leaving a
// site forward, U_mu(x) (row 24 + parity, word mu), and one with those of the
// four links reaching it from behind, U_mu(x - mu) (row 26 + parity), so the
// eight hops of a site fetch their ninth entries with two loads instead of
// eight (copies; the entries also stay in the links' own chunk rows).
constexpr int LINK_ROW_NINTH = 24;
constexpr int LINK_ROW_NINTH_BWD = 26;
// 16-bit links, site-centred copies of rows 0 and 1 only (6 words a link) for
// the hopping kernel, which rebuilds row 2 (SU(3)): per parity 12 rows from
// LINK_ROW_R12 + 12 parity, the first 6 for the links leaving the site,
// U_mu(x), the last 6 for those reaching it, U_mu(x - mu); two directions
// share three rows, word j = 6 (mu & 1) + entry at row 3 (mu >> 1) + j / 4,
// component j % 4.
constexpr int LINK_ROW_R12 = 28;
// Bits of a lattice's two-row flag, set at upload when every link's row 2
// equals conj(row 0 x row 1) (a special unitary matrix) to 1e-6 (16-bit
// hops) or 1e-7 (FP32 hops, which then read the first three of a link's five
// chunks)
constexpr int TWO_ROW_16 = 1;
constexpr int TWO_ROW_32 = 2;
inline int link_rows(int prec) { return 8 * link_chunks(prec) + ((prec == PB16 || prec == PH16) ? 28 : 0); }

template <class S>
__device__ inline void load_link(const void* g, long vh, int mu, int par, long s, cx<typename Traits<S>::R> (&u)[9]);

template <>
__device__ inline void load_link<double>(const void* g, long vh, int mu, int par, long s, cx<double> (&u)[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const double2 w = at16<double2>(row16(g, (mu * 2 + par) * 9 + e, vh), s);
    u[e] = {w.x, w.y};
  }
}
template <>
__device__ inline void load_link<float>(const void* g, long vh, int mu, int par, long s, cx<float> (&u)[9]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 w = at16<float4>(row16(g, (mu * 2 + par) * 5 + k, vh), s);
    u[2 * k] = {w.x, w.y};
    u[2 * k + 1] = {w.z, w.w};
  }
  const float4 w = at16<float4>(row16(g, (mu * 2 + par) * 5 + 4, vh), s);
  u[8] = {w.x, w.y};
}
// Row 2 of a special unitary matrix from rows 0 and 1: the rows are
// orthonormal and the determinant is one, so u2_k = conj(u0_i u1_j - u0_j u1_i)
// for (i, j, k) cyclic.
template <class R>
__device__ inline void su3_row2(cx<R> (&u)[9]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const cx<R> a = u[i], b = u[3 + j], c = u[j], e = u[3 + i];
    const R re = fmadd(a.re, b.re, fmadd(-a.im, b.im, fmadd(-c.re, e.re, c.im * e.im)));
    const R im = fmadd(a.re, b.im, fmadd(a.im, b.re, fmadd(-c.re, e.im, -(c.im * e.re))));
    u[6 + k] = mk<R>(re, -im);
  }
}
// FP32 link from its first three chunks (entries 0-5: rows 0 and 1), row 2
// rebuilt (links special unitary, TWO_ROW_32)
__device__ inline void load_link_2row(const void* g, long vh, int mu, int par, long s, cx<float> (&u)[9]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float4 w = at16<float4>(row16(g, (mu * 2 + par) * 5 + k, vh), s);
    u[2 * k] = {w.x, w.y};
    u[2 * k + 1] = {w.z, w.w};
  }
  su3_row2(u);
}
template <class R>
__device__ inline void load_link_2row(const void*, long, int, int, long, cx<R> (&)[9]) {
  static_assert(sizeof(R) == 0, "two-row links: FP32 unpacked hops only");
}

template <class S16>
__device__ inline void load_link16(const void* g, long vh, int mu, int par, long s, cx<float> (&u)[9]) {
  const long long r0 = (mu * 2 + par) * 3;
  const uint4 a = at16<uint4>(row16(g, r0, vh), s), b = at16<uint4>(row16(g, r0 + 1, vh), s),
              c = at16<uint4>(row16(g, r0 + 2, vh), s);
  u[0] = unpack2<S16>(a.x); u[1] = unpack2<S16>(a.y); u[2] = unpack2<S16>(a.z); u[3] = unpack2<S16>(a.w);
  u[4] = unpack2<S16>(b.x); u[5] = unpack2<S16>(b.y); u[6] = unpack2<S16>(b.z); u[7] = unpack2<S16>(b.w);
  u[8] = unpack2<S16>(c.x);
}
template <>
__device__ inline void load_link<bf16s>(const void* g, long vh, int mu, int par, long s, cx<float> (&u)[9]) {
  load_link16<bf16s>(g, vh, mu, par, s, u);
}
template <>
__device__ inline void load_link<f16s>(const void* g, long vh, int mu, int par, long s, cx<float> (&u)[9]) {
  load_link16<f16s>(g, vh, mu, par, s, u);
}

// ---------------------------------------------------------------------------
// batch slots
// ---------------------------------------------------------------------------
// Unit kinds: UK_RHS (one tile x one rhs), UK_SITE (one tile x one parity),
// UK_DERIV (one tile x parity x direction), UK_GRP2 / UK_GRP4 (one tile x 2 / 4
// rhs: the hopping kernel runs that many right-hand sides per wavefront).
enum UnitKind : int { UK_RHS = 0, UK_SITE = 1, UK_DERIV = 2, UK_GRP2 = 3, UK_GRP4 = 4, UK_BLK = 5, UK_COUNT = 6 };
// Right-hand sides per wavefront in the hopping kernel, per storage type
// (1, 2 or 4).  Sharing a wave shares the link loads, the link-word
// preparation and the index arithmetic, at the cost of registers.  Measured
// on gfx950 at 24^3x48: bf16 8.2 ms per 525-rhs launch with two against 8.9 ms
// with one (the 16-bit kernels keep spinors packed, so two fit in ~110
// registers); FP32 HP solves +10 % and the FP64 single-rhs path +27 % with two.
#ifndef DL_RPW16
#define DL_RPW16 2
#endif
#ifndef DL_RPW32
#define DL_RPW32 2
#endif
#ifndef DL_RPW64
#define DL_RPW64 2
#endif
template <class S> constexpr int rhs_per_wave() {
  return Traits<S>::NC == 3 ? DL_RPW16 : (Traits<S>::NC == 6 ? DL_RPW32 : DL_RPW64);
}
inline int rhs_per_wave_prec(int prec) {
  return (prec == PB16 || prec == PH16) ? DL_RPW16 : (prec == P32 ? DL_RPW32 : DL_RPW64);
}
constexpr int unit_kind_for_group(int g) { return g == 1 ? UK_RHS : (g == 2 ? UK_GRP2 : UK_GRP4); }
static_assert((DL_RPW16 == 1 || DL_RPW16 == 2 || DL_RPW16 == 4) && (DL_RPW32 == 1 || DL_RPW32 == 2 || DL_RPW32 == 4) &&
                  (DL_RPW64 == 1 || DL_RPW64 == 2 || DL_RPW64 == 4),
              "right-hand sides per wave: 1, 2 or 4");

// Site stride of every per-parity device array (spinor chunk rows, link
// chunk rows, accumulator rows): Vh rounded up to an odd number of 64-site
// tiles.  Rows then start an odd number of KiB apart; with the unpadded Vh
// (2^12 * 81 at 24^3x48, 2^15 at 16^3x32) the rows of one site sit at
// multiples of 64 KiB and compete for the same L2 sets.
__host__ __device__ inline long long pad_half(long long vh) {
  long long nt = (vh + TILE - 1) / TILE;
  if (!(nt & 1)) ++nt;
  return nt * TILE;
}

struct SlotDesc {
  int X, Y, Z, T;
  int Xh, Vh, ntile, nrhs;
  int Vp;                  // pad_half(Vh): row stride of fields, links, accumulators
  int tblk;                // time slices per block of the hopping kernel's tile order
  int bby, bbz, bseg;      // LDS-staged hop (16-bit storage, option): x-rows per block in y and z,
                           // time slices per workgroup (1); bby = 0: the slot uses the tile kernel
  int ubeg[UK_COUNT];      // first unit of this slot per UnitKind
  int rhs_begin;           // global index of this slot's rhs 0
  long long fo;            // site offset of rhs 0 in every batch field
  double bc;               // time-boundary factor
  int two_row;             // TWO_ROW_* bits: the hops of that storage class read rows 0 and 1 of
                           // the links and rebuild row 2 (links special unitary to its precision)
  const void* gauge[4];    // gauge field per precision
  const void* clv64;       // clover site matrices (FP64 class), or null: no clover term
  const void* clv32;       // clover site matrices (FP32 class, all other tiers), or null
  double* acc;             // accumulator set of this slot (contractions), or null
  uint64_t seed;           // noise
  long long src0;          // source index of rhs 0 (time dilution: of the job's first vector)
  int noise;               // DL_NOISE_*
  int acc_ops;             // DL_OPS_* of the accumulator
  const double* src_user;  // caller sources of rhs 0 (complex128 [V][12] per rhs; time dilution:
                           // the job's first vector), or null
  double* sol_user;        // caller solution array of rhs 0, or null
  void* gsave;             // guess buffer of rhs 0 to store the odd solution in, or null
  const void* gload;       // guess buffer of rhs 0 to start the odd solution from, or null
  int gprec;               // storage precision of gload
  int tdil;                // time dilution: components per noise vector (<= 1: none)
  int tclen;               // time dilution: noise vectors of the job (entries per component)
  int tentry;              // job entry of rhs 0 (entries component-major): rhs r belongs to
                           // component (tentry + r) / tclen, the slices t mod tdil == component
  int job;                 // index of the job in its call
};

// Time-dilution component of rhs r of a slot.
__host__ __device__ inline int tdil_comp(const SlotDesc& sd, int r) {
  return sd.tdil > 1 ? (sd.tentry + r) / sd.tclen : 0;
}

// Noise vector of rhs r, counted from src0 / src_user: a time-diluted slot
// may span components, its rhs r is vector (tentry + r) mod tclen of the job.
__host__ __device__ inline int src_vector(const SlotDesc& sd, int r) {
  return sd.tdil > 1 ? (sd.tentry + r) % sd.tclen : r;
}

// Per-slot site-diagonal spin coefficients of one dslash-type launch:
//   res = e (.) H(d (.) in) + f (.) y,  out = g (.) res   (per-spin complex factors)
struct Coef {
  double d[4][2], e[4][2], f[4][2], g[4][2];
  // the same factors rounded to FP32 on the host (the FP32 and 16-bit kernels
  // read these, so the values stay in scalar registers)
  float d32[4][2], e32[4][2], f32[4][2], g32[4][2];
  // clover lattices: site matrix (CloverKind) that each factor applies before
  // its per-spin constant, -1 for none: d, e, f, g
  int m[4];
};

// ---------------------------------------------------------------------------
// clover term: per-site matrices that replace the per-spin twist factors.
// The clover term commutes with gamma_5, so every matrix here is two 6 x 6
// blocks per site (spins 0, 1 and spins 2, 3; component 3 spin + colour).
// Storage per lattice and class (FP64 for the FP64 tier, FP32 otherwise):
// kind k, parity p, entry e = 36 b + 6 i + j of block b, row i, column j in
// chunk rows Vp sites long: FP64 72 rows of one complex, FP32 36 rows of two
// complex (entries e, e + 1), row (k * 2 + p) * rows + chunk.
// ---------------------------------------------------------------------------
enum CloverKind : int {
  CLV_AINV = 0,    // A(mu)^-1, A = 1 + C + 2 i kappa mu gamma_5
  CLV_AINV_M = 1,  // A(-mu)^-1
  CLV_A = 2,       // A(mu)
  CLV_A_M = 3,     // A(-mu)
  CLV_AC = 4,      // 1 + C
  CLV_KINDS = 5
};
inline int clover_rows(int prec) { return prec == P64 ? 72 : 36; }

// out[k] = sum_j M(x)[k][j] in[j] for the G right-hand sides of a wave that are
// active; M is kind `kind` of parity `par` at site s (FP64 and FP32 storage).
template <int G>
__device__ inline void site_matvec(const void* m, int kind, int par, long vp, long s, const cx<double> (&in)[G][12],
                                   cx<double> (&out)[G][12], const bool (&act)[G]) {
  const long long r0 = (long long)(kind * 2 + par) * 72;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      cx<double> row[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double2 w = at16<double2>(row16(m, r0 + 36 * b + 6 * i + j, vp), s);
        row[j] = mk<double>(w.x, w.y);
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        if (!act[r]) continue;
        cx<double> a = mk<double>(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 6; ++j) a = a + row[j] * in[r][6 * b + j];
        out[r][6 * b + i] = a;
      }
    }
}

template <int G>
__device__ inline void site_matvec(const void* m, int kind, int par, long vp, long s, const cx<float> (&in)[G][12],
                                   cx<float> (&out)[G][12], const bool (&act)[G]) {
  const long long r0 = (long long)(kind * 2 + par) * 36;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      cx<float> row[6];
#pragma unroll
      for (int j = 0; j < 6; j += 2) {
        const float4 w = at16<float4>(row16(m, r0 + (36 * b + 6 * i + j) / 2, vp), s);
        row[j] = mk<float>(w.x, w.y);
        row[j + 1] = mk<float>(w.z, w.w);
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        if (!act[r]) continue;
        cx<float> a = mk<float>(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 6; ++j) a = a + row[j] * in[r][6 * b + j];
        out[r][6 * b + i] = a;
      }
    }
}

// Hardware dispatches workgroup b to XCD (b mod 8); renumber so that each XCD
// runs one contiguous range of logical workgroups (neighbouring tiles and the
// right-hand sides of one tile then share that XCD's L2).
__device__ inline int xcd_logical_block() {
  int nb = gridDim.x, b = blockIdx.x;
  int q = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
  return x * q + (x < rem ? x : rem) + k;
}

// Unit handled by the calling wavefront (wave-uniform, so the slot and tile
// arithmetic that follows runs on the scalar unit).
__device__ inline int wave_unit() {
  return __builtin_amdgcn_readfirstlane(xcd_logical_block() * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6));
}

// Order in which the hopping kernel visits the tiles of a slot.  Tiles are
// taken in blocks of tb = sd.tblk time slices; inside a block the tb tiles at
// the same place of successive slices are consecutive.  A tile's -t / +t
// neighbours are then a few tiles away instead of a whole time slice
// (Xh*Y*Z/64 tiles), so they are still in L2 when read, while the z
// neighbours move only tb times further.  tb is tuned with the slot size;
// tb <= 1, or a lattice without whole tiles per time slice, keeps the
// lexicographic order.  The reductions index the physical tile, so the order
// never changes results.
constexpr int TBLK_DEFAULT = 4;
__device__ inline int tile_of(const SlotDesc& sd, int lt) {
  const int tb = sd.tblk;
  const int slice = sd.Xh * sd.Y * sd.Z;
  if (tb <= 1 || slice % TILE != 0) return lt;
  const int ts = slice / TILE;
  const int b = lt / (tb * ts);
  const int rem = lt - b * (tb * ts);
  const int bt = min(tb, sd.T - b * tb);
  const int k = rem / bt;
  return (b * tb + (rem - k * bt)) * ts + k;
}

__device__ inline int find_slot(const SlotDesc* slots, int nslots, int kind, int u) {
  int lo = 0, hi = nslots - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (slots[mid].ubeg[kind] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Site coordinates of even-odd index s in parity p.
struct Coords { int x, y, z, t; };
__device__ inline Coords eo_coords(const SlotDesc& sd, int s, int p) {
  Coords c;
  int xh = s % sd.Xh;
  int rest = s / sd.Xh;
  c.y = rest % sd.Y;
  rest /= sd.Y;
  c.z = rest % sd.Z;
  c.t = rest / sd.Z;
  c.x = 2 * xh + ((p + c.y + c.z + c.t) & 1);
  return c;
}
__device__ inline int eo_index(const SlotDesc& sd, int x, int y, int z, int t) {
  return (x + sd.X * (y + sd.Y * (z + sd.Z * t))) >> 1;
}

// wave64 sum, fixed butterfly order (deterministic)
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace dl
