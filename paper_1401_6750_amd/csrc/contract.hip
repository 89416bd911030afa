// One-end-trick contractions accumulated over sources (FP64 accumulators).
//
// Per site the kernels form colour-traced 4x4 Dirac outer products of the two
// vectors of each flavour structure (xi, phi = s):
//   with tau_3:    xi = gamma_5 s      -> C_ab = g5_a sum_c conj(s_ac) s_bc
//   without tau_3: xi = (1 - kappa H) s -> C_ab = sum_c conj(xi_ac) s_bc
// and, for the one-derivative insertions along nu,
//   E_ab = 1/2 sum_c [conj(xi_ac) (D s)_bc - conj((D xi)_ac) s_bc],
//   (D psi)(x) = 1/2 [U_nu(x) psi(x+nu) - U_nu(x-nu)^dag psi(x-nu)],
// accumulated per link as F(x) with E(x) = F(x) + F(x - nu) (see
// k_contract_deriv); the projection applies the shift.
// The s-s products are Hermitian (local) or anti-Hermitian (derivative), so
// the tau_3 structure keeps 16 reals and the other 32 reals per operator; the
// gamma_5 of the tau_3 structure is applied when the loops are assembled.
//
// Hopping parameter expansion (HPE variants): the structure without tau_3
// takes the pair (xi = eta, phi = (kappa B H)^n s), whose outer product
// estimates the remainder R_n of the u flavour; the d flavour's remainder is
// gamma_5 R_n^dag gamma_5, so the flavour sum of a local insertion is
// C -> (C + g5 C^dag g5) / 2 and of a derivative insertion E -> (E - g5 E^dag g5) / 2
// (the Hermitian conjugate moves the derivative's forward hop to the other
// side, which flips its sign).  The map is linear, so it is applied to the
// register block sums when they are flushed.
//
// Work split: one wavefront = 64 sites of one parity (and, for the derivative,
// one direction nu); a workgroup holds the four directions of one tile so the
// site's own spinors are fetched once into L1.  Each lane runs over the
// slot's right-hand sides in order, summing their products in registers
// (compute precision) for KB sources at a time and adding each block sum to
// the FP64 accumulator: the accumulator traffic falls as 1/KB and every
// source is visited in a fixed order (deterministic).
//
// Accumulator layout: FP64 rows [q][parity * Vp + s], Vp = pad_half(Vh).
// Components per site (reals):
//   local:   q  0..15  s-s Hermitian   (4 real diagonal, then (re, im) of
//                      (0,1) (0,2) (0,3) (1,2) (1,3) (2,3))
//            q 16..47  xi-s general    (re, im) of (a, b), index 2 (4 a + b)
//   deriv nu: base 48 + 48 nu, same two blocks (the s-s block anti-Hermitian:
//                      4 imaginary diagonal parts, then the upper triangle).
#include <stdexcept>

#include "kernels.h"

namespace dl {

int acc_components(int ops) { return (ops & 2) ? 240 : 48; }

// Register sums in the compute precision, KB sources per flush into FP64.
// The flush is a read-modify-write of every component of the site (the
// dominant HBM traffic of these kernels), so KB is as large as accuracy
// allows: an FP32 sum of KB products carries < KB * 2^-24 relative rounding,
// 4e-6 for KB = 64, far below the 2^-8 / 2^-11 storage rounding of 16-bit
// fields; FP32 fields (the high-precision tier) keep KB = 16 (1e-6).
template <class S> struct AccT { using A = float; static constexpr int KB = Traits<S>::NC == 3 ? 64 : 16; };
template <> struct AccT<double> { using A = double; static constexpr int KB = 1 << 30; };

// upper-triangle pair k = 0..5 -> (a, b): (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ constexpr int up_a(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
__device__ constexpr int up_b(int k) { return k < 3 ? k + 1 : (k < 5 ? k - 1 : 3); }

// acc: the block's first component (uniform), lane: this lane's site offset.
// DERIV: the derivative sums are kept without their constant factors in the
// source loop (1/2 on the s-s diagonal, 1/4 elsewhere, powers of two, so the
// scaling is exact) and scaled here.
template <bool DERIV, bool HPE, class A>
__device__ inline void flush(double* acc, long long V, int lane, A (&a)[48], bool xs = true) {
  // keep the 48 addresses from being computed once and held across the
  // source loop (that alone would take 96 registers)
  asm volatile("" : "+v"(lane));
  if constexpr (HPE) {
    // xi-s block -> (C + sg g5 C^dag g5) / 2, sg = +1 local, -1 derivative:
    // entry (i, j) takes sg g5_i g5_j conj(C_ji)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) {
        const int qij = 16 + 2 * (4 * i + j), qji = 16 + 2 * (4 * j + i);
        const A gg = (((i < 2) == (j < 2)) == !DERIV) ? (A)1 : (A)-1;
        const A re_ij = a[qij], im_ij = a[qij + 1], re_ji = a[qji], im_ji = a[qji + 1];
        a[qij] = (A)0.5 * (re_ij + gg * re_ji);
        a[qij + 1] = (A)0.5 * (im_ij - gg * im_ji);
        if (j != i) {
          a[qji] = (A)0.5 * (re_ji + gg * re_ij);
          a[qji + 1] = (A)0.5 * (im_ji - gg * im_ij);
        }
      }
  }
  // the accumulator pointer comes from the slot descriptor: accessed through a
  // global-address-space pointer, not as generic (flat) memory
  using GD = __attribute__((address_space(1))) double;
  GD* const g = (GD*)acc;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    GD* p = g + q * V;
    const double f = DERIV ? (q < 4 ? 0.5 : 0.25) : 1.0;
    p[lane] += f * (double)a[q];
    a[q] = (A)0;
  }
  if (xs) {   // else the xi-s block was not contracted at this site in this block
#pragma unroll
    for (int q = 16; q < 48; ++q) {
      GD* p = g + q * V;
      p[lane] += (DERIV ? 0.25 : 1.0) * (double)a[q];
      a[q] = (A)0;
    }
  }
}

// Time dilution with the expansion: eta of component c lives on the slices
// t mod D == c, so the xi-s block (xi = eta) of an rhs of component c is
// non-zero only there -- and, for the link-centred time derivative, on the
// slice before.  Elsewhere it is skipped (the single-time-slice contraction);
// the s-s block is always summed.
// The components whose xi-s terms reach a site: (t mod D, and for the time
// derivative the next slice's, else -1); without dilution both are 0 = the
// component of every rhs.
struct XsComps { int c0, c1; };
__device__ inline XsComps xs_comps(const SlotDesc& sd, int t, int nu) {
  if (sd.tdil <= 1) return {0, 0};
  const int tn = t + 1 == sd.T ? 0 : t + 1;
  return {t % sd.tdil, nu == 3 ? tn % sd.tdil : -1};
}

// ---------------------------------------------------------------------------
// 16-bit fields: the products run on the packed (re, im) words with the dot2
// instructions, two products per instruction, accumulating into the FP32
// register sums.  Products of stored 16-bit values are exact in FP32; a
// transported vector (an FP32 colour product) is rounded to the storage format
// first, as the field it came from was.
// ---------------------------------------------------------------------------
__device__ inline void load_words16(const void* f, long vp, int s, uint32_t (&w)[12]) {
  // wave-uniform row addresses plus one 32-bit lane offset: the loads take the
  // scalar-base + vector-offset form and no 64-bit address is held per lane
  // (the empty asm keeps the offset opaque, so the rhs loop cannot turn each
  // per-lane address into an induction variable of its own)
  const char* b = (const char*)f;
  uint32_t o = (uint32_t)s << 4;
  asm volatile("" : "+v"(o));
  const uint4 q0 = *(const uint4*)(b + o);
  const uint4 q1 = *(const uint4*)(b + vp * 16 + o);
  const uint4 q2 = *(const uint4*)(b + vp * 32 + o);
  w[0] = q0.x; w[1] = q0.y; w[2] = q0.z; w[3] = q0.w;
  w[4] = q1.x; w[5] = q1.y; w[6] = q1.z; w[7] = q1.w;
  w[8] = q2.x; w[9] = q2.y; w[10] = q2.z; w[11] = q2.w;
}
// (im, -re) of a packed (re, im) pair: Im(conj(a) b) = dot2(a, iq16(b)).
__device__ inline uint32_t iq16(uint32_t w) { return swap16(w) ^ 0x80000000u; }
// both halves negated
__device__ inline uint32_t neg16(uint32_t w) { return w ^ 0x80008000u; }

template <class S, bool HPE>
__device__ inline void local_rhs16(const void* sf, const void* xf, const void* pf, long long off, long vp, int s,
                                   bool xs, float (&a)[48]) {
  uint32_t sw[12];
  load_words16(field_at<S>(sf, off), vp, s, sw);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float v = a[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) v = dot2<S>(sw[3 * i + c], sw[3 * i + c], v);
    a[i] = v;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float re = a[4 + 2 * k], im = a[5 + 2 * k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      re = dot2<S>(sw[3 * up_a(k) + c], sw[3 * up_b(k) + c], re);
      im = dot2<S>(sw[3 * up_a(k) + c], iq16(sw[3 * up_b(k) + c]), im);
    }
    a[4 + 2 * k] = re;
    a[5 + 2 * k] = im;
  }
  if (xs) {
    uint32_t xw[12];
    load_words16(field_at<S>(xf, off), vp, s, xw);
    if constexpr (HPE) load_words16(field_at<S>(pf, off), vp, s, sw);   // phi from here on
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float re = a[16 + 2 * (4 * i + j)], im = a[17 + 2 * (4 * i + j)];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          re = dot2<S>(xw[3 * i + c], sw[3 * j + c], re);
          im = dot2<S>(xw[3 * i + c], iq16(sw[3 * j + c]), im);
        }
        a[16 + 2 * (4 * i + j)] = re;
        a[17 + 2 * (4 * i + j)] = im;
      }
  }
}

template <class S, bool HPE, bool DIL>
__global__ __launch_bounds__(256) void k_contract_local(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o, const void* phi_e, const void* phi_o) {
  using R = typename Traits<S>::R;
  using A = typename AccT<S>::A;
  const int u = wave_unit();
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_SITE, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_SITE];
  const int par = ul & 1, tile = ul >> 1;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc) return;
  const long vp = sd.Vp;
  const long long V = 2ll * vp;
  double* acc = sd.acc;
  const int lane_off = par * (int)vp + s;
  const void* sf = par ? s_o : s_e;
  const void* xf = par ? xi_o : xi_e;
  const void* pf = par ? phi_o : phi_e;
  XsComps xc{0, 0};
  if constexpr (DIL) xc = xs_comps(sd, eo_coords(sd, s, par).t, -1);
  bool any_xs = false;   // some rhs of the current register block had an xi-s term here
  A a[48];
#pragma unroll
  for (int q = 0; q < 48; ++q) a[q] = (A)0;
  int inblk = 0;
  // the slot's fields the loop needs, read once: the accumulator flushes are
  // stores the compiler cannot tell apart from the slot table, so fields read
  // through `sd` inside the loop would be fetched again (and waited for) on
  // every right-hand side
  const long long fo = sd.fo;
  const int nrhs = sd.nrhs, tdil = sd.tdil, tentry = sd.tentry, tclen = sd.tclen;
#pragma unroll 1
  for (int r = 0; r < nrhs; ++r) {
    const long long off = fo + (long long)r * vp;
    bool xs = true;
    if constexpr (DIL) {
      const int comp = tdil > 1 ? (tentry + r) / tclen : 0;   // tdil_comp
      xs = xc.c0 == comp || xc.c1 == comp;
    }
    any_xs = any_xs || xs;
    if constexpr (Traits<S>::NC == 3) {
      local_rhs16<S, HPE>(sf, xf, pf, off, vp, s, xs, a);
    } else {
    cx<R> sv[12];
    load_spinor<S>(field_at<S>(sf, off), vp, s, sv);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R d = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) d += sv[3 * i + c].re * sv[3 * i + c].re + sv[3 * i + c].im * sv[3 * i + c].im;
      a[i] += (A)d;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cx<R> t = mk<R>(0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) cjmac(t, sv[3 * up_a(k) + c], sv[3 * up_b(k) + c]);
      a[4 + 2 * k] += (A)t.re;
      a[5 + 2 * k] += (A)t.im;
    }
    if (xs) {
      cx<R> xv[12];
      load_spinor<S>(field_at<S>(xf, off), vp, s, xv);
      if constexpr (HPE) load_spinor<S>(field_at<S>(pf, off), vp, s, sv);   // sv = phi from here on
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> t = mk<R>(0, 0);
#pragma unroll
          for (int c = 0; c < 3; ++c) cjmac(t, xv[3 * i + c], sv[3 * j + c]);
          a[16 + 2 * (4 * i + j)] += (A)t.re;
          a[17 + 2 * (4 * i + j)] += (A)t.im;
        }
    }
    }
    if (++inblk == AccT<S>::KB) {
      flush<false, HPE>(acc, V, lane_off, a, any_xs);
      inblk = 0;
      any_xs = false;
    }
  }
  if (inblk) flush<false, HPE>(acc, V, lane_off, a, any_xs);
}

// Forward transport of one rhs field along nu: out = M psi(x+nu), M = b U_nu(x)
// with the link's boundary factor b already folded in.  16-bit fields use the
// packed colour products (coefficients cr / ci prepared once per unit).
template <class S>
__device__ inline void transport_fwd(const void* f_other, long vp, int sp, const cx<typename Traits<S>::R> (&u)[9],
                                     const uint32_t (&cr)[9], const uint32_t (&ci)[9],
                                     cx<typename Traits<S>::R> (&out)[12]) {
  using R = typename Traits<S>::R;
  if constexpr (Traits<S>::NC == 3) {
    const uint4* q = (const uint4*)f_other;
    const uint4 q0 = q[sp], q1 = q[vp + sp], q2 = q[2 * vp + sp];
    const uint32_t v[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
    colour_mul16<S>(cr, ci, v, out);
  } else {
    cx<R> v[12];
    load_spinor<S>(f_other, vp, sp, v);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<R> f = u[3 * a] * v[3 * s4];
        cmac(f, u[3 * a + 1], v[3 * s4 + 1]);
        cmac(f, u[3 * a + 2], v[3 * s4 + 2]);
        out[3 * s4 + a] = f;
      }
  }
}

// T = (colour product of v) as packed words: (re, im) in tp, (im, -re) in tq.
template <class S>
__device__ inline void pack_transport(const uint32_t (&cr)[9], const uint32_t (&ci)[9], const uint32_t (&v)[12],
                                      uint32_t (&tp)[12], uint32_t (&tq)[12]) {
  cx<float> t[12];
  colour_mul16<S>(cr, ci, v, t);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    tp[k] = pack2<S>(t[k]);
    tq[k] = pack2<S>(mk<float>(t[k].im, -t[k].re));
  }
}

// The rows one rhs of the link-centred derivative contraction reads, as
// 16-bit words: s and xi at the site (sh, xh) and at its +nu neighbour (so,
// xo), and phi at both (ph, po; HPE).  All of an rhs's rows are requested
// before its first product.
template <bool HPE>
struct DerivRows16 {
  uint32_t sh[12], so[12], xh[12], xo[12];
  uint32_t ph[HPE ? 12 : 1], po[HPE ? 12 : 1];
};

template <class S, bool HPE>
__device__ inline void deriv_fetch16(DerivRows16<HPE>& d, const void* s_here, const void* s_other,
                                     const void* x_here, const void* x_other, const void* f_here,
                                     const void* f_other, long long off, long vp, int s, int sp, bool xs) {
  load_words16(field_at<S>(s_here, off), vp, s, d.sh);
  load_words16(field_at<S>(s_other, off), vp, sp, d.so);
  if (!xs) return;
  load_words16(field_at<S>(x_here, off), vp, s, d.xh);
  load_words16(field_at<S>(x_other, off), vp, sp, d.xo);
  if constexpr (HPE) {
    load_words16(field_at<S>(f_here, off), vp, s, d.ph);
    load_words16(field_at<S>(f_other, off), vp, sp, d.po);
  }
}

// One rhs of the link-centred derivative contraction on 16-bit fields (the
// same sums as the generic body below; constant factors at the flush).
template <class S, bool HPE>
__device__ inline void deriv_compute16(const DerivRows16<HPE>& d, const uint32_t (&cr)[9], const uint32_t (&ci)[9],
                                       bool xs, float (&a)[48]) {
  uint32_t tp[12], tq[12];
  pack_transport<S>(cr, ci, d.so, tp, tq);                  // T_s
  // s-s block: F_aa = (i/2) Im sum_c conj(s_a) T_a; off the diagonal
  // conj(s_a) T_b - conj(T_a) s_b
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float v = a[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) v = dot2<S>(d.sh[3 * i + c], tq[3 * i + c], v);
    a[i] = v;
  }
#pragma unroll
  for (int k6 = 0; k6 < 6; ++k6) {
    const int ia = up_a(k6), ib = up_b(k6);
    float re = a[4 + 2 * k6], im = a[5 + 2 * k6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      re = dot2<S>(d.sh[3 * ia + c], tp[3 * ib + c], re);
      re = dot2<S>(neg16(d.sh[3 * ib + c]), tp[3 * ia + c], re);
      im = dot2<S>(d.sh[3 * ia + c], tq[3 * ib + c], im);
      im = dot2<S>(d.sh[3 * ib + c], tq[3 * ia + c], im);
    }
    a[4 + 2 * k6] = re;
    a[5 + 2 * k6] = im;
  }
  if (!xs) return;
  // xi-s block, first half: conj(xi_a) T_phi,b (phi = s unless HPE)
  if constexpr (HPE) pack_transport<S>(cr, ci, d.po, tp, tq);   // T_phi
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float re = a[16 + 2 * (4 * i + j)], im = a[17 + 2 * (4 * i + j)];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        re = dot2<S>(d.xh[3 * i + c], tp[3 * j + c], re);
        im = dot2<S>(d.xh[3 * i + c], tq[3 * j + c], im);
      }
      a[16 + 2 * (4 * i + j)] = re;
      a[17 + 2 * (4 * i + j)] = im;
    }
  // second half: - conj(T_xi,a) phi_b, with (-re, -im) and (-re, im) of T_xi
  const uint32_t* ph;
  if constexpr (HPE) ph = d.ph;
  else ph = d.sh;
  {
    cx<float> t[12];
    colour_mul16<S>(cr, ci, d.xo, t);                       // T_xi
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      tp[k] = pack2<S>(mk<float>(-t[k].re, -t[k].im));
      tq[k] = pack2<S>(mk<float>(-t[k].re, t[k].im));
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float re = a[16 + 2 * (4 * i + j)], im = a[17 + 2 * (4 * i + j)];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        re = dot2<S>(tp[3 * i + c], ph[3 * j + c], re);
        im = dot2<S>(tq[3 * i + c], swap16(ph[3 * j + c]), im);
      }
      a[16 + 2 * (4 * i + j)] = re;
      a[17 + 2 * (4 * i + j)] = im;
    }
}

// One-derivative contractions in link-centred form.  With T_psi(x) =
// U_nu(x) psi(x+nu) (boundary factor included), the symmetric insertion
//   E_ab(x) = 1/2 sum_c [conj(xi_ac)(D s)_bc - conj((D xi)_ac) s_bc]
// equals F_ab(x) + F_ab(x - nu) with the per-link quantity
//   F_ab(x) = 1/4 sum_c [conj(xi_ac(x)) T_s,bc(x) - conj(T_xi,ac(x)) s_bc(x)]
// (the backward half of D at x+nu reproduces the forward half at x).  So
// each (site, nu) needs two transports instead of four, and the projection
// adds F(x - nu) (a momentum phase for spatial nu, the previous time slice
// for nu = t).  The s-s block (xi -> s) stays anti-Hermitian.  HPE: the
// xi-s block pairs xi = eta with phi instead of s, one more transport (T_phi).
// Waves per SIMD the derivative kernel is compiled for: four for the plain
// 16-bit instance (it fits 128 registers without spills, and its loads are
// latency-bound), the compiler's choice for the others (they would spill).
template <class S, bool HPE, bool DIL>
constexpr int deriv_min_waves() { return Traits<S>::NC == 3 && !HPE && !DIL ? 4 : 1; }

template <class S, bool HPE, bool DIL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(deriv_min_waves<S, HPE, DIL>(), 8))) void
k_contract_deriv(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o, const void* phi_e, const void* phi_o) {
  using R = typename Traits<S>::R;
  using A = typename AccT<S>::A;
  const int u = wave_unit();
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_DERIV, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_DERIV];
  // tiles in time blocks of sd.tblk slices (the pass sets the context's
  // contract_tblk): the tile holding a tile's +t neighbour rows runs at
  // nearly the same time, so those rows are still cached
  const int nu = ul & 3, par = (ul >> 2) & 1, tile = tile_of(sd, ul >> 3);
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc || !(sd.acc_ops & 2)) return;
  const long vp = sd.Vp;
  const Coords c = eo_coords(sd, s, par);
  int xp[4] = {c.x, c.y, c.z, c.t};
  const int ext[4] = {sd.X, sd.Y, sd.Z, sd.T};
  R b = (R)1;
  xp[nu] += 1;
  if (xp[nu] == ext[nu]) { xp[nu] = 0; if (nu == 3) b = (R)sd.bc; }
  const int sp = eo_index(sd, xp[0], xp[1], xp[2], xp[3]);
  const void* gauge = sd.gauge[Traits<S>::prec];
  cx<R> up[9];
  uint32_t cr[9], ci[9];
  if constexpr (Traits<S>::NC == 3) {
    const long long lr = (nu * 2 + par) * 3;
    const uint4 l0 = at16<uint4>(row16(gauge, lr, vp), s), l1 = at16<uint4>(row16(gauge, lr + 1, vp), s),
                l2 = at16<uint4>(row16(gauge, lr + 2, vp), s);
    const uint32_t e[9] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w, l2.x};
    link_coef16<true>(e, b < (R)0, cr, ci);
  } else {
    load_link<S>(gauge, vp, nu, par, s, up);
#pragma unroll
    for (int k = 0; k < 9; ++k) up[k] = b * up[k];
  }
  const void* s_here = par ? s_o : s_e;
  const void* s_other = par ? s_e : s_o;
  const void* x_here = par ? xi_o : xi_e;
  const void* x_other = par ? xi_e : xi_o;
  const void* f_here = par ? phi_o : phi_e;
  const void* f_other = par ? phi_e : phi_o;
  const long long V = 2ll * vp;
  double* acc = sd.acc + (long long)(48 + 48 * nu) * V;
  const int lane_off = par * (int)vp + s;
  XsComps xc{0, 0};
  if constexpr (DIL) xc = xs_comps(sd, c.t, nu);
  bool any_xs = false;   // some rhs of the current register block had an xi-s term here
  A a[48];
#pragma unroll
  for (int q = 0; q < 48; ++q) a[q] = (A)0;
  int inblk = 0;
  // the slot's fields the loop needs, read once: the accumulator flushes are
  // stores the compiler cannot tell apart from the slot table, so fields read
  // through `sd` inside the loop would be fetched again (and waited for) on
  // every right-hand side
  const long long fo = sd.fo;
  const int nrhs = sd.nrhs, tdil = sd.tdil, tentry = sd.tentry, tclen = sd.tclen;
  auto xs_of = [&](int r) -> bool {   // the xi-s terms of rhs r reach this site
    if constexpr (DIL) {
      const int comp = tdil > 1 ? (tentry + r) / tclen : 0;   // tdil_comp
      return xc.c0 == comp || xc.c1 == comp;
    }
    return true;
  };
  if constexpr (Traits<S>::NC == 3) {
    // 16-bit fields (fetching the next rhs's rows during the current one's
    // arithmetic needs a second buffer, 244 VGPRs, and measured slower)
    DerivRows16<HPE> d;
#pragma unroll 1
    for (int r = 0; r < nrhs; ++r) {
      const bool xs = xs_of(r);
      deriv_fetch16<S, HPE>(d, s_here, s_other, x_here, x_other, f_here, f_other, fo + (long long)r * vp, vp, s,
                            sp, xs);
      any_xs = any_xs || xs;
      deriv_compute16<S, HPE>(d, cr, ci, xs, a);
      if (++inblk == AccT<S>::KB) {
        flush<true, HPE>(acc, V, lane_off, a, any_xs);
        inblk = 0;
        any_xs = false;
      }
    }
  } else {
#pragma unroll 1
  for (int r = 0; r < nrhs; ++r) {
    const long long off = fo + (long long)r * vp;
    const bool xs = xs_of(r);
    any_xs = any_xs || xs;
    cx<R> sv[12], t[12];
    load_spinor<S>(field_at<S>(s_here, off), vp, s, sv);
    transport_fwd<S>(field_at<S>(s_other, off), vp, sp, up, cr, ci, t);   // t = T_s
    // s-s block: F_ab = 1/4 sum_c [conj(s_a) T_b - conj(T_a) s_b]; the sums
    // below omit the constant factors, applied at the flush
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R im = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        im = fmadd(sv[3 * i + k].re, t[3 * i + k].im, im);
        im = fmadd(-sv[3 * i + k].im, t[3 * i + k].re, im);
      }
      a[i] += (A)im;                             // F_aa = (i/2) Im sum_c conj(s_a) T_a
    }
#pragma unroll
    for (int k6 = 0; k6 < 6; ++k6) {
      cx<R> t1 = mk<R>(0, 0), t2 = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cjmac(t1, sv[3 * up_a(k6) + k], t[3 * up_b(k6) + k]);
        cjmac(t2, t[3 * up_a(k6) + k], sv[3 * up_b(k6) + k]);
      }
      a[4 + 2 * k6] += (A)(t1.re - t2.re);
      a[5 + 2 * k6] += (A)(t1.im - t2.im);
    }
    // xi-s block, first half: 1/4 conj(xi_a) T_phi,b (phi = s unless HPE)
    if (xs) {
      cx<R> xv[12];
      load_spinor<S>(field_at<S>(x_here, off), vp, s, xv);
      if constexpr (HPE) transport_fwd<S>(field_at<S>(f_other, off), vp, sp, up, cr, ci, t);   // t = T_phi
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> w = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 3; ++k) cjmac(w, xv[3 * i + k], t[3 * j + k]);
          a[16 + 2 * (4 * i + j)] += (A)w.re;
          a[17 + 2 * (4 * i + j)] += (A)w.im;
        }
      // second half: -1/4 conj(T_xi,a) phi_b
      if constexpr (HPE) load_spinor<S>(field_at<S>(f_here, off), vp, s, sv);   // sv = phi
      transport_fwd<S>(field_at<S>(x_other, off), vp, sp, up, cr, ci, t);   // t = T_xi
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> w = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 3; ++k) cjmac(w, t[3 * i + k], sv[3 * j + k]);
          a[16 + 2 * (4 * i + j)] -= (A)w.re;
          a[17 + 2 * (4 * i + j)] -= (A)w.im;
        }
    }
    if (++inblk == AccT<S>::KB) {
      flush<true, HPE>(acc, V, lane_off, a, any_xs);
      inblk = 0;
      any_xs = false;
    }
  }
  }
  if (inblk) flush<true, HPE>(acc, V, lane_off, a, any_xs);
}

#define DISPATCH_PREC(prec, H, D, KERNEL, ...)                                               \
  switch (prec) {                                                                            \
    case P64: hipLaunchKernelGGL((KERNEL<double, H, D>), __VA_ARGS__); break;                \
    case P32: hipLaunchKernelGGL((KERNEL<float, H, D>), __VA_ARGS__); break;                 \
    case PB16: hipLaunchKernelGGL((KERNEL<bf16s, H, D>), __VA_ARGS__); break;                \
    case PH16: hipLaunchKernelGGL((KERNEL<f16s, H, D>), __VA_ARGS__); break;                 \
    default: throw std::runtime_error("bad precision");                                     \
  }

void launch_contract_local(int prec, const SlotDesc* slots, int nslots, int total_units, const void* s_e,
                           const void* s_o, const void* xi_e, const void* xi_o, const void* phi_e,
                           const void* phi_o, bool dil, hipStream_t st) {
  if (!total_units) return;
  const dim3 grid((total_units + 3) / 4), block(256);
  if (phi_e && dil) {
    DISPATCH_PREC(prec, true, true, k_contract_local, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  } else if (phi_e) {
    DISPATCH_PREC(prec, true, false, k_contract_local, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  } else {
    DISPATCH_PREC(prec, false, false, k_contract_local, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  }
}

void launch_contract_deriv(int prec, const SlotDesc* slots, int nslots, int total_units, const void* s_e,
                           const void* s_o, const void* xi_e, const void* xi_o, const void* phi_e,
                           const void* phi_o, bool dil, hipStream_t st) {
  if (!total_units) return;
  const dim3 grid((total_units + 3) / 4), block(256);
  if (phi_e && dil) {
    DISPATCH_PREC(prec, true, true, k_contract_deriv, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  } else if (phi_e) {
    DISPATCH_PREC(prec, true, false, k_contract_deriv, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  } else {
    DISPATCH_PREC(prec, false, false, k_contract_deriv, grid, block, 0, st, slots, nslots, total_units, s_e, s_o,
                  xi_e, xi_o, phi_e, phi_o);
  }
}

}  // namespace dl
