// One-end-trick contractions accumulated over sources (FP64 accumulators).
//
// Per site the kernels form colour-traced 4x4 Dirac outer products of the two
// vectors of each flavour structure (xi, phi = s):
//   with tau_3:    xi = gamma_5 s      -> C_ab = g5_a sum_c conj(s_ac) s_bc
//   without tau_3: xi = (1 - kappa H) s -> C_ab = sum_c conj(xi_ac) s_bc
// and, for the one-derivative insertions along nu,
//   E_ab = 1/2 sum_c [conj(xi_ac) (D s)_bc - conj((D xi)_ac) s_bc],
//   (D psi)(x) = 1/2 [U_nu(x) psi(x+nu) - U_nu(x-nu)^dag psi(x-nu)].
// The s-s products are Hermitian (local) or anti-Hermitian (derivative), so
// the tau_3 structure keeps 16 reals and the other 32 reals per operator; the
// gamma_5 of the tau_3 structure is applied when the loops are assembled.
//
// Work split: one wavefront = 64 sites of one parity (and, for the derivative,
// one direction nu); a workgroup holds the four directions of one tile so the
// site's own spinors are fetched once into L1.  Each lane runs over the
// slot's right-hand sides in order, summing their products in registers
// (compute precision) for KB sources at a time and adding each block sum to
// the FP64 accumulator: the accumulator traffic falls as 1/KB and every
// source is visited in a fixed order (deterministic).
//
// Accumulator component layout per site (reals):
//   local:   q  0..15  s-s Hermitian   (4 real diagonal, then (re, im) of
//                      (0,1) (0,2) (0,3) (1,2) (1,3) (2,3))
//            q 16..47  xi-s general    (re, im) of (a, b), index 2 (4 a + b)
//   deriv nu: base 48 + 48 nu, same two blocks (the s-s block anti-Hermitian:
//                      4 imaginary diagonal parts, then the upper triangle).
#include <stdexcept>

#include "kernels.h"

namespace dl {

int acc_components(int ops) { return (ops & 2) ? 240 : 48; }

// register sums in the compute precision, KB sources per flush
template <class S> struct AccT { using A = float; static constexpr int KB = 16; };
template <> struct AccT<double> { using A = double; static constexpr int KB = 1 << 30; };

// upper-triangle pair k = 0..5 -> (a, b): (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ constexpr int up_a(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
__device__ constexpr int up_b(int k) { return k < 3 ? k + 1 : (k < 5 ? k - 1 : 3); }

// acc: the block's first component (uniform), lane: this lane's site offset.
template <class A>
__device__ inline void flush(double* acc, long long V, int lane, A (&a)[48]) {
  // keep the 48 addresses from being computed once and held across the
  // source loop (that alone would take 96 registers)
  asm volatile("" : "+v"(lane));
#pragma unroll
  for (int q = 0; q < 48; ++q) {
    double* p = acc + q * V;
    p[lane] += (double)a[q];
    a[q] = (A)0;
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_contract_local(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o) {
  using R = typename Traits<S>::R;
  using A = typename AccT<S>::A;
  const int u = xcd_logical_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_SITE, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_SITE];
  const int par = ul & 1, tile = ul >> 1;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc) return;
  const long vh = sd.Vh;
  const long long V = 2ll * vh;
  double* acc = sd.acc;
  const int lane_off = par * (int)vh + s;
  const void* sf = par ? s_o : s_e;
  const void* xf = par ? xi_o : xi_e;
  A a[48];
#pragma unroll
  for (int q = 0; q < 48; ++q) a[q] = (A)0;
  int inblk = 0;
#pragma unroll 1
  for (int r = 0; r < sd.nrhs; ++r) {
    const long long off = sd.fo + (long long)r * vh;
    cx<R> sv[12], xv[12];
    load_spinor<S>(field_at<S>(sf, off), vh, s, sv);
    load_spinor<S>(field_at<S>(xf, off), vh, s, xv);
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
    if (++inblk == AccT<S>::KB) {
      flush(acc, V, lane_off, a);
      inblk = 0;
    }
  }
  if (inblk) flush(acc, V, lane_off, a);
}

// (D psi)(x) along nu from the neighbour spinors of one rhs field:
// 1/2 [U_nu(x) psi(x+nu) bp - U_nu(x-nu)^dag psi(x-nu) bm], bp / bm the
// time-boundary factors.
template <class S>
__device__ inline void cov_deriv(const void* f_other, long vh, int sp, int sm, typename Traits<S>::R bp,
                                 typename Traits<S>::R bm, const cx<typename Traits<S>::R> (&up)[9],
                                 const cx<typename Traits<S>::R> (&um)[9], cx<typename Traits<S>::R> (&out)[12]) {
  using R = typename Traits<S>::R;
  cx<R> v[12];
  load_spinor<S>(f_other, vh, sp, v);
#pragma unroll
  for (int sp4 = 0; sp4 < 4; ++sp4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> f = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac(f, up[3 * a + k], v[3 * sp4 + k]);
      out[3 * sp4 + a] = bp * f;
    }
  load_spinor<S>(f_other, vh, sm, v);
#pragma unroll
  for (int sp4 = 0; sp4 < 4; ++sp4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> b = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cjmac(b, um[3 * k + a], v[3 * sp4 + k]);
      out[3 * sp4 + a] = out[3 * sp4 + a] - bm * b;
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_contract_deriv(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o) {
  using R = typename Traits<S>::R;
  using A = typename AccT<S>::A;
  const int u = xcd_logical_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_DERIV, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_DERIV];
  const int nu = ul & 3, par = (ul >> 2) & 1, tile = ul >> 3;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc || !(sd.acc_ops & 2)) return;
  const long vh = sd.Vh;
  const Coords c = eo_coords(sd, s, par);
  int xp[4] = {c.x, c.y, c.z, c.t}, xm[4] = {c.x, c.y, c.z, c.t};
  const int ext[4] = {sd.X, sd.Y, sd.Z, sd.T};
  R bp = (R)0.5, bm = (R)0.5;
  xp[nu] += 1;
  if (xp[nu] == ext[nu]) { xp[nu] = 0; if (nu == 3) bp = (R)(0.5 * sd.bc); }
  xm[nu] -= 1;
  if (xm[nu] < 0) { xm[nu] = ext[nu] - 1; if (nu == 3) bm = (R)(0.5 * sd.bc); }
  const int sp = eo_index(sd, xp[0], xp[1], xp[2], xp[3]);
  const int sm = eo_index(sd, xm[0], xm[1], xm[2], xm[3]);
  const void* gauge = sd.gauge[Traits<S>::prec];
  cx<R> up[9], um[9];
  load_link<S>(gauge, vh, nu, par, s, up);
  load_link<S>(gauge, vh, nu, 1 - par, sm, um);
  const void* s_here = par ? s_o : s_e;
  const void* s_other = par ? s_e : s_o;
  const void* x_here = par ? xi_o : xi_e;
  const void* x_other = par ? xi_e : xi_o;
  const long long V = 2ll * vh;
  double* acc = sd.acc + (long long)(48 + 48 * nu) * V;
  const int lane_off = par * (int)vh + s;
  A a[48];
#pragma unroll
  for (int q = 0; q < 48; ++q) a[q] = (A)0;
  int inblk = 0;
#pragma unroll 1
  for (int r = 0; r < sd.nrhs; ++r) {
    const long long off = sd.fo + (long long)r * vh;
    cx<R> sv[12], d[12];
    load_spinor<S>(field_at<S>(s_here, off), vh, s, sv);
    cov_deriv<S>(field_at<S>(s_other, off), vh, sp, sm, bp, bm, up, um, d);   // d = D s
    // s-s block: E_ab = 1/2 sum_c [conj(s_a) (Ds)_b - conj((Ds)_a) s_b], anti-Hermitian
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R im = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) im += sv[3 * i + k].re * d[3 * i + k].im - sv[3 * i + k].im * d[3 * i + k].re;
      a[i] += (A)im;
    }
#pragma unroll
    for (int k6 = 0; k6 < 6; ++k6) {
      cx<R> t1 = mk<R>(0, 0), t2 = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cjmac(t1, sv[3 * up_a(k6) + k], d[3 * up_b(k6) + k]);
        cjmac(t2, d[3 * up_a(k6) + k], sv[3 * up_b(k6) + k]);
      }
      a[4 + 2 * k6] += (A)((R)0.5 * (t1.re - t2.re));
      a[5 + 2 * k6] += (A)((R)0.5 * (t1.im - t2.im));
    }
    // xi-s block, first half: 1/2 conj(xi_a) (Ds)_b
    {
      cx<R> xv[12];
      load_spinor<S>(field_at<S>(x_here, off), vh, s, xv);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> t = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 3; ++k) cjmac(t, xv[3 * i + k], d[3 * j + k]);
          a[16 + 2 * (4 * i + j)] += (A)((R)0.5 * t.re);
          a[17 + 2 * (4 * i + j)] += (A)((R)0.5 * t.im);
        }
    }
    // second half: -1/2 conj((D xi)_a) s_b
    cov_deriv<S>(field_at<S>(x_other, off), vh, sp, sm, bp, bm, up, um, d);   // d = D xi
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<R> t = mk<R>(0, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) cjmac(t, d[3 * i + k], sv[3 * j + k]);
        a[16 + 2 * (4 * i + j)] -= (A)((R)0.5 * t.re);
        a[17 + 2 * (4 * i + j)] -= (A)((R)0.5 * t.im);
      }
    if (++inblk == AccT<S>::KB) {
      flush(acc, V, lane_off, a);
      inblk = 0;
    }
  }
  if (inblk) flush(acc, V, lane_off, a);
}

#define DISPATCH_PREC(prec, KERNEL, ...)                                                     \
  switch (prec) {                                                                            \
    case P64: hipLaunchKernelGGL((KERNEL<double>), __VA_ARGS__); break;                      \
    case P32: hipLaunchKernelGGL((KERNEL<float>), __VA_ARGS__); break;                       \
    case PB16: hipLaunchKernelGGL((KERNEL<bf16s>), __VA_ARGS__); break;                      \
    case PH16: hipLaunchKernelGGL((KERNEL<f16s>), __VA_ARGS__); break;                       \
    default: throw std::runtime_error("bad precision");                                     \
  }

void launch_contract_local(int prec, const SlotDesc* slots, int nslots, int total_units, const void* s_e,
                           const void* s_o, const void* xi_e, const void* xi_o, hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_contract_local, dim3((total_units + 3) / 4), dim3(256), 0, st, slots, nslots,
                total_units, s_e, s_o, xi_e, xi_o);
}

void launch_contract_deriv(int prec, const SlotDesc* slots, int nslots, int total_units, const void* s_e,
                           const void* s_o, const void* xi_e, const void* xi_o, hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_contract_deriv, dim3((total_units + 3) / 4), dim3(256), 0, st, slots, nslots,
                total_units, s_e, s_o, xi_e, xi_o);
}

}  // namespace dl
