// Even-odd twisted-mass Wilson hopping kernel with fused site-local epilogues.
//
// One wavefront handles one unit = 64 consecutive even-odd sites of one
// right-hand side of one batch slot; units of one tile are consecutive for all
// right-hand sides of the slot, and each XCD receives a contiguous range of
// units, so a tile's gauge links are fetched once into that XCD's L2 and
// reused by every right-hand side.
//
// Operator pieces (kappa normalised, chiral basis, gamma_5 = diag(1,1,-1,-1)):
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)
// A hop through (1 -+ gamma_mu) is done on the two independent spin
// combinations h0, h1 (colour vectors) and the lower two spin components are
// rebuilt from them, so each neighbour costs two SU(3) x colour products.
//
// Epilogue (per-spin complex factors, set per slot):
//   result = e (.) H(d (.) in) + f (.) y
// optionally followed by the CG update x += alpha p, r -= alpha result.
#include <stdexcept>

#include "kernels.h"

namespace dl {

template <class R>
__device__ inline void su3_mul(const cx<R> (&u)[9], const cx<R> (&h)[3], cx<R> (&w)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = u[3 * a] * h[0];
    cmac(s, u[3 * a + 1], h[1]);
    cmac(s, u[3 * a + 2], h[2]);
    w[a] = s;
  }
}

template <class R>
__device__ inline void su3_dag_mul(const cx<R> (&u)[9], const cx<R> (&h)[3], cx<R> (&w)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = mk<R>(0, 0);
    cjmac(s, u[a], h[0]);
    cjmac(s, u[3 + a], h[1]);
    cjmac(s, u[6 + a], h[2]);
    w[a] = s;
  }
}

// Spin projection: v (12 complex, index 3*spin+colour) -> h0, h1 for
// (1 - gamma_mu) (FWD) or (1 + gamma_mu) (!FWD).
template <int MU, bool FWD, class R>
__device__ inline void project(const cx<R> (&v)[12], cx<R> (&h0)[3], cx<R> (&h1)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> p0 = v[c], p1 = v[3 + c], p2 = v[6 + c], p3 = v[9 + c];
    if (MU == 0) {         // gamma_1 psi = (-i p3, -i p2, i p1, i p0)
      h0[c] = FWD ? p0 + times_i(p3) : p0 - times_i(p3);
      h1[c] = FWD ? p1 + times_i(p2) : p1 - times_i(p2);
    } else if (MU == 1) {  // gamma_2 psi = (-p3, p2, p1, -p0)
      h0[c] = FWD ? p0 + p3 : p0 - p3;
      h1[c] = FWD ? p1 - p2 : p1 + p2;
    } else if (MU == 2) {  // gamma_3 psi = (-i p2, i p3, i p0, -i p1)
      h0[c] = FWD ? p0 + times_i(p2) : p0 - times_i(p2);
      h1[c] = FWD ? p1 - times_i(p3) : p1 + times_i(p3);
    } else {               // gamma_4 psi = (p2, p3, p0, p1)
      h0[c] = FWD ? p0 - p2 : p0 + p2;
      h1[c] = FWD ? p1 - p3 : p1 + p3;
    }
  }
}

// Accumulate the full four-spinor rebuilt from the projected pair (w0, w1).
template <int MU, bool FWD, class R>
__device__ inline void reconstruct(cx<R> (&acc)[12], const cx<R> (&w0)[3], const cx<R> (&w1)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + w0[c];
    acc[3 + c] = acc[3 + c] + w1[c];
    if (MU == 0) {
      acc[6 + c] = acc[6 + c] + (FWD ? times_mi(w1[c]) : times_i(w1[c]));
      acc[9 + c] = acc[9 + c] + (FWD ? times_mi(w0[c]) : times_i(w0[c]));
    } else if (MU == 1) {
      acc[6 + c] = FWD ? acc[6 + c] - w1[c] : acc[6 + c] + w1[c];
      acc[9 + c] = FWD ? acc[9 + c] + w0[c] : acc[9 + c] - w0[c];
    } else if (MU == 2) {
      acc[6 + c] = acc[6 + c] + (FWD ? times_mi(w0[c]) : times_i(w0[c]));
      acc[9 + c] = acc[9 + c] + (FWD ? times_i(w1[c]) : times_mi(w1[c]));
    } else {
      acc[6 + c] = FWD ? acc[6 + c] - w0[c] : acc[6 + c] + w0[c];
      acc[9 + c] = FWD ? acc[9 + c] - w1[c] : acc[9 + c] + w1[c];
    }
  }
}

template <class S, int MU, bool HAS_D>
__device__ inline void hop_dir(const SlotDesc& sd, const void* gauge, const void* inb, const Coords& c,
                               int s, int p_out, const cx<typename Traits<S>::R> (&d)[4],
                               cx<typename Traits<S>::R> (&acc)[12]) {
  using R = typename Traits<S>::R;
  const long vh = sd.Vh;
  // forward neighbour x + mu
  {
    int xn = c.x, yn = c.y, zn = c.z, tn = c.t;
    R sign = 1;
    if (MU == 0) xn = (c.x + 1 == sd.X) ? 0 : c.x + 1;
    if (MU == 1) yn = (c.y + 1 == sd.Y) ? 0 : c.y + 1;
    if (MU == 2) zn = (c.z + 1 == sd.Z) ? 0 : c.z + 1;
    if (MU == 3) {
      if (c.t + 1 == sd.T) { tn = 0; sign = (R)sd.bc; } else tn = c.t + 1;
    }
    int sn = eo_index(sd, xn, yn, zn, tn);
    cx<R> v[12];
    load_spinor<S>(inb, vh, sn, v);
    if (HAS_D) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = d[k / 3] * v[k];
    }
    cx<R> h0[3], h1[3], w0[3], w1[3];
    project<MU, true>(v, h0, h1);
    cx<R> u[9];
    load_link<S>(gauge, vh, MU, p_out, s, u);
    if (MU == 3) {
#pragma unroll
      for (int k = 0; k < 9; ++k) u[k] = sign * u[k];
    }
    su3_mul(u, h0, w0);
    su3_mul(u, h1, w1);
    reconstruct<MU, true>(acc, w0, w1);
  }
  // backward neighbour x - mu
  {
    int xn = c.x, yn = c.y, zn = c.z, tn = c.t;
    R sign = 1;
    if (MU == 0) xn = (c.x == 0) ? sd.X - 1 : c.x - 1;
    if (MU == 1) yn = (c.y == 0) ? sd.Y - 1 : c.y - 1;
    if (MU == 2) zn = (c.z == 0) ? sd.Z - 1 : c.z - 1;
    if (MU == 3) {
      if (c.t == 0) { tn = sd.T - 1; sign = (R)sd.bc; } else tn = c.t - 1;
    }
    int sn = eo_index(sd, xn, yn, zn, tn);
    cx<R> v[12];
    load_spinor<S>(inb, vh, sn, v);
    if (HAS_D) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = d[k / 3] * v[k];
    }
    cx<R> h0[3], h1[3], w0[3], w1[3];
    project<MU, false>(v, h0, h1);
    cx<R> u[9];
    load_link<S>(gauge, vh, MU, 1 - p_out, sn, u);
    if (MU == 3) {
#pragma unroll
      for (int k = 0; k < 9; ++k) u[k] = sign * u[k];
    }
    su3_dag_mul(u, h0, w0);
    su3_dag_mul(u, h1, w1);
    reconstruct<MU, false>(acc, w0, w1);
  }
}

template <class S, int F>
__global__ __launch_bounds__(256) void k_dslash(DslashArgs a) {
  using R = typename Traits<S>::R;
  const int u = xcd_logical_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (u >= a.total_units) return;
  const int lane = threadIdx.x & 63;
  const int si = find_slot(a.slots, a.nslots, UK_RHS, u);
  const SlotDesc& sd = a.slots[si];
  const int ul = u - sd.ubeg[UK_RHS];
  const int tile = ul / sd.nrhs;
  const int r = ul - tile * sd.nrhs;
  const int g = sd.rhs_begin + r;
  if (a.active && !a.active[g]) return;
  const int s = tile * TILE + lane;
  const bool valid = s < sd.Vh;
  const long vh = sd.Vh;
  const long long off = sd.fo + (long long)r * vh;
  double nrm = 0.0;
  if (valid) {
    const Coef& cf = a.coef[si];
    cx<R> d[4], e[4], f[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      d[k] = mk<R>((R)cf.d[k][0], (R)cf.d[k][1]);
      e[k] = mk<R>((R)cf.e[k][0], (R)cf.e[k][1]);
      f[k] = mk<R>((R)cf.f[k][0], (R)cf.f[k][1]);
    }
    const Coords c = eo_coords(sd, s, a.p_out);
    const void* gauge = sd.gauge[Traits<S>::prec];
    const void* inb = field_at<S>(a.in, off);
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
    constexpr bool HD = (F & F_D) != 0;
    hop_dir<S, 0, HD>(sd, gauge, inb, c, s, a.p_out, d, acc);
    hop_dir<S, 1, HD>(sd, gauge, inb, c, s, a.p_out, d, acc);
    hop_dir<S, 2, HD>(sd, gauge, inb, c, s, a.p_out, d, acc);
    hop_dir<S, 3, HD>(sd, gauge, inb, c, s, a.p_out, d, acc);
    cx<R> res[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) res[k] = e[k / 3] * acc[k];
    if (F & F_Y) {
      cx<R> yv[12];
      load_spinor<S>(field_at<S>(a.y, off), vh, s, yv);
#pragma unroll
      for (int k = 0; k < 12; ++k) res[k] = res[k] + f[k / 3] * yv[k];
    }
    if (F & F_XR) {
      const R al = (R)a.alpha[g];
      cx<R> xv[12], rv[12], pv[12];
      load_spinor<S>(field_at<S>(a.x, off), vh, s, xv);
      load_spinor<S>(field_at<S>(a.r, off), vh, s, rv);
      load_spinor<S>(field_at<S>(a.p, off), vh, s, pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        xv[k] = xv[k] + al * pv[k];
        rv[k] = rv[k] - al * res[k];
      }
      store_spinor<S>(field_at<S>(a.x, off), vh, s, xv);
      quantize<S>(rv);                       // the norm is that of the stored residual
      store_spinor<S>(field_at<S>(a.r, off), vh, s, rv);
      if (F & F_NORM) nrm = norm2(rv);
    } else {
      quantize<S>(res);
      store_spinor<S>(field_at<S>(a.out, off), vh, s, res);
      if (F & F_OUT2) store_spinor<S>(field_at<S>(a.out2, off), vh, s, res);
      if (F & F_NORM) nrm = norm2(res);
    }
  }
  if (F & F_NORM) {
    nrm = wave_sum(nrm);
    if (lane == 0) a.partial[u] = nrm;
  }
}

template <class S>
static void launch_dslash_t(int flags, const DslashArgs& a, hipStream_t st) {
  const int wpb = 4;
  const int blocks = (a.total_units + wpb - 1) / wpb;
  if (blocks == 0) return;
  dim3 grid(blocks), block(64 * wpb);
  switch (flags) {
    case 0: hipLaunchKernelGGL((k_dslash<S, 0>), grid, block, 0, st, a); break;
    case F_D: hipLaunchKernelGGL((k_dslash<S, F_D>), grid, block, 0, st, a); break;
    case F_Y: hipLaunchKernelGGL((k_dslash<S, F_Y>), grid, block, 0, st, a); break;
    case F_D | F_Y: hipLaunchKernelGGL((k_dslash<S, F_D | F_Y>), grid, block, 0, st, a); break;
    case F_Y | F_NORM: hipLaunchKernelGGL((k_dslash<S, F_Y | F_NORM>), grid, block, 0, st, a); break;
    case F_Y | F_NORM | F_OUT2:
      hipLaunchKernelGGL((k_dslash<S, F_Y | F_NORM | F_OUT2>), grid, block, 0, st, a); break;
    case F_Y | F_XR | F_NORM:
      hipLaunchKernelGGL((k_dslash<S, F_Y | F_XR | F_NORM>), grid, block, 0, st, a); break;
    default: throw std::runtime_error("unsupported dslash flag combination");
  }
}

void launch_dslash(int prec, int flags, const DslashArgs& a, hipStream_t st) {
  switch (prec) {
    case P64: launch_dslash_t<double>(flags, a, st); break;
    case P32: launch_dslash_t<float>(flags, a, st); break;
    case PB16: launch_dslash_t<bf16s>(flags, a, st); break;
    case PH16: launch_dslash_t<f16s>(flags, a, st); break;
    default: throw std::runtime_error("bad precision");
  }
}

}  // namespace dl
