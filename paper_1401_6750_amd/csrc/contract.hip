// One-end-trick contractions, FP64 accumulation over sources, momentum
// projection and the final Gamma / TSM assembly.
//
// Per site the kernels form colour-traced 4x4 Dirac outer products of the two
// vectors of each flavour structure (xi, phi = s):
//   with tau_3:    xi = gamma_5 s      -> C_ab = g5_a sum_c conj(s_ac) s_bc
//   without tau_3: xi = (1 - kappa H) s -> C_ab = sum_c conj(xi_ac) s_bc
// and, for the one-derivative insertions along nu,
//   E_ab = 1/2 sum_c [conj(xi_ac) (D s)_bc - conj((D xi)_ac) s_bc],
//   (D psi)(x) = 1/2 [U_nu(x) psi(x+nu) - U_nu(x-nu)^dag psi(x-nu)].
// The s-s products are Hermitian (local) or anti-Hermitian (derivative), so
// the tau_3 structure keeps 16 reals and the other 32 reals per operator.
// A right-hand-side block is summed in FP64 registers before one
// read-modify-write of the FP64 accumulator, so accumulator traffic falls
// with the block size.
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

__constant__ int c_upper_a[6] = {0, 0, 0, 1, 1, 2};
__constant__ int c_upper_b[6] = {1, 2, 3, 2, 3, 3};

template <class S>
__global__ __launch_bounds__(256) void k_contract_local(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o) {
  using R = typename Traits<S>::R;
  const int u = xcd_logical_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_SITE, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_SITE];
  const int par = ul & 1, tile = ul >> 1;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc) return;
  const long vh = sd.Vh;
  const void* sf = par ? s_o : s_e;
  const void* xf = par ? xi_o : xi_e;
  double a_ss[16], a_xs[32];
#pragma unroll
  for (int q = 0; q < 16; ++q) a_ss[q] = 0.0;
#pragma unroll
  for (int q = 0; q < 32; ++q) a_xs[q] = 0.0;
  for (int r = 0; r < sd.nrhs; ++r) {
    const long long off = sd.fo + (long long)r * vh;
    cx<R> sv[12], xv[12];
    load_spinor<S>(field_at<S>(sf, off), vh, s, sv);
    load_spinor<S>(field_at<S>(xf, off), vh, s, xv);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      R d = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) d += sv[3 * a + c].re * sv[3 * a + c].re + sv[3 * a + c].im * sv[3 * a + c].im;
      a_ss[a] += (double)d;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = (k < 3) ? 0 : (k < 5 ? 1 : 2);
      const int b = (k < 3) ? k + 1 : (k < 5 ? k - 1 : 3);
      cx<R> t = mk<R>(0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) cjmac(t, sv[3 * a + c], sv[3 * b + c]);
      a_ss[4 + 2 * k] += (double)t.re;
      a_ss[5 + 2 * k] += (double)t.im;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        cx<R> t = mk<R>(0, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) cjmac(t, xv[3 * a + c], sv[3 * b + c]);
        a_xs[2 * (4 * a + b)] += (double)t.re;
        a_xs[2 * (4 * a + b) + 1] += (double)t.im;
      }
  }
  const long long V = 2ll * vh;
  double* acc = sd.acc + (long long)par * vh + s;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q * V] += a_ss[q];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[(16 + q) * V] += a_xs[q];
}

// D psi at site (c, par) along nu for one rhs field pair (even, odd).
template <class S>
__device__ inline void cov_deriv(const SlotDesc& sd, const void* f_other, long vh, int sp, int sm, bool wrap_p,
                                 bool wrap_m, const cx<typename Traits<S>::R> (&up)[9],
                                 const cx<typename Traits<S>::R> (&um)[9], cx<typename Traits<S>::R> (&out)[12]) {
  using R = typename Traits<S>::R;
  cx<R> vp[12], vm[12];
  load_spinor<S>(f_other, vh, sp, vp);
  load_spinor<S>(f_other, vh, sm, vm);
  const R bp = wrap_p ? (R)(0.5 * sd.bc) : (R)0.5;
  const R bm = wrap_m ? (R)(0.5 * sd.bc) : (R)0.5;
#pragma unroll
  for (int sp4 = 0; sp4 < 4; ++sp4) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> f = mk<R>(0, 0), b = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cmac(f, up[3 * a + k], vp[3 * sp4 + k]);
        cjmac(b, um[3 * k + a], vm[3 * sp4 + k]);
      }
      out[3 * sp4 + a] = bp * f - bm * b;
    }
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_contract_deriv(const SlotDesc* slots, int nslots, int total_units,
                                                        const void* s_e, const void* s_o, const void* xi_e,
                                                        const void* xi_o) {
  using R = typename Traits<S>::R;
  const int u = xcd_logical_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_DERIV, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_DERIV];
  const int fl = ul & 1, nu = (ul >> 1) & 3, par = (ul >> 3) & 1, tile = ul >> 4;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh || !sd.acc || !(sd.acc_ops & 2)) return;
  const long vh = sd.Vh;
  const Coords c = eo_coords(sd, s, par);
  int xp[4] = {c.x, c.y, c.z, c.t}, xm[4] = {c.x, c.y, c.z, c.t};
  const int ext[4] = {sd.X, sd.Y, sd.Z, sd.T};
  bool wrap_p = false, wrap_m = false;
  xp[nu] += 1;
  if (xp[nu] == ext[nu]) { xp[nu] = 0; wrap_p = (nu == 3); }
  xm[nu] -= 1;
  if (xm[nu] < 0) { xm[nu] = ext[nu] - 1; wrap_m = (nu == 3); }
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
  double* acc = sd.acc + (long long)(48 + 48 * nu) * V + (long long)par * vh + s;
  if (fl == 0) {
    double a_ss[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a_ss[q] = 0.0;
    for (int r = 0; r < sd.nrhs; ++r) {
      const long long off = sd.fo + (long long)r * vh;
      cx<R> sv[12], ds[12];
      load_spinor<S>(field_at<S>(s_here, off), vh, s, sv);
      cov_deriv<S>(sd, field_at<S>(s_other, off), vh, sp, sm, wrap_p, wrap_m, up, um, ds);
      // E_ab = 1/2 sum_c [conj(s_a) ds_b - conj(ds_a) s_b]  (anti-Hermitian)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        R im = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) im += sv[3 * a + k].re * ds[3 * a + k].im - sv[3 * a + k].im * ds[3 * a + k].re;
        a_ss[a] += (double)im;   // Im E_aa = Im(conj(s) ds)
      }
#pragma unroll
      for (int k6 = 0; k6 < 6; ++k6) {
        const int a = (k6 < 3) ? 0 : (k6 < 5 ? 1 : 2);
        const int b = (k6 < 3) ? k6 + 1 : (k6 < 5 ? k6 - 1 : 3);
        cx<R> t1 = mk<R>(0, 0), t2 = mk<R>(0, 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          cjmac(t1, sv[3 * a + k], ds[3 * b + k]);
          cjmac(t2, ds[3 * a + k], sv[3 * b + k]);
        }
        a_ss[4 + 2 * k6] += 0.5 * (double)(t1.re - t2.re);
        a_ss[5 + 2 * k6] += 0.5 * (double)(t1.im - t2.im);
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q * V] += a_ss[q];
  } else {
    double a_xs[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) a_xs[q] = 0.0;
    for (int r = 0; r < sd.nrhs; ++r) {
      const long long off = sd.fo + (long long)r * vh;
      cx<R> sv[12], ds[12], xv[12], dx[12];
      load_spinor<S>(field_at<S>(s_here, off), vh, s, sv);
      load_spinor<S>(field_at<S>(x_here, off), vh, s, xv);
      cov_deriv<S>(sd, field_at<S>(s_other, off), vh, sp, sm, wrap_p, wrap_m, up, um, ds);
      cov_deriv<S>(sd, field_at<S>(x_other, off), vh, sp, sm, wrap_p, wrap_m, up, um, dx);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          cx<R> t1 = mk<R>(0, 0), t2 = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            cjmac(t1, xv[3 * a + k], ds[3 * b + k]);
            cjmac(t2, dx[3 * a + k], sv[3 * b + k]);
          }
          a_xs[2 * (4 * a + b)] += 0.5 * (double)(t1.re - t2.re);
          a_xs[2 * (4 * a + b) + 1] += 0.5 * (double)(t1.im - t2.im);
        }
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[(16 + q) * V] += a_xs[q];
  }
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

// ---------------------------------------------------------------------------
// momentum projection: proj[q][t][p] = sum_xvec phase_p(xvec) acc[q][x]
// phase_p(x) = px[p][x] py[p][y] pz[p][z], complex128 tables [Np][L]
// ---------------------------------------------------------------------------
template <int PC>
__global__ __launch_bounds__(256) void k_project(const double* acc, int X, int Y, int Z, int T, int np,
                                                 const double2* px, const double2* py, const double2* pz,
                                                 double2* proj) {
  const int nchunk = (np + PC - 1) / PC;
  int b = blockIdx.x;
  const int ch = b % nchunk;
  b /= nchunk;
  const int t = b % T;
  const int q = b / T;
  const int p0 = ch * PC;
  const int Vs = X * Y * Z;
  const long long vh = (long long)Vs * T / 2;
  const int Xh = X / 2;
  double sre[PC], sim[PC];
#pragma unroll
  for (int j = 0; j < PC; ++j) sre[j] = sim[j] = 0.0;
  const double* a = acc + (long long)q * 2 * vh;
  for (int i = threadIdx.x; i < Vs; i += blockDim.x) {
    const int par = i / (Vs / 2);
    const int sl = i - par * (Vs / 2);
    const long long s = (long long)t * (Vs / 2) + sl;
    const int xh = sl % Xh;
    int rest = sl / Xh;
    const int y = rest % Y;
    const int z = rest / Y;
    const int x = 2 * xh + ((par + y + z + t) & 1);
    const double v = a[par * vh + s];
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      const int p = p0 + j;
      if (p < np) {
        const double2 fx = px[p * X + x], fy = py[p * Y + y], fz = pz[p * Z + z];
        const double re1 = fx.x * fy.x - fx.y * fy.y, im1 = fx.x * fy.y + fx.y * fy.x;
        const double re = re1 * fz.x - im1 * fz.y, im = re1 * fz.y + im1 * fz.x;
        sre[j] += v * re;
        sim[j] += v * im;
      }
    }
  }
  __shared__ double red[4][PC][2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < PC; ++j) {
    const double r = wave_sum(sre[j]), im = wave_sum(sim[j]);
    if (lane == 0) { red[wv][j][0] = r; red[wv][j][1] = im; }
  }
  __syncthreads();
  if (threadIdx.x < PC) {
    const int j = threadIdx.x, p = p0 + j;
    if (p < np) {
      const double r = (red[0][j][0] + red[1][j][0]) + (red[2][j][0] + red[3][j][0]);
      const double im = (red[0][j][1] + red[1][j][1]) + (red[2][j][1] + red[3][j][1]);
      proj[((long long)q * T + t) * np + p] = make_double2(r, im);
    }
  }
}

void launch_project(const double* acc, int nq, int X, int Y, int Z, int T, int np, const double* phase_x,
                    const double* phase_y, const double* phase_z, double* proj, hipStream_t st) {
  if (np <= 0 || nq <= 0) return;
  const double2 *px = (const double2*)phase_x, *py = (const double2*)phase_y, *pz = (const double2*)phase_z;
  if (np <= 8) {
    hipLaunchKernelGGL(k_project<8>, dim3(nq * T), dim3(256), 0, st, acc, X, Y, Z, T, np, px, py, pz,
                       (double2*)proj);
  } else if (np <= 16) {
    hipLaunchKernelGGL(k_project<16>, dim3(nq * T), dim3(256), 0, st, acc, X, Y, Z, T, np, px, py, pz,
                       (double2*)proj);
  } else {
    const int nchunk = (np + 31) / 32;
    hipLaunchKernelGGL(k_project<32>, dim3(nq * T * nchunk), dim3(256), 0, st, acc, X, Y, Z, T, np, px, py,
                       pz, (double2*)proj);
  }
}

// ---------------------------------------------------------------------------
// final assembly: Gamma rebuild, TSM combination, prefactors
// ---------------------------------------------------------------------------
struct GammaTable {
  int col[16][4];       // Gamma_n has one nonzero per row a, at column col[n][a]
  double ph[16][4][2];  // its value
};
__constant__ GammaTable c_gamma;

// Projected complex value of the 4x4 matrix element (a, b) of one operator
// block: `blk` points at the block's first component [q][t][p].
__device__ inline double2 op_entry(const double2* blk, int hermitian_kind, int a, int b, long long stride,
                                   long long tp) {
  // hermitian_kind: 0 general (32 reals), 1 Hermitian (16), 2 anti-Hermitian (16)
  if (hermitian_kind == 0) {
    const double2 re = blk[(2 * (4 * a + b)) * stride + tp], im = blk[(2 * (4 * a + b) + 1) * stride + tp];
    return make_double2(re.x - im.y, re.y + im.x);           // P(re) + i P(im)
  }
  if (a == b) {
    const double2 d = blk[a * stride + tp];
    if (hermitian_kind == 1) return d;                       // real diagonal
    return make_double2(-d.y, d.x);                          // i P(im diag)
  }
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const int k = lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5);
  const double2 re = blk[(4 + 2 * k) * stride + tp], im = blk[(5 + 2 * k) * stride + tp];
  if (a < b) return make_double2(re.x - im.y, re.y + im.x);   // P(re) + i P(im)
  if (hermitian_kind == 1) return make_double2(re.x + im.y, re.y - im.x);  // P(re) - i P(im)
  return make_double2(-re.x - im.y, -re.y + im.x);          // -P(re) + i P(im)
}

__global__ __launch_bounds__(256) void k_loops_finalize(const double2* plp, const double2* php, const double2* plc,
                                                        double w_lp, double w_hp, int nops, int T, int np,
                                                        double2 pf_t3, double2 pf_1, double2* out) {
  const long long n_out = 2ll * nops * 16 * T * np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_out) return;
  const long long tp = i % ((long long)T * np);
  long long rest = i / ((long long)T * np);
  const int n = (int)(rest % 16);
  rest /= 16;
  const int op = (int)(rest % nops);
  const int fl = (int)(rest / nops);
  const long long stride = (long long)T * np;
  const int base = (op == 0 ? 0 : 48 + 48 * (op - 1)) + (fl == 0 ? 0 : 16);
  const int kind = fl == 1 ? 0 : (op == 0 ? 1 : 2);
  double re = 0.0, im = 0.0;
  for (int a = 0; a < 4; ++a) {
    const int b = c_gamma.col[n][a];
    const double gr = c_gamma.ph[n][a][0], gi = c_gamma.ph[n][a][1];
    const double g5 = (fl == 0 && a >= 2) ? -1.0 : 1.0;   // tau_3 structure: xi = gamma_5 s
    double2 v = make_double2(0.0, 0.0);
    if (w_lp != 0.0) {
      const double2 x = op_entry(plp + (long long)base * stride, kind, a, b, stride, tp);
      v.x += w_lp * x.x; v.y += w_lp * x.y;
    }
    if (w_hp != 0.0) {
      const double2 x = op_entry(php + (long long)base * stride, kind, a, b, stride, tp);
      const double2 y = op_entry(plc + (long long)base * stride, kind, a, b, stride, tp);
      v.x += w_hp * (x.x - y.x); v.y += w_hp * (x.y - y.y);
    }
    re += g5 * (gr * v.x - gi * v.y);
    im += g5 * (gr * v.y + gi * v.x);
  }
  const double2 pf = fl == 0 ? pf_t3 : pf_1;
  out[i] = make_double2(pf.x * re - pf.y * im, pf.x * im + pf.y * re);
}

void set_gamma_table(const int col[16][4], const double ph[16][4][2]) {
  GammaTable t;
  for (int n = 0; n < 16; ++n)
    for (int a = 0; a < 4; ++a) {
      t.col[n][a] = col[n][a];
      t.ph[n][a][0] = ph[n][a][0];
      t.ph[n][a][1] = ph[n][a][1];
    }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_gamma), &t, sizeof(t)) != hipSuccess)
    throw std::runtime_error("hipMemcpyToSymbol(gamma table) failed");
}

void launch_loops_finalize(const double* proj_lp, const double* proj_hp, const double* proj_lpc, double w_lp,
                           double w_hp, int nops, int T, int np, double kappa, double mu, double* out,
                           hipStream_t st) {
  const long long n_out = 2ll * nops * 16 * T * np;
  if (n_out == 0) return;
  // physical-normalisation prefactors: tau_3  -2 i mu (2 kappa)^2,  no tau_3  4 kappa
  const double2 pf_t3 = make_double2(0.0, -2.0 * mu * 4.0 * kappa * kappa);
  const double2 pf_1 = make_double2(4.0 * kappa, 0.0);
  hipLaunchKernelGGL(k_loops_finalize, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st,
                     (const double2*)proj_lp, (const double2*)proj_hp, (const double2*)proj_lpc, w_lp, w_hp,
                     nops, T, np, pf_t3, pf_1, (double2*)out);
}

}  // namespace dl
