// Momentum projection of the FP64 loop accumulators and the final assembly of
// the loops: Gamma rebuild from the 4x4 outer products, TSM combination of the
// three accumulator sets and the one-end-trick prefactors.
#include <stdexcept>

#include "kernels.h"

namespace dl {
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

// Backward of the projection and Gamma rebuild: per-site spin matrices
//   Omega_{f,op}(x) = w_f sum_n [sum_p conj(g[f,op,n,t,p]) e^{-ip.x}] Gamma_n
// (w_f = prefactor / number of sources), layout [f][op][entry 4a+b][V] complex.
__global__ __launch_bounds__(256) void k_omega(const double2* g, int nops, int X, int Y, int Z, int T, int np,
                                               const double2* px, const double2* py, const double2* pz,
                                               double2 w_t3, double2 w_1, double2* omega) {
  const long long V = (long long)X * Y * Z * T;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * 2 * nops) return;
  const long long site = i % V;
  const int fo = (int)(i / V);
  const int op = fo % nops, fl = fo / nops;
  const long long vh = V / 2;
  const int par = (int)(site / vh);
  const long long s = site - par * vh;
  const int Xh = X / 2;
  const int xh = (int)(s % Xh);
  long long rest = s / Xh;
  const int y = (int)(rest % Y);
  rest /= Y;
  const int z = (int)(rest % Z);
  const int t = (int)(rest / Z);
  const int x = 2 * xh + ((par + y + z + t) & 1);
  const double2 w = fl == 0 ? w_t3 : w_1;
  double2 m[16];
  for (int e = 0; e < 16; ++e) m[e] = make_double2(0.0, 0.0);
  for (int n = 0; n < 16; ++n) {
    const double2* gn = g + ((((long long)fl * nops + op) * 16 + n) * T + t) * np;
    double ar = 0.0, ai = 0.0;
    for (int p = 0; p < np; ++p) {
      const double2 fx = px[p * X + x], fy = py[p * Y + y], fz = pz[p * Z + z];
      const double re1 = fx.x * fy.x - fx.y * fy.y, im1 = fx.x * fy.y + fx.y * fy.x;
      const double phr = re1 * fz.x - im1 * fz.y, phi = re1 * fz.y + im1 * fz.x;
      const double2 q = gn[p];   // conj(q) * phase
      ar += q.x * phr + q.y * phi;
      ai += q.x * phi - q.y * phr;
    }
    const double cr = w.x * ar - w.y * ai, ci = w.x * ai + w.y * ar;
    for (int a = 0; a < 4; ++a) {
      const int b = c_gamma.col[n][a];
      const double gr = c_gamma.ph[n][a][0], gi = c_gamma.ph[n][a][1];
      m[4 * a + b].x += cr * gr - ci * gi;
      m[4 * a + b].y += cr * gi + ci * gr;
    }
  }
  double2* o = omega + (long long)fo * 16 * V + site;
  for (int e = 0; e < 16; ++e) o[e * V] = m[e];
}

void launch_omega(const double* g, int nops, int X, int Y, int Z, int T, int np, const double* phase_x,
                  const double* phase_y, const double* phase_z, double kappa, double mu, long long nsrc,
                  double* omega, hipStream_t st) {
  const long long n = (long long)X * Y * Z * T * 2 * nops;
  const double2 w_t3 = make_double2(0.0, -2.0 * mu * 4.0 * kappa * kappa / (double)nsrc);
  const double2 w_1 = make_double2(4.0 * kappa / (double)nsrc, 0.0);
  hipLaunchKernelGGL(k_omega, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double2*)g, nops, X, Y,
                     Z, T, np, (const double2*)phase_x, (const double2*)phase_y, (const double2*)phase_z, w_t3, w_1,
                     (double2*)omega);
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
