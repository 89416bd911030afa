// Momentum projection of the FP64 loop accumulators and the final assembly of
// the loops: Gamma rebuild from the 4x4 outer products, TSM combination of the
// three accumulator sets and the one-end-trick prefactors.
#include <stdexcept>

#include "kernels.h"

namespace dl {
// ---------------------------------------------------------------------------
// momentum projection, separable over x, y, z:
//   proj[q][t][p] = sum_{x,y,z} e^{-2 pi i (kx x/X + ky y/Y + kz z/Z)} v_q(x,y,z,t)
// of the TSM-combined accumulator value v = sum_sets w_set acc_set.
// Stage 1+2 (one workgroup per (q, t, z) plane): the plane goes to LDS, is
// summed over x for every distinct kx, then over y for every distinct
// (kx, ky) pair of the momentum list (twiddles from LDS roots of unity).  Stage 3 (one thread per (q, t, p)):
// the sum over z.  Each accumulator value is read once, in whole rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_proj_plane(const double* a0, const double* a1, const double* a2, double w0,
                                                    double w1, double w2, int X, int Y, int Z, int T, long long vp,
                                                    int nkx, int nkxy, const double2* roots_x,
                                                    const double2* roots_y, const int* kx_mod, const int* ky_mod,
                                                    const int* pair_ix, double2* r2) {
  // LDS: the plane v[Y][X], its x-transform r1[Y][nkx], the roots of unity
  // e^{-2 pi i m / X} and e^{-2 pi i m / Y}; the twiddle of (k, x) is root
  // (k x mod X), stepped by k per x.
  extern __shared__ double lds[];
  double* v = lds;                                   // [Y][X]
  double2* r1 = (double2*)(lds + X * Y);             // [Y][nkx]
  double2* wx = r1 + Y * nkx;                        // [X]
  double2* wy = wx + X;                              // [Y]
  int b = blockIdx.x;
  const int z = b % Z;
  b /= Z;
  const int t = b % T;
  const int q = b / T;
  const int Xh = X / 2, half = Xh * Y;
  const long long base = (long long)q * 2 * vp + (long long)half * (z + (long long)Z * t);
  for (int i = threadIdx.x; i < X * Y; i += blockDim.x) {
    const int par = i / half, rem = i - par * half;
    const int y = rem / Xh, xh = rem - y * Xh;
    const int x = 2 * xh + ((par + y + z + t) & 1);
    const long long k = base + par * vp + rem;
    double val = 0.0;
    if (a0) val += w0 * a0[k];
    if (a1) val += w1 * a1[k];
    if (a2) val += w2 * a2[k];
    v[y * X + x] = val;
  }
  for (int i = threadIdx.x; i < X; i += blockDim.x) wx[i] = roots_x[i];
  for (int i = threadIdx.x; i < Y; i += blockDim.x) wy[i] = roots_y[i];
  __syncthreads();
  for (int o = threadIdx.x; o < Y * nkx; o += blockDim.x) {
    const int y = o / nkx, ix = o - y * nkx;
    const int m = kx_mod[ix];
    const double* row = v + y * X;
    double re = 0.0, im = 0.0;
    int idx = 0;
#pragma unroll 4
    for (int x = 0; x < X; ++x) {
      const double val = row[x];
      const double2 f = wx[idx];
      re += val * f.x;
      im += val * f.y;
      idx += m;
      if (idx >= X) idx -= X;
    }
    r1[o] = make_double2(re, im);
  }
  __syncthreads();
  double2* out = r2 + ((long long)(q * T + t) * Z + z) * nkxy;
  for (int j = threadIdx.x; j < nkxy; j += blockDim.x) {
    const int ix = pair_ix[j], m = ky_mod[j];
    double re = 0.0, im = 0.0;
    int idx = 0;
#pragma unroll 4
    for (int y = 0; y < Y; ++y) {
      const double2 a = r1[y * nkx + ix], f = wy[idx];
      re += a.x * f.x - a.y * f.y;
      im += a.x * f.y + a.y * f.x;
      idx += m;
      if (idx >= Y) idx -= Y;
    }
    out[j] = make_double2(re, im);
  }
}

// Stage 3.  Rows q >= q_link hold link-centred derivative sums F(x, nu)
// (nu = (q - q_link) / 48) whose site value is F(x) + F(x - nu): spatial nu
// multiplies the projection by 1 + e^{-2 pi i n_nu / L_nu}, nu = t adds the
// projection of time slice t - 1 (periodic wrap; the boundary sign is inside F).
// Threads take the momenta in (kz, pair) order: neighbouring lanes read
// neighbouring r2 entries and share the kz twiddles.
__global__ __launch_bounds__(256) void k_proj_z(const double2* r2, int nq, int q_link, int Z, int T, int np, int nkxy,
                                                const double2* pz, const int* pj, const int* pk, const int* order,
                                                const double2* shift, double2* proj) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nq * T * np) return;
  const int p = order[(int)(i % np)];
  const long long qt = i / np;
  const int t = (int)(qt % T), q = (int)(qt / T);
  const int j = pj[p];
  const double2* ph = pz + (long long)pk[p] * Z;
  auto zsum = [&](int tt) {
    const double2* row = r2 + (long long)(q * T + tt) * Z * nkxy + j;
    double re = 0.0, im = 0.0;
    for (int z = 0; z < Z; ++z) {
      const double2 a = row[(long long)z * nkxy], f = ph[z];
      re += a.x * f.x - a.y * f.y;
      im += a.x * f.y + a.y * f.x;
    }
    return make_double2(re, im);
  };
  double2 r = zsum(t);
  if (q >= q_link) {
    const int nu = (q - q_link) / 48;
    if (nu < 3) {
      const double2 f = shift[p * 3 + nu];
      r = make_double2(r.x * f.x - r.y * f.y, r.x * f.y + r.y * f.x);
    } else {
      const double2 o = zsum(t == 0 ? T - 1 : t - 1);
      r.x += o.x;
      r.y += o.y;
    }
  }
  proj[qt * np + p] = r;
}

void launch_project(const double* const acc[3], const double w[3], int nq, int q_link, int X, int Y, int Z, int T,
                    const ProjTables& tb, double* r2, double* proj, hipStream_t st) {
  if (tb.np <= 0 || nq <= 0) return;
  const long long vp = pad_half((long long)X * Y * Z * T / 2);
  const size_t lds = sizeof(double) * (size_t)X * Y + sizeof(double2) * ((size_t)Y * tb.nkx + X + Y);
  // gfx950 gives a workgroup up to 160 KiB of LDS; above 64 KiB the kernel
  // has to be allowed the larger dynamic allocation first
  if (lds > 163840) throw std::runtime_error("momentum projection: x-y plane too large for LDS");
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)k_proj_plane, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    throw std::runtime_error("momentum projection: cannot raise the LDS limit of k_proj_plane");
  hipLaunchKernelGGL(k_proj_plane, dim3((unsigned)(nq * T * Z)), dim3(256), lds, st, acc[0], acc[1], acc[2], w[0],
                     w[1], w[2], X, Y, Z, T, vp, tb.nkx, tb.nkxy, (const double2*)tb.roots_x,
                     (const double2*)tb.roots_y, tb.kx_mod, tb.ky_mod, tb.pair_ix, (double2*)r2);
  const long long n = (long long)nq * T * tb.np;
  hipLaunchKernelGGL(k_proj_z, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double2*)r2, nq, q_link,
                     Z, T, tb.np, tb.nkxy, (const double2*)tb.pz, tb.pj, tb.pk, tb.order, (const double2*)tb.shift,
                     (double2*)proj);
}

__global__ __launch_bounds__(256) void k_fill_zero(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Zero n doubles with a kernel (a fill that a captured graph replays faithfully).
void launch_fill_zero(double* p, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

// ---------------------------------------------------------------------------
// final assembly: Gamma rebuild and prefactors (the TSM sets are combined
// before the projection)
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

__global__ __launch_bounds__(256) void k_loops_finalize(const double2* pr, int nops, int T, int np, double2 pf_t3,
                                                        double2 pf_1, const double2* exact, double2* out) {
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
    const double2 v = op_entry(pr + (long long)base * stride, kind, a, b, stride, tp);
    re += g5 * (gr * v.x - gi * v.y);
    im += g5 * (gr * v.y + gi * v.x);
  }
  if (exact && fl == 1 && tp % np == 0) {   // momentum 0 comes first
    re += exact[op * 16 + n].x;
    im += exact[op * 16 + n].y;
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

void launch_loops_finalize(const double* proj, int nops, int T, int np, double kappa, double mu,
                           const double* exact, double* out, hipStream_t st) {
  const long long n_out = 2ll * nops * 16 * T * np;
  if (n_out == 0) return;
  // physical-normalisation prefactors: tau_3  -2 i mu (2 kappa)^2,  no tau_3  4 kappa
  const double2 pf_t3 = make_double2(0.0, -2.0 * mu * 4.0 * kappa * kappa);
  const double2 pf_1 = make_double2(4.0 * kappa, 0.0);
  hipLaunchKernelGGL(k_loops_finalize, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st,
                     (const double2*)proj, nops, T, np, pf_t3, pf_1, (const double2*)exact, (double2*)out);
}

}  // namespace dl
