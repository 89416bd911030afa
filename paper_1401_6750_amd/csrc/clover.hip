// Clover term of the twisted-mass operator (the Wilson-and-clover variant the
// paper expects its package to support, Section 2.4): the per-site matrices
// that take the place of the per-spin twist factors, and the site-local
// factor applied to a field before a hop that needs it at every neighbour.
//
// Operator (kappa normalisation): M = 1 + C - kappa H + 2 i kappa mu gamma_5,
// C(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x), sigma_{mu nu} =
// (i/2)[gamma_mu, gamma_nu], Fhat = (Q - Q^dag) / 8 with Q the four plaquettes
// of the (mu, nu) plane at x walked in the sense U_mu(x) U_nu(x+mu)
// U_mu(x+nu)^dag U_nu(x)^dag.  C commutes with gamma_5: two 6 x 6 blocks.
#include <stdexcept>

#include "kernels.h"

namespace dl {

namespace {

inline int grid_for(int units, int wpb) { return (units + wpb - 1) / wpb; }

struct M3 {
  cx<double> a[9];
};

__device__ inline M3 mul(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = s + x.a[3 * i + k] * y.a[3 * k + j];
      r.a[3 * i + j] = s;
    }
  return r;
}

__device__ inline M3 dag(const M3& x) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = conj(x.a[3 * j + i]);
  return r;
}

struct C4 {
  int v[4];
};

// link U_mu at lattice coordinates c (periodic wrap) from the packed FP64 field
__device__ inline M3 link_at(const void* g64, long vp, int mu, const C4& c, const int (&L)[4]) {
  int w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (c.v[k] % L[k] + L[k]) % L[k];
  const long lex = w[0] + (long)L[0] * (w[1] + (long)L[1] * (w[2] + (long)L[2] * w[3]));
  const int par = (w[0] + w[1] + w[2] + w[3]) & 1;
  M3 u;
  load_link<double>(g64, vp, mu, par, lex >> 1, u.a);
  return u;
}

// Gauss-Jordan inverse of an n x n complex matrix with partial pivoting (rows
// swapped in place; a is destroyed, inv receives the inverse).
__device__ inline void invert6(cx<double> (&a)[36], cx<double> (&inv)[36]) {
  for (int i = 0; i < 36; ++i) inv[i] = mk<double>(i % 7 == 0 ? 1.0 : 0.0, 0.0);
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = -1.0;
    for (int r = c; r < 6; ++r) {
      const double m = a[6 * r + c].re * a[6 * r + c].re + a[6 * r + c].im * a[6 * r + c].im;
      if (m > best) { best = m; piv = r; }
    }
    if (piv != c)
      for (int k = 0; k < 6; ++k) {
        cx<double> t = a[6 * c + k]; a[6 * c + k] = a[6 * piv + k]; a[6 * piv + k] = t;
        t = inv[6 * c + k]; inv[6 * c + k] = inv[6 * piv + k]; inv[6 * piv + k] = t;
      }
    const cx<double> p = a[6 * c + c];
    const double den = p.re * p.re + p.im * p.im;
    const cx<double> pi = mk<double>(p.re / den, -p.im / den);
    for (int k = 0; k < 6; ++k) {
      a[6 * c + k] = a[6 * c + k] * pi;
      inv[6 * c + k] = inv[6 * c + k] * pi;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const cx<double> f = a[6 * r + c];
      for (int k = 0; k < 6; ++k) {
        a[6 * r + k] = a[6 * r + k] - f * a[6 * c + k];
        inv[6 * r + k] = inv[6 * r + k] - f * inv[6 * c + k];
      }
    }
  }
}

__device__ inline void store_block(double2* o64, float4* o32, long vp, int kind, int par, long s, int b,
                                   const cx<double> (&m)[36]) {
  double2* p = o64 + (long)(kind * 2 + par) * 72 * vp + s;
  float4* q = o32 + (long)(kind * 2 + par) * 36 * vp + s;
  for (int e = 0; e < 36; ++e) p[(long)(36 * b + e) * vp] = make_double2(m[e].re, m[e].im);
  for (int e = 0; e < 36; e += 2)
    q[(long)((36 * b + e) / 2) * vp] =
        make_float4((float)m[e].re, (float)m[e].im, (float)m[e + 1].re, (float)m[e + 1].im);
}

}  // namespace

// sigma_{mu nu} of the six planes (mu < nu, order 01 02 03 12 13 23), complex 4 x 4
struct SigmaTable {
  double v[6][4][4][2];
};

__global__ __launch_bounds__(64) void k_clover_build(const void* g64, int X, int Y, int Z, int T, long vp,
                                                     double kappa, double mu, double csw, SigmaTable sg,
                                                     double2* o64, float4* o32) {
  const long lex = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long V = (long)X * Y * Z * T;
  if (lex >= V) return;
  const int L[4] = {X, Y, Z, T};
  int c[4];
  {
    long r = lex;
    c[0] = (int)(r % X); r /= X;
    c[1] = (int)(r % Y); r /= Y;
    c[2] = (int)(r % Z);
    c[3] = (int)(r / Z);
  }
  const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
  const long s = lex >> 1;
  // C blocks: T_b[3 s' + a][3 r' + c'] = i kappa c_sw sum_planes sigma[2b+s'][2b+r'] F[a][c']
  cx<double> tb[2][36];
  for (int b = 0; b < 2; ++b)
    for (int e = 0; e < 36; ++e) tb[b][e] = mk<double>(0.0, 0.0);
  int plane = 0;
  for (int m = 0; m < 4; ++m)
    for (int n = m + 1; n < 4; ++n, ++plane) {
      auto at = [&](int dm, int dn) {
        C4 y{{c[0], c[1], c[2], c[3]}};
        y.v[m] += dm;
        y.v[n] += dn;
        return y;
      };
      const M3 um = link_at(g64, vp, m, at(0, 0), L), un = link_at(g64, vp, n, at(0, 0), L);
      // x -> x+m -> x+m+n -> x+n -> x
      M3 q = mul(mul(um, link_at(g64, vp, n, at(1, 0), L)), mul(dag(link_at(g64, vp, m, at(0, 1), L)), dag(un)));
      // x -> x+n -> x+n-m -> x-m -> x
      const M3 p2 = mul(mul(un, dag(link_at(g64, vp, m, at(-1, 1), L))),
                        mul(dag(link_at(g64, vp, n, at(-1, 0), L)), link_at(g64, vp, m, at(-1, 0), L)));
      // x -> x-m -> x-m-n -> x-n -> x
      const M3 p3 = mul(mul(dag(link_at(g64, vp, m, at(-1, 0), L)), dag(link_at(g64, vp, n, at(-1, -1), L))),
                        mul(link_at(g64, vp, m, at(-1, -1), L), link_at(g64, vp, n, at(0, -1), L)));
      // x -> x-n -> x-n+m -> x+m -> x
      const M3 p4 = mul(mul(dag(link_at(g64, vp, n, at(0, -1), L)), link_at(g64, vp, m, at(0, -1), L)),
                        mul(link_at(g64, vp, n, at(1, -1), L), dag(um)));
      for (int e = 0; e < 9; ++e) q.a[e] = q.a[e] + p2.a[e] + p3.a[e] + p4.a[e];
      // i kappa c_sw Fhat, Fhat = (Q - Q^dag) / 8
      cx<double> f[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const cx<double> d = q.a[3 * i + j] - conj(q.a[3 * j + i]);
          f[3 * i + j] = times_i((kappa * csw / 8.0) * d);
        }
      for (int b = 0; b < 2; ++b)
        for (int sp = 0; sp < 2; ++sp)
          for (int rp = 0; rp < 2; ++rp) {
            const cx<double> sv = mk<double>(sg.v[plane][2 * b + sp][2 * b + rp][0], sg.v[plane][2 * b + sp][2 * b + rp][1]);
            if (sv.re == 0.0 && sv.im == 0.0) continue;
            for (int a = 0; a < 3; ++a)
              for (int cc = 0; cc < 3; ++cc) {
                const int row = 3 * sp + a, col = 3 * rp + cc;
                tb[b][6 * row + col] = tb[b][6 * row + col] + sv * f[3 * a + cc];
              }
          }
    }
  for (int b = 0; b < 2; ++b) {
    const double tw = 2.0 * kappa * mu * (b == 0 ? 1.0 : -1.0);   // 2 kappa mu gamma_5 on block b
    cx<double> ac[36], ap[36], am[36], inv[36], work[36];
    for (int e = 0; e < 36; ++e) {
      const double one = (e % 7 == 0) ? 1.0 : 0.0;
      ac[e] = mk<double>(one, 0.0) + tb[b][e];
      ap[e] = ac[e] + mk<double>(0.0, e % 7 == 0 ? tw : 0.0);
      am[e] = ac[e] - mk<double>(0.0, e % 7 == 0 ? tw : 0.0);
    }
    store_block(o64, o32, vp, CLV_AC, par, s, b, ac);
    store_block(o64, o32, vp, CLV_A, par, s, b, ap);
    store_block(o64, o32, vp, CLV_A_M, par, s, b, am);
    for (int e = 0; e < 36; ++e) work[e] = ap[e];
    invert6(work, inv);
    store_block(o64, o32, vp, CLV_AINV, par, s, b, inv);
    for (int e = 0; e < 36; ++e) work[e] = am[e];
    invert6(work, inv);
    store_block(o64, o32, vp, CLV_AINV_M, par, s, b, inv);
  }
}

void launch_clover_build(const void* g64, const int dims[4], long long vp, double kappa, double mu, double csw,
                         const double (&sigma)[6][4][4][2], void* o64, void* o32, hipStream_t st) {
  SigmaTable t;
  for (int p = 0; p < 6; ++p)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int k = 0; k < 2; ++k) t.v[p][a][b][k] = sigma[p][a][b][k];
  const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
  hipLaunchKernelGGL(k_clover_build, dim3((unsigned)((V + 63) / 64)), dim3(64), 0, st, g64, dims[0], dims[1],
                     dims[2], dims[3], (long)vp, kappa, mu, csw, t, (double2*)o64, (float4*)o32);
}

// ---------------------------------------------------------------------------
// site factor before a hop: out = d (.) (M_d in) on clover slots (rounded to the
// storage type), out = in (bit copy) elsewhere; the hop then applies d only on
// the slots without a clover term.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_site_factor(const SlotDesc* slots, int nslots, int total_units,
                                                     const Coef* coef, int par, const void* in, void* out,
                                                     const int* gate) {
  using R = typename Traits<S>::R;
  const int u = wave_unit();
  if (u >= total_units) return;
  const int si = find_slot(slots, nslots, UK_RHS, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_RHS];
  const int tile = ul / sd.nrhs, r = ul - tile * sd.nrhs;
  const int g = sd.rhs_begin + r;
  if (gate && !gate[g]) return;
  const int s = tile * TILE + (threadIdx.x & 63);
  if (s >= sd.Vh) return;
  const long vp = sd.Vp;
  const long long off = sd.fo + (long long)r * vp;
  const Coef& cf = coef[si];
  const void* clv = Traits<S>::prec == P64 ? sd.clv64 : sd.clv32;
  cx<R> v[1][12];
  load_spinor<S>(field_at<S>(in, off), vp, s, v[0]);
  if (clv && cf.m[0] >= 0) {
    cx<R> w[1][12];
    const bool act[1] = {true};
    site_matvec<1>(clv, cf.m[0], par, vp, s, v, w, act);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[0][k] = mk<R>((R)cf.d[k / 3][0], (R)cf.d[k / 3][1]) * w[0][k];
  }
  store_spinor<S>(field_at<S>(out, off), vp, s, v[0]);
}

void launch_site_factor(int prec, const SlotDesc* slots, int nslots, int total_units, const Coef* coef, int par,
                        const void* in, void* out, const int* gate, hipStream_t st) {
  if (!total_units) return;
  dim3 grid(grid_for(total_units, 4)), block(256);
  switch (prec) {
    case P64: hipLaunchKernelGGL(k_site_factor<double>, grid, block, 0, st, slots, nslots, total_units, coef, par, in, out, gate); break;
    case P32: hipLaunchKernelGGL(k_site_factor<float>, grid, block, 0, st, slots, nslots, total_units, coef, par, in, out, gate); break;
    case PB16: hipLaunchKernelGGL(k_site_factor<bf16s>, grid, block, 0, st, slots, nslots, total_units, coef, par, in, out, gate); break;
    case PH16: hipLaunchKernelGGL(k_site_factor<f16s>, grid, block, 0, st, slots, nslots, total_units, coef, par, in, out, gate); break;
    default: throw std::runtime_error("bad precision");
  }
}

}  // namespace dl
