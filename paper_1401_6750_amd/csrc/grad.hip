// Backward pass of the loops: the insertion operator B + B^dag applied to the
// solutions, and the small reductions of the mu-derivative.
//
// With upstream gradient g = dF/dL^* and per-site spin matrices
//   Omega_{f,op}(x) = (pf_f / N) sum_n [sum_p conj(g[f,op,n,t,p]) e^{-ip.x}] Gamma_n
// (built by k_omega), every loop is s^dag B s with
//   B = gamma_5 Q_tau3 + M_0^dag Q_1,
//   Q_f = Omega_{f,0} + 1/2 sum_nu (Omega_{f,nu} D_nu + D_nu Omega_{f,nu}),
// D_nu the symmetric covariant derivative (anti-Hermitian).  k_insert_apply
// writes, per site and right-hand side,
//   A = Q_1 s,
//   C = gamma_5 Q_tau3 s + Q_tau3^dag (gamma_5 s) + Q_1 s + Q_1^dag (M_0 s),
// so that (B + B^dag) s = M_0^dag A + C - A... folded as C' below (one more
// hopping launch), together with per-unit partial sums of s^dag gamma_5 Q_tau3 s.
//
// In terms of the colour-transported neighbours T+ = U_nu(x) u(x+nu) b+,
// T- = U_nu(x-nu)^dag u(x-nu) b- (b+- the time-boundary factors):
//   (Q u)_nu     = 1/4 [Omega(x)(T+ - T-) + Omega(x+nu) T+ - Omega(x-nu) T-]
//   (Q^dag u)_nu = -1/4 [Omega(x+nu)^dag T+ - Omega(x-nu)^dag T- + Omega(x)^dag (T+ - T-)]
// (spin matrices commute with the colour transport).
#include <stdexcept>

#include "kernels.h"

namespace dl {

// out += sign * M u for a 4x4 spin matrix (complex128 entries, or their
// adjoint when DAG) acting on a colour-spinor; G5: on gamma_5 u instead (the
// sign of spins 2, 3 flipped, exactly as a negated copy of u would give, with
// no copy held in registers).
template <bool DAG, bool G5 = false>
__device__ inline void spin_mat_acc(const double2 (&m)[16], const cx<double> (&u)[12], double sign,
                                    cx<double> (&out)[12]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double2 e = DAG ? m[4 * b + a] : m[4 * a + b];
      const cx<double> w = DAG ? mk<double>(e.x, -e.y) : mk<double>(e.x, e.y);
      const double sb = (G5 && b >= 2) ? -sign : sign;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[3 * a + c] = out[3 * a + c] + sb * (w * u[3 * b + c]);
    }
}

__device__ inline void load_omega(const double2* om, long long V, long long site, double2 (&m)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) m[e] = om[e * V + site];
}

__device__ inline void g5(cx<double> (&v)[12]) {
#pragma unroll
  for (int k = 6; k < 12; ++k) v[k] = mk<double>(-v[k].re, -v[k].im);
}

// transported neighbours along nu for one field (FP64 batch field of the
// other parity): tp = U(x) u(x+nu) bp, tm = U(x-nu)^dag u(x-nu) bm
__device__ inline void transport(const void* f_other, long vp, int sp, int sm, double bp, double bm,
                                 const cx<double> (&up)[9], const cx<double> (&um)[9], cx<double> (&tp)[12],
                                 cx<double> (&tm)[12]) {
  cx<double> v[12];
  load_spinor<double>(f_other, vp, sp, v);
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<double> f = mk<double>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac(f, up[3 * a + k], v[3 * s4 + k]);
      tp[3 * s4 + a] = bp * f;
    }
  load_spinor<double>(f_other, vp, sm, v);
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<double> b = mk<double>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cjmac(b, um[3 * k + a], v[3 * s4 + k]);
      tm[3 * s4 + a] = bm * b;
    }
}

__global__ __launch_bounds__(256) void k_insert_apply(const SlotDesc* slots, int nslots, int total_units, int p_out,
                                                      int nops, const double2* omega, const void* s_e,
                                                      const void* s_o, const void* m_e, const void* m_o,
                                                      void* a_out, void* c_out, double* part_re,
                                                      double* part_im) {
  const int u = wave_unit();
  if (u >= total_units) return;
  const int lane = threadIdx.x & 63;
  const int si = find_slot(slots, nslots, UK_RHS, u);
  const SlotDesc& sd = slots[si];
  const int ul = u - sd.ubeg[UK_RHS];
  const int tile = ul / sd.nrhs;
  const int r = ul - tile * sd.nrhs;
  const int s = tile * TILE + lane;
  const long vh = sd.Vh;                 // Omega: [..][V] over par * Vh + s
  const long vp = sd.Vp;                 // fields and links: padded rows
  const long long V = 2ll * vh;
  const long long off = sd.fo + (long long)r * vp;
  double dre = 0.0, dim = 0.0;
  if (s < sd.Vh) {
    const int par = p_out;
    const long long site = (long long)par * vh + s;
    const void* s_here = field_at<double>(par ? s_o : s_e, off);
    const void* s_oth = field_at<double>(par ? s_e : s_o, off);
    const void* m_here = field_at<double>(par ? m_o : m_e, off);
    const void* m_oth = field_at<double>(par ? m_e : m_o, off);
    cx<double> sv[12], mv[12];
    load_spinor<double>(s_here, vp, s, sv);
    load_spinor<double>(m_here, vp, s, mv);
    cx<double> qt3[12], A[12], C[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) qt3[k] = A[k] = C[k] = mk<double>(0, 0);
    const double2* om_t3 = omega;                           // [op][16][V]
    const double2* om_1 = omega + (long long)nops * 16 * V;
    double2 w[16];
    // local parts
    load_omega(om_t3, V, site, w);
    spin_mat_acc<false>(w, sv, 1.0, qt3);
    spin_mat_acc<true, true>(w, sv, 1.0, C);
    load_omega(om_1, V, site, w);
    spin_mat_acc<false>(w, sv, 1.0, A);
    spin_mat_acc<true>(w, mv, 1.0, C);
    if (nops > 1) {
      const Coords c = eo_coords(sd, s, par);
      const int ext[4] = {sd.X, sd.Y, sd.Z, sd.T};
      const void* g64 = sd.gauge[P64];
      for (int nu = 0; nu < 4; ++nu) {
        int xp[4] = {c.x, c.y, c.z, c.t}, xm[4] = {c.x, c.y, c.z, c.t};
        double bp = 1.0, bm = 1.0;
        xp[nu] += 1;
        if (xp[nu] == ext[nu]) { xp[nu] = 0; if (nu == 3) bp = sd.bc; }
        xm[nu] -= 1;
        if (xm[nu] < 0) { xm[nu] = ext[nu] - 1; if (nu == 3) bm = sd.bc; }
        const int sp = eo_index(sd, xp[0], xp[1], xp[2], xp[3]);
        const int sm = eo_index(sd, xm[0], xm[1], xm[2], xm[3]);
        const long long site_p = (long long)(1 - par) * vh + sp, site_m = (long long)(1 - par) * vh + sm;
        cx<double> up[9], um[9];
        load_link<double>(g64, vp, nu, par, s, up);
        load_link<double>(g64, vp, nu, 1 - par, sm, um);
        cx<double> tp[12], tm[12], dt[12];
        transport(s_oth, vp, sp, sm, bp, bm, up, um, tp, tm);
#pragma unroll
        for (int k = 0; k < 12; ++k) dt[k] = tp[k] - tm[k];
        // tau_3 flavour: Q s and Q^dag (gamma5 s); gamma5 commutes with the transport
        const double2* o3 = om_t3 + (long long)(1 + nu) * 16 * V;
        load_omega(o3, V, site, w);
        spin_mat_acc<false>(w, dt, 0.25, qt3);
        spin_mat_acc<true, true>(w, dt, -0.25, C);
        load_omega(o3, V, site_p, w);
        spin_mat_acc<false>(w, tp, 0.25, qt3);
        spin_mat_acc<true, true>(w, tp, -0.25, C);
        load_omega(o3, V, site_m, w);
        spin_mat_acc<false>(w, tm, -0.25, qt3);
        spin_mat_acc<true, true>(w, tm, 0.25, C);
        // no-tau_3 flavour: Q_1 s into A, Q_1^dag (M_0 s) into C
        const double2* o1 = om_1 + (long long)(1 + nu) * 16 * V;
        load_omega(o1, V, site, w);
        spin_mat_acc<false>(w, dt, 0.25, A);
        load_omega(o1, V, site_p, w);
        spin_mat_acc<false>(w, tp, 0.25, A);
        load_omega(o1, V, site_m, w);
        spin_mat_acc<false>(w, tm, -0.25, A);
        transport(m_oth, vp, sp, sm, bp, bm, up, um, tp, tm);
#pragma unroll
        for (int k = 0; k < 12; ++k) dt[k] = tp[k] - tm[k];
        load_omega(o1, V, site, w);
        spin_mat_acc<true>(w, dt, -0.25, C);
        load_omega(o1, V, site_p, w);
        spin_mat_acc<true>(w, tp, -0.25, C);
        load_omega(o1, V, site_m, w);
        spin_mat_acc<true>(w, tm, 0.25, C);
      }
    }
    // C += gamma5 Q_tau3 s + Q_1 s;  reduction s^dag gamma5 Q_tau3 s
    cx<double> q5[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) q5[k] = qt3[k];
    g5(q5);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      C[k] = C[k] + q5[k] + A[k];
      dre += sv[k].re * q5[k].re + sv[k].im * q5[k].im;
      dim += sv[k].re * q5[k].im - sv[k].im * q5[k].re;
    }
    store_spinor<double>(field_at<double>(a_out, off), vp, s, A);
    store_spinor<double>(field_at<double>(c_out, off), vp, s, C);
  }
  dre = wave_sum(dre);
  dim = wave_sum(dim);
  if (lane == 0) {
    part_re[u] = dre;
    part_im[u] = dim;
  }
}

void launch_insert_apply(const SlotDesc* slots, int nslots, int total_units, int p_out, int nops,
                         const double* omega, const void* s_e, const void* s_o, const void* m_e, const void* m_o,
                         void* a_out, void* c_out, double* part_re, double* part_im, hipStream_t st) {
  if (!total_units) return;
  hipLaunchKernelGGL(k_insert_apply, dim3((total_units + 3) / 4), dim3(256), 0, st, slots, nslots, total_units,
                     p_out, nops, (const double2*)omega, s_e, s_o, m_e, m_o, a_out, c_out, part_re, part_im);
}

// z = gamma5 z' on complex128 [n sites][4][3] arrays; with dot != null also the
// per-block partial sums of conj(s) . z' (256 sites per block)
__global__ __launch_bounds__(256) void k_g5_lex(const double2* zin, double2* zout, const double2* s, long long nsite,
                                                double* part_re, double* part_im) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double dre = 0.0, dim = 0.0;
  if (i < nsite) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double2 z = zin[i * 12 + k];
      if (s) {
        const double2 a = s[i * 12 + k];
        dre += a.x * z.x + a.y * z.y;
        dim += a.x * z.y - a.y * z.x;
      }
      zout[i * 12 + k] = k < 6 ? z : make_double2(-z.x, -z.y);
    }
  }
  if (part_re) {
    __shared__ double red[2][4];
    dre = wave_sum(dre);
    dim = wave_sum(dim);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][wv] = dre; red[1][wv] = dim; }
    __syncthreads();
    if (threadIdx.x == 0) {
      part_re[blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      part_im[blockIdx.x] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
  }
}

void launch_g5_lex(const double* zin, double* zout, const double* s, long long nsite, double* part_re,
                   double* part_im, hipStream_t st) {
  if (nsite <= 0) return;
  const unsigned blocks = (unsigned)((nsite + 255) / 256);
  hipLaunchKernelGGL(k_g5_lex, dim3(blocks), dim3(256), 0, st, (const double2*)zin, (double2*)zout,
                     (const double2*)s, nsite, part_re, part_im);
}

// Fixed-order sum of n partials into out[0] (one workgroup).
__global__ __launch_bounds__(256) void k_sum(const double* part, long long n, double* out) {
  __shared__ double red[4];
  double v = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

void launch_sum(const double* part, long long n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, part, n, out);
}

}  // namespace dl
