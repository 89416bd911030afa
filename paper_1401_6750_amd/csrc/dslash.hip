// Even-odd twisted-mass Wilson hopping kernel with fused site-local epilogues.
//
// One wavefront handles one unit = 64 consecutive even-odd sites of G right-
// hand sides of one batch slot (G = rhs_per_wave, two for every storage
// precision by default): the site coordinates, the eight neighbour indices
// and every gauge link are computed / loaded once and used for all G
// right-hand sides.  Units of one tile are consecutive for all right-hand-side
// groups of the slot, tiles are visited in time-blocked order (tile_of), and
// each XCD receives a contiguous range of units, so a tile's links are
// fetched once into that XCD's L2.  In 16-bit storage the design minimises
// per-(site, rhs) work that is not arithmetic of the hop: the colour
// products run on the packed 16-bit words (dot2) with every sign taken as an
// input modifier, conversions use the packed hardware converts, neighbour
// indices are offsets of the lexicographic index.
//
// Operator pieces (kappa normalised, chiral basis, gamma_5 = diag(1,1,-1,-1)):
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)
// In FP32 / FP64 a hop through (1 -+ gamma_mu) is done on the two independent
// spin combinations h0, h1 (colour vectors) and the lower two spin components
// are rebuilt from them, so each neighbour costs two SU(3) x colour products;
// the 16-bit path multiplies all four spin components (see hop).
//
// Epilogue (per-spin complex factors, set per slot):
//   res = e (.) H(d (.) in) + f (.) y,   out = g (.) res
// optionally followed by the CG residual update r -= alpha res (x takes its
// step alpha p in update_p).
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

// Accumulate the full four-spinor rebuilt from the projected pair (w0, w1),
// times the hop's boundary factor `sign` (used for MU = 3 only, folded into
// the adds as FMAs).  INIT: the first hop of a site assigns instead of adding.
template <int MU, bool FWD, bool INIT, class R>
__device__ inline void reconstruct(cx<R> (&acc)[12], const cx<R> (&w0)[3], const cx<R> (&w1)[3], R sign) {
  auto put = [&](cx<R>& a, cx<R> w) {
    if (INIT) a = w; else a = a + w;
  };
  auto put_s = [&](cx<R>& a, cx<R> w, R f) {   // a (+)= f w
    if (INIT) a = f * w; else a = mk<R>(fmadd(f, w.re, a.re), fmadd(f, w.im, a.im));
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {
      put(acc[c], w0[c]);
      put(acc[3 + c], w1[c]);
      put(acc[6 + c], FWD ? times_mi(w1[c]) : times_i(w1[c]));
      put(acc[9 + c], FWD ? times_mi(w0[c]) : times_i(w0[c]));
    } else if (MU == 1) {
      put(acc[c], w0[c]);
      put(acc[3 + c], w1[c]);
      if (INIT) {
        acc[6 + c] = FWD ? mk<R>(-w1[c].re, -w1[c].im) : w1[c];
        acc[9 + c] = FWD ? w0[c] : mk<R>(-w0[c].re, -w0[c].im);
      } else {
        acc[6 + c] = FWD ? acc[6 + c] - w1[c] : acc[6 + c] + w1[c];
        acc[9 + c] = FWD ? acc[9 + c] + w0[c] : acc[9 + c] - w0[c];
      }
    } else if (MU == 2) {
      put(acc[c], w0[c]);
      put(acc[3 + c], w1[c]);
      put(acc[6 + c], FWD ? times_mi(w0[c]) : times_i(w0[c]));
      put(acc[9 + c], FWD ? times_i(w1[c]) : times_mi(w1[c]));
    } else {
      const R ms = -sign;
      put_s(acc[c], w0[c], sign);
      put_s(acc[3 + c], w1[c], sign);
      put_s(acc[6 + c], w0[c], FWD ? ms : sign);
      put_s(acc[9 + c], w1[c], FWD ? ms : sign);
    }
  }
}


// reconstruct() for one colour row c.
template <int MU, bool FWD, bool INIT, class R>
__device__ inline void reconstruct_row(cx<R> (&acc)[12], int c, cx<R> w0, cx<R> w1, R sign) {
  auto put = [&](int idx, cx<R> w) {
    if (INIT) acc[idx] = w; else acc[idx] = acc[idx] + w;
  };
  auto put_s = [&](int idx, cx<R> w, R f) {
    if (INIT) acc[idx] = f * w; else acc[idx] = mk<R>(fmadd(f, w.re, acc[idx].re), fmadd(f, w.im, acc[idx].im));
  };
  if (MU == 0) {
    put(c, w0);
    put(3 + c, w1);
    put(6 + c, FWD ? times_mi(w1) : times_i(w1));
    put(9 + c, FWD ? times_mi(w0) : times_i(w0));
  } else if (MU == 1) {
    put(c, w0);
    put(3 + c, w1);
    if (INIT) {
      acc[6 + c] = FWD ? mk<R>(-w1.re, -w1.im) : w1;
      acc[9 + c] = FWD ? w0 : mk<R>(-w0.re, -w0.im);
    } else {
      acc[6 + c] = FWD ? acc[6 + c] - w1 : acc[6 + c] + w1;
      acc[9 + c] = FWD ? acc[9 + c] + w0 : acc[9 + c] - w0;
    }
  } else if (MU == 2) {
    put(c, w0);
    put(3 + c, w1);
    put(6 + c, FWD ? times_mi(w0) : times_i(w0));
    put(9 + c, FWD ? times_i(w1) : times_mi(w1));
  } else {
    const R ms = -sign;
    put_s(c, w0, sign);
    put_s(3 + c, w1, sign);
    put_s(6 + c, w0, FWD ? ms : sign);
    put_s(9 + c, w1, FWD ? ms : sign);
  }
}

// Spin projection of one hop as (h0, h1) = (psi_0 + c0 psi_B0, psi_1 + c1 psi_B1),
// c in {+1, -1, +i, -i} coded 0..3 (the same combinations as project()).
template <int MU, bool FWD> struct ProjSpec;
template <> struct ProjSpec<0, true> { static constexpr int b0 = 3, c0 = 2, b1 = 2, c1 = 2; };
template <> struct ProjSpec<0, false> { static constexpr int b0 = 3, c0 = 3, b1 = 2, c1 = 3; };
template <> struct ProjSpec<1, true> { static constexpr int b0 = 3, c0 = 0, b1 = 2, c1 = 1; };
template <> struct ProjSpec<1, false> { static constexpr int b0 = 3, c0 = 1, b1 = 2, c1 = 0; };
template <> struct ProjSpec<2, true> { static constexpr int b0 = 2, c0 = 2, b1 = 3, c1 = 3; };
template <> struct ProjSpec<2, false> { static constexpr int b0 = 2, c0 = 3, b1 = 3, c1 = 2; };
template <> struct ProjSpec<3, true> { static constexpr int b0 = 2, c0 = 1, b1 = 3, c1 = 1; };
template <> struct ProjSpec<3, false> { static constexpr int b0 = 2, c0 = 0, b1 = 3, c1 = 0; };

// One hop (direction MU, forward or backward) for every right-hand side of
// the group, unpacked arithmetic: FP32 / FP64 storage, and 16-bit storage with
// the input factor d.  The link is loaded once; the spin projection comes
// first and two colour vectors are multiplied.
template <class S, int MU, bool FWD, bool HAS_D, bool INIT, bool TWO, int G>
__device__ inline void hop(const void* gauge, long vp, int link_par, int link_site, int nb, typename Traits<S>::R sign,
                           const void* const (&ld)[G], int nr, const bool (&act)[G],
                           const cx<typename Traits<S>::R> (&d)[4], cx<typename Traits<S>::R> (&acc)[G][12]) {
  using R = typename Traits<S>::R;
  cx<R> u[9];
  if constexpr (TWO) load_link_2row(gauge, vp, MU, link_par, link_site, u);
  else load_link<S>(gauge, vp, MU, link_par, link_site, u);
  // 16-bit fields (this path: hops with an input factor): every member's
  // neighbour row is requested with the link, without a branch (an inactive
  // member reads an active member's row, `ld`), so the hop waits once for all
  // of them (8.6 -> 8.3 ms per 525-rhs launch); FP32 and FP64 rows are loaded
  // member by member (preloading made the FP32 hop 2.5 % slower)
  constexpr bool PRE = Traits<S>::NC == 3;
  cx<R> vpre[PRE ? G : 1][12];
  if constexpr (PRE) {
#pragma unroll
    for (int i = 0; i < G; ++i) load_spinor<S>(ld[i], vp, nb, vpre[i]);
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    if (i >= nr || !act[i]) continue;
    cx<R> v[12];
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = vpre[i][k];
    } else {
      load_spinor<S>(ld[i], vp, nb, v);
    }
    if (HAS_D) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = d[k / 3] * v[k];
    }
    cx<R> h0[3], h1[3], w0[3], w1[3];
    project<MU, FWD>(v, h0, h1);
    if (FWD) {
      su3_mul(u, h0, w0);
      su3_mul(u, h1, w1);
    } else {
      su3_dag_mul(u, h0, w0);
      su3_dag_mul(u, h1, w1);
    }
    reconstruct<MU, FWD, INIT>(acc[i], w0, w1, sign);
  }
}

// The eight hops of a site in the order x+, x-, y+, ..., t- (nbr: neighbour
// sites in that order), unpacked arithmetic.  TWO (FP32 storage, SU(3)
// links): rows 0 and 1 of each link (its first three chunks) are loaded and
// row 2 rebuilt, 3 link loads per hop instead of 5.
template <class S, bool HD, bool TWO, int G>
__device__ __forceinline__ void hops_unpacked(const void* gauge, long vp, int p_out, int s, const int (&nbr)[8],
                                              typename Traits<S>::R sp, typename Traits<S>::R sm,
                                              const void* const (&ld)[G], int nr, const bool (&act)[G],
                                              const cx<typename Traits<S>::R> (&d)[4],
                                              cx<typename Traits<S>::R> (&acc)[G][12]) {
  using R = typename Traits<S>::R;
  const int q = 1 - p_out;
  hop<S, 0, true, HD, true, TWO>(gauge, vp, p_out, s, nbr[0], (R)1, ld, nr, act, d, acc);
  hop<S, 0, false, HD, false, TWO>(gauge, vp, q, nbr[1], nbr[1], (R)1, ld, nr, act, d, acc);
  hop<S, 1, true, HD, false, TWO>(gauge, vp, p_out, s, nbr[2], (R)1, ld, nr, act, d, acc);
  hop<S, 1, false, HD, false, TWO>(gauge, vp, q, nbr[3], nbr[3], (R)1, ld, nr, act, d, acc);
  hop<S, 2, true, HD, false, TWO>(gauge, vp, p_out, s, nbr[4], (R)1, ld, nr, act, d, acc);
  hop<S, 2, false, HD, false, TWO>(gauge, vp, q, nbr[5], nbr[5], (R)1, ld, nr, act, d, acc);
  hop<S, 3, true, HD, false, TWO>(gauge, vp, p_out, s, nbr[6], sp, ld, nr, act, d, acc);
  hop<S, 3, false, HD, false, TWO>(gauge, vp, q, nbr[7], nbr[7], sm, ld, nr, act, d, acc);
}

// ---- software-pipelined 16-bit hops ---------------------------------------
// The words one hop needs (link chunks, neighbour spinor of every group
// member) are loaded one hop ahead of the arithmetic that uses them, so a
// wave has the next hop's loads in flight while it computes the current one.
template <int G>
struct HopWords {
  uint32_t e[9];
  uint32_t v[G][12];
};

// NINE: the ninth link entry is `nine` (fetched with those of the site's other
// forward links) instead of a load of its own.
template <int MU, bool NINE, int G>
__device__ inline void hop_load16(HopWords<G>& h, const void* gauge, long vp, int link_par, int link_site, int nb,
                                  const void* const (&inb)[G], uint32_t nine) {
  const long long lr = (MU * 2 + link_par) * 3;
  const uint4 l0 = at16<uint4>(row16(gauge, lr, vp), link_site), l1 = at16<uint4>(row16(gauge, lr + 1, vp), link_site);
  h.e[0] = l0.x; h.e[1] = l0.y; h.e[2] = l0.z; h.e[3] = l0.w;
  h.e[4] = l1.x; h.e[5] = l1.y; h.e[6] = l1.z; h.e[7] = l1.w;
  if constexpr (NINE) h.e[8] = nine;
  else h.e[8] = at16<uint4>(row16(gauge, lr + 2, vp), link_site).x;
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint4 q0 = at16<uint4>(inb[i], nb), q1 = at16<uint4>(row16(inb[i], 1, vp), nb),
                q2 = at16<uint4>(row16(inb[i], 2, vp), nb);
    h.v[i][0] = q0.x; h.v[i][1] = q0.y; h.v[i][2] = q0.z; h.v[i][3] = q0.w;
    h.v[i][4] = q1.x; h.v[i][5] = q1.y; h.v[i][6] = q1.z; h.v[i][7] = q1.w;
    h.v[i][8] = q2.x; h.v[i][9] = q2.y; h.v[i][10] = q2.z; h.v[i][11] = q2.w;
  }
}

// Two-row links (SU(3)): rows 0 and 1 of two directions from three chunks of
// the site-centred rows (LINK_ROW_R12), forward (BWD = 0) or backward.
struct Link12 {
  uint32_t w[12];
};
__device__ inline void load_link12(Link12& L, const void* gauge, long vp, int par, int bwd, int pair, int s) {
  const long long r = LINK_ROW_R12 + 12 * par + 6 * bwd + 3 * pair;
  const uint4 a = at16<uint4>(row16(gauge, r, vp), s), b = at16<uint4>(row16(gauge, r + 1, vp), s),
              c = at16<uint4>(row16(gauge, r + 2, vp), s);
  L.w[0] = a.x; L.w[1] = a.y; L.w[2] = a.z; L.w[3] = a.w;
  L.w[4] = b.x; L.w[5] = b.y; L.w[6] = b.z; L.w[7] = b.w;
  L.w[8] = c.x; L.w[9] = c.y; L.w[10] = c.z; L.w[11] = c.w;
}
// The words of one hop from a two-row pair (direction M of the pair) and the
// neighbour spinor of every group member.
template <int G>
__device__ inline void hop_load12(HopWords<G>& h, const Link12& L, int m, long vp, int nb,
                                  const void* const (&inb)[G]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) h.e[k] = L.w[6 * m + k];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint4 q0 = at16<uint4>(inb[i], nb), q1 = at16<uint4>(row16(inb[i], 1, vp), nb),
                q2 = at16<uint4>(row16(inb[i], 2, vp), nb);
    h.v[i][0] = q0.x; h.v[i][1] = q0.y; h.v[i][2] = q0.z; h.v[i][3] = q0.w;
    h.v[i][4] = q1.x; h.v[i][5] = q1.y; h.v[i][6] = q1.z; h.v[i][7] = q1.w;
    h.v[i][8] = q2.x; h.v[i][9] = q2.y; h.v[i][10] = q2.z; h.v[i][11] = q2.w;
  }
}
// Row 2 of an SU(3) link from rows 0 and 1: the rows are orthonormal and the
// determinant is one, so row 2 is the complex conjugate of the cross product
// of rows 0 and 1, u2_k = conj(u0_i u1_j - u0_j u1_i), (i, j, k) cyclic.
// Each part is a chain of two dot2 products on the stored words (exact
// products, FP32 sums; signs by input modifiers, the imaginary part against
// the half-swapped words of row 1), rounded to the storage format as a stored
// entry is:
//   Re = (Re a_i, -Im a_i) . b_j + (-Re a_j, Im a_j) . b_i
//   Im = a_j . swap(b_i) - a_i . swap(b_j)      (a = row 0, b = row 1)
template <class S>
__device__ inline void link_row2(uint32_t (&e)[9]) {
  uint32_t sb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) sb[k] = swap16(e[3 + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const float re = Chain2<S, 0, 1, 1, 0>::run(e[i], e[j], e[3 + j], e[3 + i]);
    const float im = Chain2<S, 0, 0, 1, 1>::run(e[j], e[i], sb[i], sb[j]);
    e[6 + k] = pack2<S>(mk<float>(re, im));
  }
}

// Coefficient operand of the packed colour products: the link word w (SW =
// false) or its half-swapped form (SW = true), with the signs of its low / high
// half flipped (NLO / NHI) by the dot2 input modifiers, so no instruction is
// spent on signs.  Row a of U (forward) or U^dag (backward):
//   forward:  cr = (Re U_ab, -Im U_ab) = w with NHI,  ci = (Im U_ab, Re U_ab) = swap(w)
//   backward: cr = (Re U_ba,  Im U_ba) = w,            ci = (-Im U_ba, Re U_ba) = swap(w) with NLO
// and the projection factors -1, +i, -i of the second spin component select
// -cr, -ci, ci for the real part (-ci, cr, -cr for the imaginary part).
template <bool SW, int NLO, int NHI>
struct Coef16 {
  static constexpr bool sw = SW;
  static constexpr int lo = NLO, hi = NHI;
};
template <class O> using NegOf = Coef16<O::sw, 1 - O::lo, 1 - O::hi>;
template <bool FWD> using CrOf = Coef16<false, 0, FWD ? 1 : 0>;
template <bool FWD> using CiOf = Coef16<true, FWD ? 0 : 1, 0>;
// projection code c (0: +1, 1: -1, 2: +i, 3: -i) -> operands of the real and imaginary part
template <int C, bool FWD>
using ProjRe = std::conditional_t<C == 0, CrOf<FWD>, std::conditional_t<C == 1, NegOf<CrOf<FWD>>,
               std::conditional_t<C == 2, NegOf<CiOf<FWD>>, CiOf<FWD>>>>;
template <int C, bool FWD>
using ProjIm = std::conditional_t<C == 0, CiOf<FWD>, std::conditional_t<C == 1, NegOf<CiOf<FWD>>,
               std::conditional_t<C == 2, CrOf<FWD>, NegOf<CrOf<FWD>>>>>;

// Re or Im of one colour row of M (h_a + c h_b): three products with the
// operand O1 on spin sa and three with O2 on spin sb.
template <class S, class O1, class O2>
__device__ inline float chain16(const uint32_t (&w)[3], const uint32_t (&sw)[3], const uint32_t (&v)[12], int sa,
                                int sb) {
  return Chain6<S, O1::lo, O1::hi, O2::lo, O2::hi>::run(
      O1::sw ? sw[0] : w[0], O1::sw ? sw[1] : w[1], O1::sw ? sw[2] : w[2], O2::sw ? sw[0] : w[0],
      O2::sw ? sw[1] : w[1], O2::sw ? sw[2] : w[2], v[3 * sa], v[3 * sa + 1], v[3 * sa + 2], v[3 * sb],
      v[3 * sb + 1], v[3 * sb + 2]);
}

// The arithmetic of one hop, one colour row a at a time (only that row's
// link words are live).
template <class S, int MU, bool FWD, bool INIT, int G>
__device__ inline void hop_compute16(const HopWords<G>& h, float sign, const bool (&act)[G],
                                     cx<float> (&acc)[G][12]) {
  using PS = ProjSpec<MU, FWD>;
  using Cr = CrOf<FWD>;
  using Ci = CiOf<FWD>;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uint32_t w[3], sw[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      w[b] = FWD ? h.e[3 * a + b] : h.e[3 * b + a];
      sw[b] = swap16(w[b]);
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (!act[i]) continue;
      const uint32_t (&v)[12] = h.v[i];
      const cx<float> w0 = mk<float>(chain16<S, Cr, ProjRe<PS::c0, FWD>>(w, sw, v, 0, PS::b0),
                                     chain16<S, Ci, ProjIm<PS::c0, FWD>>(w, sw, v, 0, PS::b0));
      const cx<float> w1 = mk<float>(chain16<S, Cr, ProjRe<PS::c1, FWD>>(w, sw, v, 1, PS::b1),
                                     chain16<S, Ci, ProjIm<PS::c1, FWD>>(w, sw, v, 1, PS::b1));
      reconstruct_row<MU, FWD, INIT>(acc[i], a, w0, w1, sign);
    }
  }
}

// The eight hops of a site on 16-bit fields, in the order x+, x-, y+, ..., t-,
// each hop's link and neighbour words loaded while the previous hop computes.
// TWO_ROW (SU(3) links): rows 0 and 1 of the eight links from the site-centred
// two-row copies, two directions per three loads, and row 2 rebuilt before
// each hop's arithmetic (12 link loads for the site instead of 18); otherwise
// all nine entries, the ninth of the four forward and of the four backward
// links from one load each.  nbr: neighbour sites in that order.
template <class S, bool TWO_ROW, int G>
__device__ __forceinline__ void hops16(const void* gauge, long vp, int p_out, int s, const int (&nbr)[8], float sp,
                                       float sm, const void* const (&ld)[G], const bool (&act)[G],
                                       cx<float> (&acc)[G][12]) {
  const int q = 1 - p_out;
  HopWords<G> h0, h1;
  if constexpr (TWO_ROW) {
    Link12 lf, lb;
    load_link12(lf, gauge, vp, p_out, 0, 0, s);
    load_link12(lb, gauge, vp, p_out, 1, 0, s);
    hop_load12(h0, lf, 0, vp, nbr[0], ld);
    hop_load12(h1, lb, 0, vp, nbr[1], ld);
    link_row2<S>(h0.e);
    hop_compute16<S, 0, true, true>(h0, 1.0f, act, acc);
    hop_load12(h0, lf, 1, vp, nbr[2], ld);
    link_row2<S>(h1.e);
    hop_compute16<S, 0, false, false>(h1, 1.0f, act, acc);
    hop_load12(h1, lb, 1, vp, nbr[3], ld);
    load_link12(lf, gauge, vp, p_out, 0, 1, s);
    load_link12(lb, gauge, vp, p_out, 1, 1, s);
    link_row2<S>(h0.e);
    hop_compute16<S, 1, true, false>(h0, 1.0f, act, acc);
    hop_load12(h0, lf, 0, vp, nbr[4], ld);
    link_row2<S>(h1.e);
    hop_compute16<S, 1, false, false>(h1, 1.0f, act, acc);
    hop_load12(h1, lb, 0, vp, nbr[5], ld);
    link_row2<S>(h0.e);
    hop_compute16<S, 2, true, false>(h0, 1.0f, act, acc);
    hop_load12(h0, lf, 1, vp, nbr[6], ld);
    link_row2<S>(h1.e);
    hop_compute16<S, 2, false, false>(h1, 1.0f, act, acc);
    hop_load12(h1, lb, 1, vp, nbr[7], ld);
    link_row2<S>(h0.e);
    hop_compute16<S, 3, true, false>(h0, sp, act, acc);
    link_row2<S>(h1.e);
    hop_compute16<S, 3, false, false>(h1, sm, act, acc);
  } else {
    const uint4 nf = at16<uint4>(row16(gauge, LINK_ROW_NINTH + p_out, vp), s);
    const uint4 nb = at16<uint4>(row16(gauge, LINK_ROW_NINTH_BWD + p_out, vp), s);
    hop_load16<0, true>(h0, gauge, vp, p_out, s, nbr[0], ld, nf.x);
    hop_load16<0, true>(h1, gauge, vp, q, nbr[1], nbr[1], ld, nb.x);
    hop_compute16<S, 0, true, true>(h0, 1.0f, act, acc);
    hop_load16<1, true>(h0, gauge, vp, p_out, s, nbr[2], ld, nf.y);
    hop_compute16<S, 0, false, false>(h1, 1.0f, act, acc);
    hop_load16<1, true>(h1, gauge, vp, q, nbr[3], nbr[3], ld, nb.y);
    hop_compute16<S, 1, true, false>(h0, 1.0f, act, acc);
    hop_load16<2, true>(h0, gauge, vp, p_out, s, nbr[4], ld, nf.z);
    hop_compute16<S, 1, false, false>(h1, 1.0f, act, acc);
    hop_load16<2, true>(h1, gauge, vp, q, nbr[5], nbr[5], ld, nb.z);
    hop_compute16<S, 2, true, false>(h0, 1.0f, act, acc);
    hop_load16<3, true>(h0, gauge, vp, p_out, s, nbr[6], ld, nf.w);
    hop_compute16<S, 2, false, false>(h1, 1.0f, act, acc);
    hop_load16<3, true>(h1, gauge, vp, q, nbr[7], nbr[7], ld, nb.w);
    hop_compute16<S, 3, true, false>(h0, sp, act, acc);
    hop_compute16<S, 3, false, false>(h1, sm, act, acc);
  }
}

// A per-spin factor in the compute precision (FP32 kernels take the host's
// FP32 rounding of the factor, the same value as converting it here).
__device__ inline void load_coef(const double (&c)[4][2], const float (&)[4][2], cx<double> (&out)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = mk<double>(c[k][0], c[k][1]);
}
__device__ inline void load_coef(const double (&)[4][2], const float (&c)[4][2], cx<float> (&out)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = mk<float>(c[k][0], c[k][1]);
}

// Site-local epilogue of a hop (see the file header): res = e (.) acc + f (.) y,
// then the CG residual update, the post factor, the norm partial and the stores.
template <class S, int F, int G>
__device__ __forceinline__ void dslash_epilogue(const DslashArgs& a, const SlotDesc& sd, const Coef& cf,
                                                const void* clv, int me, int mf, int mg, int p_out, long vp, int s,
                                                const long long (&off)[G], int r0, const bool (&act)[G],
                                                const cx<typename Traits<S>::R> (&e)[4],
                                                const cx<typename Traits<S>::R> (&f)[4],
                                                const cx<typename Traits<S>::R> (&g)[4],
                                                cx<typename Traits<S>::R> (&acc)[G][12], double (&nrm)[G]) {
  using R = typename Traits<S>::R;
  (void)cf;
  if constexpr ((F & F_CLV) != 0) {
    if (me >= 0) {
      cx<R> t[G][12];
      site_matvec<G>(clv, me, p_out, vp, s, acc, t, act);
#pragma unroll
      for (int i = 0; i < G; ++i)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[i][k] = t[i][k];
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    if (!act[i]) continue;
    cx<R> res[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) res[k] = e[k / 3] * acc[i][k];
    cx<R> yv[12];
    if (F & F_Y) {
      load_spinor<S>(field_at<S>(a.y, off[i]), vp, s, yv);
      if constexpr ((F & F_CLV) != 0) {
        if (mf >= 0) {
          cx<R> yi[1][12], yo[1][12];
          const bool one[1] = {true};
#pragma unroll
          for (int k = 0; k < 12; ++k) yi[0][k] = yv[k];
          site_matvec<1>(clv, mf, p_out, vp, s, yi, yo, one);
#pragma unroll
          for (int k = 0; k < 12; ++k) yv[k] = yo[0][k];
        }
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) res[k] = res[k] + f[k / 3] * yv[k];
    }
    if (F & F_XR) {
      const R al = (R)a.alpha[sd.rhs_begin + r0 + i];
      cx<R> rv[12];
      load_spinor<S>(field_at<S>(a.r, off[i]), vp, s, rv);
#pragma unroll
      for (int k = 0; k < 12; ++k) rv[k] = rv[k] - al * res[k];
      quantize<S>(rv);                       // the norm is that of the stored residual
      store_spinor<S>(field_at<S>(a.r, off[i]), vp, s, rv);
      if (F & F_NORM) nrm[i] = norm2(rv);
    } else {
      if (F & F_POST) {
        if (F & F_NORM) nrm[i] = norm2(res);  // norm before the post factor
        if constexpr ((F & F_CLV) != 0) {
          if (mg >= 0) {
            cx<R> ri[1][12], ro[1][12];
            const bool one[1] = {true};
#pragma unroll
            for (int k = 0; k < 12; ++k) ri[0][k] = res[k];
            site_matvec<1>(clv, mg, p_out, vp, s, ri, ro, one);
#pragma unroll
            for (int k = 0; k < 12; ++k) res[k] = ro[0][k];
          }
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) res[k] = g[k / 3] * res[k];
      } else if (F & F_NORM) {
        quantize<S>(res);                     // the norm of the stored values
        nrm[i] = norm2(res);
      }
      store_spinor<S>(field_at<S>(a.out, off[i]), vp, s, res);
      if (F & F_OUT2) store_spinor<S>(field_at<S>(a.out2, off[i]), vp, s, res);
      if (F & F_DUAL) {
        // second epilogue on the same hop: g (.) H + f (.) y  (y is in yv)
        cx<R> res2[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) res2[k] = g[k / 3] * acc[i][k] + f[k / 3] * yv[k];
        store_spinor<S>(field_at<S>(a.out2, off[i]), vp, s, res2);
      }
    }
  }
}

template <class S, int F>
__global__ __launch_bounds__(256) void k_dslash(DslashArgs a) {
  using R = typename Traits<S>::R;
  constexpr int G = rhs_per_wave<S>();
  constexpr int UK = unit_kind_for_group(G);
  const int u = wave_unit();
  if (u >= a.total_units) return;
  const int lane = threadIdx.x & 63;
  const int si = find_slot(a.slots, a.nslots, UK, u);
  const SlotDesc& sd = a.slots[si];
  // the F_CLV instance runs the slots with a clover term, the plain one the
  // others, so a slot's arithmetic never depends on what shares its batch
  if (((F & F_CLV) != 0) != (sd.clv64 != nullptr)) return;
  const int ngrp = (sd.nrhs + G - 1) / G;
  const int ul = u - sd.ubeg[UK];
  const int lt = ul / ngrp;
  const int tile = tile_of(sd, lt);
  const int r0 = (ul - lt * ngrp) * G;
  const int nr = min(G, sd.nrhs - r0);
  bool act[G];
  bool any = false;
#pragma unroll
  for (int i = 0; i < G; ++i) {
    act[i] = i < nr && (!a.active || a.active[sd.rhs_begin + r0 + i]);
    any = any || act[i];
  }
  if (!any) return;
  const int s = tile * TILE + lane;
  const bool valid = s < sd.Vh;
  const long vp = sd.Vp;   // row stride of fields and link chunk rows
  long long off[G];
#pragma unroll
  for (int i = 0; i < G; ++i) off[i] = sd.fo + (long long)(r0 + i) * vp;
  double nrm[G];
#pragma unroll
  for (int i = 0; i < G; ++i) nrm[i] = 0.0;
  if (valid) {
    const Coef& cf = a.coef[si];
    cx<R> d[4], e[4], f[4], g[4];
    load_coef(cf.d, cf.d32, d);
    load_coef(cf.e, cf.e32, e);
    load_coef(cf.f, cf.f32, f);
    load_coef(cf.g, cf.g32, g);
    const int p_out = a.p_out;
    // clover slots: the site matrices of e, f, g (kind per factor, -1 none);
    // d was applied to the input beforehand (launch_site_factor)
    const void* clv = nullptr;
    int me = -1, mf = -1, mg = -1;
    if constexpr ((F & F_CLV) != 0) {
      clv = Traits<S>::prec == P64 ? sd.clv64 : sd.clv32;
      if (clv) {
        me = cf.m[1];
        mf = cf.m[2];
        mg = cf.m[3];
        if (cf.m[0] >= 0)
#pragma unroll
          for (int k = 0; k < 4; ++k) d[k] = mk<R>((R)1, (R)0);
      }
    }
    const Coords c = eo_coords(sd, s, p_out);
    // neighbour even-odd indices from the lexicographic index: a step along
    // y, z or t moves lex by an even stride, one along x flips the parity bit
    const int X = sd.X, XY = sd.X * sd.Y, XYZ = XY * sd.Z;
    const int lex = c.x + X * c.y + XY * c.z + XYZ * c.t;
    const int nxp = (c.x + 1 == sd.X ? lex - (X - 1) : lex + 1) >> 1;
    const int nxm = (c.x == 0 ? lex + (X - 1) : lex - 1) >> 1;
    const int nyp = (c.y + 1 == sd.Y ? lex - (XY - X) : lex + X) >> 1;
    const int nym = (c.y == 0 ? lex + (XY - X) : lex - X) >> 1;
    const int nzp = (c.z + 1 == sd.Z ? lex - (XYZ - XY) : lex + XY) >> 1;
    const int nzm = (c.z == 0 ? lex + (XYZ - XY) : lex - XY) >> 1;
    const int VV = XYZ * sd.T;
    const int ntp = (c.t + 1 == sd.T ? lex - (VV - XYZ) : lex + XYZ) >> 1;
    const int ntm = (c.t == 0 ? lex + (VV - XYZ) : lex - XYZ) >> 1;
    const R sp = (c.t + 1 == sd.T) ? (R)sd.bc : (R)1;
    const R sm = (c.t == 0) ? (R)sd.bc : (R)1;
    const void* gauge = sd.gauge[Traits<S>::prec];
    const void* inb[G];
#pragma unroll
    for (int i = 0; i < G; ++i) inb[i] = field_at<S>(a.in, off[i]);
    // set by the first hop of every active member; an inactive member skips
    // every hop and its accumulator is never read
    cx<R> acc[G][12];
    constexpr bool HD = (F & F_D) != 0;
    const int q = 1 - p_out;
    // members that are inactive read the first active member's field
    const void* fa = nullptr;
#pragma unroll
    for (int i = G - 1; i >= 0; --i)
      if (act[i]) fa = inb[i];
    const void* ld[G];
#pragma unroll
    for (int i = 0; i < G; ++i) ld[i] = act[i] ? inb[i] : fa;
    if constexpr (Traits<S>::NC == 3 && !HD) {
      const int nbr[8] = {nxp, nxm, nyp, nym, nzp, nzm, ntp, ntm};
      if (sd.two_row & TWO_ROW_16) hops16<S, true>(gauge, vp, p_out, s, nbr, (float)sp, (float)sm, ld, act, acc);
      else hops16<S, false>(gauge, vp, p_out, s, nbr, (float)sp, (float)sm, ld, act, acc);
    } else {
    const int nbr[8] = {nxp, nxm, nyp, nym, nzp, nzm, ntp, ntm};
    if constexpr (Traits<S>::prec == P32) {
      if (sd.two_row & TWO_ROW_32) hops_unpacked<S, HD, true>(gauge, vp, p_out, s, nbr, sp, sm, ld, nr, act, d, acc);
      else hops_unpacked<S, HD, false>(gauge, vp, p_out, s, nbr, sp, sm, ld, nr, act, d, acc);
    } else {
      hops_unpacked<S, HD, false>(gauge, vp, p_out, s, nbr, sp, sm, ld, nr, act, d, acc);
    }
    }
    dslash_epilogue<S, F, G>(a, sd, cf, clv, me, mf, mg, p_out, vp, s, off, r0, act, e, f, g, acc, nrm);
  }
  if (F & F_NORM) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (i >= nr) break;
      const double t = wave_sum(nrm[i]);
      if (lane == 0 && act[i]) a.partial[sd.ubeg[UK_RHS] + tile * sd.nrhs + r0 + i] = t;
    }
  }
}

// ---- LDS-staged 16-bit hop (option "block_hop"; the tile kernel is faster) ---
// One workgroup is one unit: a block of bby x bbz whole x-rows (y, z) at one
// time slice of one slot, two right-hand sides.  The input-parity rows of the
// block and its y / z halo rows are staged in LDS (whole rows, eight in flight
// per wave), so six of the eight neighbour spinors of an output site come from
// LDS; the t neighbours and the links are read from global memory as in
// k_dslash.  Thread tid < bby * bbz * Xh owns output site k = tid mod Xh of row
// tid / Xh; the per-site arithmetic is that of k_dslash (same hop order).  The
// norm partial of a (block, slice) goes to partial slot blk * T + t (a fixed
// summation order that depends on the lattice shape only).
// LDS word (rhs i, row R, chunk c, site k): ((i * nrows + R) * 3 + c) * Xh + k;
// rows: centre row r -> r (nc = bby * bbz, r = ry + bby rz), halo h -> nc + h:
// h < bbz y = y0 - 1, < 2 bbz y = y0 + bby (z = z0 + h mod bbz), < 2 bbz + bby
// z = z0 - 1, else z = z0 + bbz (y = y0 + h - 2 bbz (- bby)).
template <int MU, bool NINE, int G>
__device__ inline void hop_fill16(HopWords<G>& h, const void* gauge, long vp, int link_par, int link_site,
                                  const uint4* const (&src)[G], int cstride, uint32_t nine) {
  const long long lr = (MU * 2 + link_par) * 3;
  const uint4 l0 = at16<uint4>(row16(gauge, lr, vp), link_site), l1 = at16<uint4>(row16(gauge, lr + 1, vp), link_site);
  h.e[0] = l0.x; h.e[1] = l0.y; h.e[2] = l0.z; h.e[3] = l0.w;
  h.e[4] = l1.x; h.e[5] = l1.y; h.e[6] = l1.z; h.e[7] = l1.w;
  if constexpr (NINE) h.e[8] = nine;
  else h.e[8] = at16<uint4>(row16(gauge, lr + 2, vp), link_site).x;
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint4 q0 = src[i][0], q1 = src[i][cstride], q2 = src[i][2 * cstride];
    h.v[i][0] = q0.x; h.v[i][1] = q0.y; h.v[i][2] = q0.z; h.v[i][3] = q0.w;
    h.v[i][4] = q1.x; h.v[i][5] = q1.y; h.v[i][6] = q1.z; h.v[i][7] = q1.w;
    h.v[i][8] = q2.x; h.v[i][9] = q2.y; h.v[i][10] = q2.z; h.v[i][11] = q2.w;
  }
}

template <class S, int F>
__global__ __launch_bounds__(256) void k_dslash_blk(DslashArgs a) {
  static_assert(Traits<S>::NC == 3 && (F & (F_D | F_CLV)) == 0, "16-bit storage, no input factor, no clover");
  using R = typename Traits<S>::R;
  constexpr int G = 2;
  extern __shared__ uint4 lds[];
  __shared__ double red[4][G];
  const int u = xcd_logical_block();
  if (u >= a.total_units) return;
  const int si = find_slot(a.slots, a.nslots, UK_BLK, u);
  const SlotDesc& sd = a.slots[si];
  const int ngrp = (sd.nrhs + G - 1) / G;
  const int ul = u - sd.ubeg[UK_BLK];
  const int grp = ul % ngrp;
  const int nseg = sd.T / sd.bseg;
  const int seg = (ul / ngrp) % nseg;
  const int blk = ul / ngrp / nseg;
  const int r0 = grp * G;
  const int nr = min(G, sd.nrhs - r0);
  bool act[G];
  bool any = false;
#pragma unroll
  for (int i = 0; i < G; ++i) {
    act[i] = i < nr && (!a.active || a.active[sd.rhs_begin + r0 + i]);
    any = any || act[i];
  }
  if (!any) return;   // uniform over the workgroup
  const int X = sd.X, Y = sd.Y, Z = sd.Z, T = sd.T, Xh = sd.Xh;
  const int by = sd.bby, bz = sd.bbz;
  const int nby = Y / by;
  const int y0 = (blk % nby) * by, z0 = (blk / nby) * bz;
  const int nc = by * bz, nh = 2 * (by + bz), nrows = nc + nh;
  const long vp = sd.Vp;
  const int p_out = a.p_out, q = 1 - p_out;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const bool mine = tid < nc * Xh;
  const int rr = tid / Xh, k = tid - rr * Xh;
  const int ry = rr % by, rz = rr / by;
  const int y = y0 + ry, z = z0 + rz;
  long long off[G];
  const uint4* inb[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    off[i] = sd.fo + (long long)(r0 + i) * vp;
    inb[i] = (const uint4*)field_at<S>(a.in, off[i]);
  }
  const Coef& cf = a.coef[si];
  cx<R> e[4], f[4], g[4];
  load_coef(cf.e, cf.e32, e);
  load_coef(cf.f, cf.f32, f);
  load_coef(cf.g, cf.g32, g);
  const void* gauge = sd.gauge[Traits<S>::prec];
  const long ntile = sd.ntile;
  if ((F & F_NORM) && blk == 0 && seg == 0) {
    // partial slots beyond the blocks' (blk * T + t) range stay zero
    const long used = (long)(Y / by) * (Z / bz) * T;
    for (long j = used + tid; j < ntile; j += nthr)
#pragma unroll
      for (int i = 0; i < G; ++i)
        if (act[i]) a.partial[sd.ubeg[UK_RHS] + j * sd.nrhs + r0 + i] = 0.0;
  }
  // stage the centre rows of slice tc (with_c; `ring` 0) and the halo rows of
  // slice th (with_h); rows wrap periodically (the time-boundary factor belongs
  // to the hop, not to the stored values).  A wave loads whole rows, lane
  // l < 3 Xh taking chunk l / Xh of site l mod Xh; up to eight rows are loaded
  // before any of them is written to LDS.
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nthr >> 6;
  const int lc = lane / Xh, lk = lane - lc * Xh;
  const bool lane_ok = lane < 3 * Xh;
  const long lane_off = (long)lc * vp + lk;
  const int lane_lds = lc * Xh + lk;
  auto row_of = [&](int Rw, int tc, int th, int ring, long& eo, int& lrow) {
    int yy, zz, tt;
    if (Rw < nc) {
      yy = y0 + Rw % by;
      zz = z0 + Rw / by;
      tt = tc;
      lrow = ring * nc + Rw;
    } else {
      const int h = Rw - nc;
      tt = th;
      lrow = nc + h;
      if (h < bz) { yy = y0 - 1; zz = z0 + h; }
      else if (h < 2 * bz) { yy = y0 + by; zz = z0 + h - bz; }
      else if (h < 2 * bz + by) { yy = y0 + h - 2 * bz; zz = z0 - 1; }
      else { yy = y0 + h - 2 * bz - by; zz = z0 + bz; }
    }
    yy = (yy + Y) % Y;
    zz = (zz + Z) % Z;
    tt = (tt + T) % T;
    eo = (long)X * (yy + (long)Y * (zz + (long)Z * tt)) / 2;
  };
  auto stage = [&](int ring, int tc, bool with_c, int th, bool with_h) {
    const int rb = with_c ? 0 : nc, re = with_h ? nc + nh : nc;
    const int nrw = re - rb, total = G * nrw;
    auto fetch = [&](int it, uint4& v, int& dst) {
      dst = -1;
      if (it >= total) return;
      const int i = it >= nrw ? 1 : 0;   // G = 2; selects, not a dynamic array index
      if (!((i ? act[1] : act[0]) && lane_ok)) return;
      long eo;
      int lrow;
      row_of(rb + it - i * nrw, tc, th, ring, eo, lrow);
      v = (i ? inb[1] : inb[0])[lane_off + eo];
      dst = (i * nrows + lrow) * 3 * Xh + lane_lds;
    };
    for (int base = wv; base < total; base += 8 * nw) {
      uint4 v0, v1, v2, v3, v4, v5, v6, v7;
      int d0, d1, d2, d3, d4, d5, d6, d7;
      fetch(base, v0, d0);
      fetch(base + nw, v1, d1);
      fetch(base + 2 * nw, v2, d2);
      fetch(base + 3 * nw, v3, d3);
      fetch(base + 4 * nw, v4, d4);
      fetch(base + 5 * nw, v5, d5);
      fetch(base + 6 * nw, v6, d6);
      fetch(base + 7 * nw, v7, d7);
      if (d0 >= 0) lds[d0] = v0;
      if (d1 >= 0) lds[d1] = v1;
      if (d2 >= 0) lds[d2] = v2;
      if (d3 >= 0) lds[d3] = v3;
      if (d4 >= 0) lds[d4] = v4;
      if (d5 >= 0) lds[d5] = v5;
      if (d6 >= 0) lds[d6] = v6;
      if (d7 >= 0) lds[d7] = v7;
    }
  };
  // one time slice per workgroup: seg is the slice
  const int t = seg;
  stage(0, t, true, t, true);
  __syncthreads();
  const int XY = X * Y, XYZ = XY * Z, VV = XYZ * T;
  {
    double nrm[G];
#pragma unroll
    for (int i = 0; i < G; ++i) nrm[i] = 0.0;
    if (mine) {
      const int x = 2 * k + ((p_out + y + z + t) & 1);
      const int lex = x + X * y + XY * z + XYZ * t;
      const int s = lex >> 1;
      const int nxm = (x == 0 ? lex + (X - 1) : lex - 1) >> 1;
      const int nym = (y == 0 ? lex + (XY - X) : lex - X) >> 1;
      const int nzm = (z == 0 ? lex + (XYZ - XY) : lex - XY) >> 1;
      const int ntp = (t + 1 == T ? lex - (VV - XYZ) : lex + XYZ) >> 1;
      const int ntm = (t == 0 ? lex + (VV - XYZ) : lex - XYZ) >> 1;
      const float sp = (t + 1 == T) ? (float)sd.bc : 1.0f;
      const float sm = (t == 0) ? (float)sd.bc : 1.0f;
      auto row = [&](int i, int lrow, int kk) { return lds + ((i * nrows + lrow) * 3) * Xh + kk; };
      const int kxp = ((x + 1) % X) >> 1, kxm = ((x + X - 1) % X) >> 1;
      const int cr = rr;
      const int ryp = ry + 1 < by ? cr + 1 : nc + bz + rz;
      const int rym = ry > 0 ? cr - 1 : nc + rz;
      const int rzp = rz + 1 < bz ? cr + by : nc + 2 * bz + by + ry;
      const int rzm = rz > 0 ? cr - by : nc + 2 * bz + ry;
      const uint4* pxp[G]; const uint4* pxm[G]; const uint4* pyp[G]; const uint4* pym[G];
      const uint4* pzp[G]; const uint4* pzm[G];
      const void* ld[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        pxp[i] = row(i, cr, kxp); pxm[i] = row(i, cr, kxm);
        pyp[i] = row(i, ryp, k); pym[i] = row(i, rym, k);
        pzp[i] = row(i, rzp, k); pzm[i] = row(i, rzm, k);
      }
      // t neighbours from global memory; inactive members read the first active one's field
      {
        const void* fa = nullptr;
#pragma unroll
        for (int i = G - 1; i >= 0; --i)
          if (act[i]) fa = (const void*)inb[i];
#pragma unroll
        for (int i = 0; i < G; ++i) ld[i] = act[i] ? (const void*)inb[i] : fa;
      }
      const uint4 nf = at16<uint4>(row16(gauge, LINK_ROW_NINTH + p_out, vp), s);
      const uint4 nbw = at16<uint4>(row16(gauge, LINK_ROW_NINTH_BWD + p_out, vp), s);
      cx<float> acc[G][12];
      HopWords<G> h0, h1;
      // the hops in the tile kernel's order (x, y, z, t; per-site results are
      // the same bits: with SU(3) links row 2 is rebuilt from the stored rows
      // 0 and 1, the words the tile kernel reads from the two-row copies)
      const bool two = (sd.two_row & TWO_ROW_16) != 0;
      hop_fill16<0, true>(h0, gauge, vp, p_out, s, pxp, Xh, nf.x);
      hop_fill16<0, true>(h1, gauge, vp, q, nxm, pxm, Xh, nbw.x);
      if (two) link_row2<S>(h0.e);
      hop_compute16<S, 0, true, true>(h0, 1.0f, act, acc);
      hop_fill16<1, true>(h0, gauge, vp, p_out, s, pyp, Xh, nf.y);
      if (two) link_row2<S>(h1.e);
      hop_compute16<S, 0, false, false>(h1, 1.0f, act, acc);
      hop_fill16<1, true>(h1, gauge, vp, q, nym, pym, Xh, nbw.y);
      if (two) link_row2<S>(h0.e);
      hop_compute16<S, 1, true, false>(h0, 1.0f, act, acc);
      hop_fill16<2, true>(h0, gauge, vp, p_out, s, pzp, Xh, nf.z);
      if (two) link_row2<S>(h1.e);
      hop_compute16<S, 1, false, false>(h1, 1.0f, act, acc);
      hop_fill16<2, true>(h1, gauge, vp, q, nzm, pzm, Xh, nbw.z);
      if (two) link_row2<S>(h0.e);
      hop_compute16<S, 2, true, false>(h0, 1.0f, act, acc);
      hop_load16<3, true>(h0, gauge, vp, p_out, s, ntp, ld, nf.w);
      if (two) link_row2<S>(h1.e);
      hop_compute16<S, 2, false, false>(h1, 1.0f, act, acc);
      hop_load16<3, true>(h1, gauge, vp, q, ntm, ntm, ld, nbw.w);
      if (two) link_row2<S>(h0.e);
      hop_compute16<S, 3, true, false>(h0, sp, act, acc);
      if (two) link_row2<S>(h1.e);
      hop_compute16<S, 3, false, false>(h1, sm, act, acc);
      dslash_epilogue<S, F, G>(a, sd, cf, nullptr, -1, -1, -1, p_out, vp, s, off, r0, act, e, f, g, acc, nrm);
    }
    if (F & F_NORM) {
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const double w = wave_sum(nrm[i]);
        if (lane == 0) red[wave][i] = w;
      }
      __syncthreads();
      if (tid == 0) {
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if (!act[i]) continue;
          double v = 0.0;
          for (int w = 0; w < (nthr >> 6); ++w) v += red[w][i];
          a.partial[sd.ubeg[UK_RHS] + ((long)blk * T + t) * sd.nrhs + r0 + i] = v;
        }
      }
    }
  }
}

template <class S>
static void launch_dslash_blk_t(int flags, const DslashArgs& a, int threads, size_t lds, hipStream_t st) {
  if (a.total_units == 0) return;
  dim3 grid(a.total_units), block(threads);
  switch (flags) {
    case 0: hipLaunchKernelGGL((k_dslash_blk<S, 0>), grid, block, lds, st, a); break;
    case F_Y: hipLaunchKernelGGL((k_dslash_blk<S, F_Y>), grid, block, lds, st, a); break;
    case F_Y | F_NORM: hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_NORM>), grid, block, lds, st, a); break;
    case F_Y | F_NORM | F_POST:
      hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_NORM | F_POST>), grid, block, lds, st, a); break;
    case F_Y | F_NORM | F_OUT2:
      hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_NORM | F_OUT2>), grid, block, lds, st, a); break;
    case F_Y | F_XR | F_NORM:
      hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_XR | F_NORM>), grid, block, lds, st, a); break;
    case F_Y | F_POST: hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_POST>), grid, block, lds, st, a); break;
    case F_Y | F_DUAL: hipLaunchKernelGGL((k_dslash_blk<S, F_Y | F_DUAL>), grid, block, lds, st, a); break;
    default: throw std::runtime_error("unsupported flag combination for the block hop");
  }
}

bool dslash_blk_supports(int prec, int flags) {
  if (prec != PB16 && prec != PH16) return false;
  switch (flags) {
    case 0: case F_Y: case F_Y | F_NORM: case F_Y | F_NORM | F_POST: case F_Y | F_NORM | F_OUT2:
    case F_Y | F_XR | F_NORM: case F_Y | F_POST: case F_Y | F_DUAL:
      return true;
  }
  return false;
}

void launch_dslash_blk(int prec, int flags, const DslashArgs& a, int threads, size_t lds, hipStream_t st) {
  switch (prec) {
    case PB16: launch_dslash_blk_t<bf16s>(flags, a, threads, lds, st); break;
    case PH16: launch_dslash_blk_t<f16s>(flags, a, threads, lds, st); break;
    default: throw std::runtime_error("block hop: 16-bit storage only");
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
    case F_Y | F_NORM | F_POST:
      hipLaunchKernelGGL((k_dslash<S, F_Y | F_NORM | F_POST>), grid, block, 0, st, a); break;
    case F_Y | F_NORM | F_OUT2:
      hipLaunchKernelGGL((k_dslash<S, F_Y | F_NORM | F_OUT2>), grid, block, 0, st, a); break;
    case F_Y | F_XR | F_NORM:
      hipLaunchKernelGGL((k_dslash<S, F_Y | F_XR | F_NORM>), grid, block, 0, st, a); break;
    case F_Y | F_POST: hipLaunchKernelGGL((k_dslash<S, F_Y | F_POST>), grid, block, 0, st, a); break;
    case F_Y | F_DUAL: hipLaunchKernelGGL((k_dslash<S, F_Y | F_DUAL>), grid, block, 0, st, a); break;
    case F_CLV: hipLaunchKernelGGL((k_dslash<S, F_CLV>), grid, block, 0, st, a); break;
    case F_CLV | F_D: hipLaunchKernelGGL((k_dslash<S, F_CLV | F_D>), grid, block, 0, st, a); break;
    case F_CLV | F_Y: hipLaunchKernelGGL((k_dslash<S, F_CLV | F_Y>), grid, block, 0, st, a); break;
    case F_CLV | F_D | F_Y: hipLaunchKernelGGL((k_dslash<S, F_CLV | F_D | F_Y>), grid, block, 0, st, a); break;
    case F_CLV | F_Y | F_NORM:
      hipLaunchKernelGGL((k_dslash<S, F_CLV | F_Y | F_NORM>), grid, block, 0, st, a); break;
    case F_CLV | F_Y | F_NORM | F_POST:
      hipLaunchKernelGGL((k_dslash<S, F_CLV | F_Y | F_NORM | F_POST>), grid, block, 0, st, a); break;
    case F_CLV | F_Y | F_NORM | F_OUT2:
      hipLaunchKernelGGL((k_dslash<S, F_CLV | F_Y | F_NORM | F_OUT2>), grid, block, 0, st, a); break;
    case F_CLV | F_Y | F_XR | F_NORM:
      hipLaunchKernelGGL((k_dslash<S, F_CLV | F_Y | F_XR | F_NORM>), grid, block, 0, st, a); break;
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
