// Host-side launchers of the HIP kernels (implemented in the *.hip files).
#pragma once

#include "common.h"

namespace dl {

// dslash epilogue / prologue flags
enum DslashFlags : int {
  F_D = 1,      // multiply the input by the per-spin factor d on load
  F_Y = 2,      // add f (.) y
  F_NORM = 4,   // per-unit partial of ||result||^2 (or ||r||^2 with F_XR)
  F_XR = 8,     // CG update r -= alpha result (result not stored; x moves in update_p)
  F_OUT2 = 16,  // also store the result to a second field
  F_POST = 32,  // store g (.) result (the norm is taken before the factor)
  F_DUAL = 64,  // with F_Y: also out2 = g (.) H(d (.) in) + f (.) y from the same hop
  F_CLV = 256,  // clover slots: e, f, g apply their site matrix (Coef.m) before the per-spin
                // factor; d is 1 there (launch_site_factor applied it beforehand)
};

struct DslashArgs {
  const SlotDesc* slots;
  int nslots;
  int total_units;
  const Coef* coef;
  int p_out;
  const void* in;
  void* out;
  const void* y;
  double* partial;
  const int* active;
  void* x;
  void* r;
  const void* p;
  const double* alpha;
  void* out2;
};

void launch_dslash(int prec, int flags, const DslashArgs& a, hipStream_t st);
// The LDS-staged hop (16-bit storage; slots with bby > 0, UK_BLK units, one
// workgroup of `threads` threads and `lds` bytes of dynamic LDS per unit) and
// the flag combinations it is built for.
void launch_dslash_blk(int prec, int flags, const DslashArgs& a, int threads, size_t lds, hipStream_t st);
bool dslash_blk_supports(int prec, int flags);

// Clover site matrices (CloverKind) of a lattice from its packed FP64 links:
// o64 / o32 hold CLV_KINDS x 2 parities x clover_rows chunk rows of vp sites.
// sigma: sigma_{mu nu} of the planes 01 02 03 12 13 23 (complex 4 x 4).
void launch_clover_build(const void* g64, const int dims[4], long long vp, double kappa, double mu, double csw,
                         const double (&sigma)[6][4][4][2], void* o64, void* o32, hipStream_t st);
// out = d (.) (M_d in) on slots with a clover term and a d matrix (Coef.m[0]),
// out = in elsewhere; fields of parity par, UK_RHS units, gated rhs skipped.
void launch_site_factor(int prec, const SlotDesc* slots, int nslots, int total_units, const Coef* coef, int par,
                        const void* in, void* out, const int* gate, hipStream_t st);

// finalize kinds
enum FinKind : int { FK_INIT = 0, FK_ALPHA = 1, FK_BETA = 2, FK_STORE = 3 };

struct CgScalars {
  double* rr;      // current <r, r>
  double* cc;      // <c, c> of the normal-equation right-hand side
  double* alpha;
  double* beta;
  double* tol2;    // tol^2
  double* out;     // FK_STORE destination
  int* active;
  int* iters;
  int* maxiter;
  int* status;
  int* upd;        // 1: x += alpha p of this iteration still to be applied
};

void launch_finalize(int kind, const SlotDesc* slots, int nslots, int nrhs_total,
                     const double* partial, const CgScalars& cs, hipStream_t st);

// Per-rhs state of the reliable updates of the high-precision tier, kept on
// the device so that a whole step (decision, update, CG iteration) replays
// from a graph without the host.
struct HpState {
  double* rr_ru;   // <r, r> right after the last reliable update
  int* hflag;      // this step: 0 nothing, 1 reliable update, 2 verification of an rhs whose
                   // iterated residual converged
  int* flag;       // hflag != 0: gate of the update kernels
  int* react;      // verification failed: CG restarts from the true residual this step
  int* verified;   // converged and verified (or given up at the iteration cap)
  int* ru_count;   // reliable updates so far
  int* pending;    // [1] rhs still iterating or awaiting verification (after k_hp_pending)
  double delta2;   // update when <r, r> fell below delta2 times its value after the last one
};
// Decide, per rhs, this step's reliable update or verification (sets hflag,
// flag, clears react).
void launch_hp_decide(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st);
// After the update of the flagged rhs: count it, record <r, r>, and settle
// verifications (verified, restart with react, or iteration cap).
void launch_hp_post(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st);
// hp.pending[0] = number of rhs still active or awaiting verification.
void launch_hp_pending(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st);

// x += alpha p where upd is set (every rhs that took this iteration's step),
// Initial guesses: copy the odd solution field of every slot with gsave to
// its guess buffer (raw words, the field's precision), and load slots with
// gload (precision gprec) into a field of precision `prec` (zeros elsewhere).
void launch_guess_store(int prec, const SlotDesc* slots, int nslots, int total_units, const void* f,
                        hipStream_t st);
void launch_guess_load(int prec, const SlotDesc* slots, int nslots, int total_units, void* f, hipStream_t st);

// then p = r + beta p for the right-hand sides still active
void launch_update_p(int prec, const SlotDesc* slots, int nslots, int total_units, void* p,
                     const void* r, void* x, const double* alpha, const double* beta, const int* active,
                     const int* upd, hipStream_t st);

// set a batch field to zero on parity-free half fields
void launch_zero(int prec, const SlotDesc* slots, int nslots, int total_units, void* f,
                 const int* active, hipStream_t st);

// eta (parity p) of every rhs: Z2 / Z4 from the counter generator, or packed
// from the caller's complex128 sources
void launch_sources(int prec, const SlotDesc* slots, int nslots, int total_units, int parity,
                    void* eta, hipStream_t st);

// unpack even and odd half fields to the caller's complex128 solution arrays
void launch_unpack(int prec, const SlotDesc* slots, int nslots, int total_units, int parity,
                   const void* f, hipStream_t st);

// out = (S_out) in, for active rhs (or all when active is null); add != 0: out += in
void launch_convert(int prec_in, int prec_out, const SlotDesc* slots, int nslots, int total_units,
                    const void* in, void* out, int add, const int* active, hipStream_t st);

// r64 = c64 - ap64, r32 = (float) r64, partial ||r64||^2, for rhs with flag set
void launch_residual_replace(const SlotDesc* slots, int nslots, int total_units, const void* c64,
                             const void* ap64, void* r64, void* r32, double* partial,
                             const int* flag, hipStream_t st);

// partial ||a - b||^2 and ||b||^2 (FP64 fields) for the true residual report
void launch_diff_norms(const SlotDesc* slots, int nslots, int total_units, const void* a,
                       const void* b, double* partial_diff, double* partial_b, hipStream_t st);

// gauge packing: FP64 [t][z][y][x][mu][3][3] (device) -> four even-odd layouts;
// *not_su3 (device, cleared by the caller) gets the TWO_ROW_* bits of the
// storage classes for which a link's row 2 is not conj(row 0 x row 1) to
// their threshold
void launch_pack_gauge(const double* src, int X, int Y, int Z, int T, void* g64, void* g32,
                       void* gb16, void* gh16, int* not_su3, hipStream_t st);

// loop contractions of a block of solutions into FP64 accumulators.
// Without phi (null): the one-end-trick structures, (xi, s) pairs with
// xi = (1 - kappa H) s.  With phi: hopping-parameter-expanded loops without
// tau_3, the pair (xi = eta, phi = (kappa B H)^n s), symmetrised into the flavour
// sum (local C -> (C + g5 C^dag g5) / 2, derivative E -> (E - g5 E^dag g5) / 2).
// dil: some slot is time-diluted (with phi: the xi-s block of an rhs is then
// contracted only next to its component's time slices).
void launch_contract_local(int prec, const SlotDesc* slots, int nslots, int total_units,
                           const void* s_e, const void* s_o, const void* xi_e, const void* xi_o,
                           const void* phi_e, const void* phi_o, bool dil, hipStream_t st);
void launch_contract_deriv(int prec, const SlotDesc* slots, int nslots, int total_units,
                           const void* s_e, const void* s_o, const void* xi_e, const void* xi_o,
                           const void* phi_e, const void* phi_o, bool dil, hipStream_t st);

// Tables of the separable momentum projection (device pointers), built on the
// host from the momentum list: distinct kx values, distinct (kx, ky) pairs.
struct ProjTables {
  int np, nkx, nkxy;
  const double* roots_x;  // [X] complex e^{-2 pi i m / X}
  const double* roots_y;  // [Y] complex e^{-2 pi i m / Y}
  const int* kx_mod;    // [nkx] kx mod X of distinct value ix
  const int* ky_mod;    // [nkxy] ky mod Y of pair j
  const int* pair_ix;   // [nkxy] kx index of pair j
  const double* pz;     // [nkz][Z] complex e^{-2 pi i kz z / Z}, kz of distinct value k
  const int* pj;        // [np] pair index of momentum p
  const int* pk;        // [np] distinct-kz index of momentum p
  const int* order;     // [np] momenta sorted by (kz, pair): the z-sum's thread order
  const double* shift;  // [np][3] complex 1 + e^{-2 pi i n_nu / L_nu}
};
// proj [nq][T][Np] complex = projection of sum_k w[k] acc[k] (null sets
// skipped); rows q >= q_link are link-centred derivative sums (pass nq for
// none).  r2: scratch of nq*T*Z*nkxy complex.
void launch_project(const double* const acc[3], const double w[3], int nq, int q_link, int X, int Y, int Z, int T,
                    const ProjTables& tb, double* r2, double* proj, hipStream_t st);

// Zero n doubles with a fill kernel.
void launch_fill_zero(double* p, long long n, hipStream_t st);

// Gamma rebuild and prefactors -> out [2][nops][16][T][Np] complex.
// exact (device [nops][16] complex, or null): added to the loops without
// tau_3 at momentum 0 before the prefactor (exact part of the hopping
// parameter expansion, already multiplied by the spatial volume and weights).
void launch_loops_finalize(const double* proj, int nops, int T, int np, double kappa, double mu,
                           const double* exact, double* out, hipStream_t st);

// Number of FP64 accumulator components per site for an ops mask.
int acc_components(int ops);

// ---- backward pass ---------------------------------------------------------
// Omega fields [2][nops][16][V] complex from the upstream gradient g
// [2][nops][16][T][Np] (device) and the phase tables of the projection.
void launch_omega(const double* g, int nops, int X, int Y, int Z, int T, int np, const double* phase_x,
                  const double* phase_y, const double* phase_z, double kappa, double mu, long long nsrc,
                  double* omega, hipStream_t st);
// A = Q_1 s, C = gamma5 Q_t3 s + Q_t3^dag gamma5 s + Q_1 s + Q_1^dag M_0 s on parity p_out
// (FP64 batch fields), per-unit partials of s^dag gamma5 Q_t3 s.
void launch_insert_apply(const SlotDesc* slots, int nslots, int total_units, int p_out, int nops,
                         const double* omega, const void* s_e, const void* s_o, const void* m_e, const void* m_o,
                         void* a_out, void* c_out, double* part_re, double* part_im, hipStream_t st);
// zout = gamma5 zin on complex128 site arrays; optional partials of conj(s) . zin per 256 sites
void launch_g5_lex(const double* zin, double* zout, const double* s, long long nsite, double* part_re,
                   double* part_im, hipStream_t st);
// out[0] = fixed-order sum of n partials
void launch_sum(const double* part, long long n, double* out, hipStream_t st);

}  // namespace dl
