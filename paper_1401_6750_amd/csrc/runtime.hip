// Host runtime: batched even-odd CGNR solves (the stochastic inversions of
// the paper's eq. (1)), source generation, contractions and loop assembly.
//
// A batch is a list of slots (lattice, block of consecutive sources) of one
// precision class.  Every kernel launch covers the whole batch, so lattices of
// different sizes and any number of right-hand sides advance together; each
// right-hand side carries its own CG scalars and retires on its own
// convergence, after which its units exit at once.
#include <algorithm>
#include <cctype>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <sys/stat.h>

#include "runtime.h"

namespace dl {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(DL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void* Pool::get(size_t bytes) {
  auto it = free_.find(bytes);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    cached_bytes -= bytes;
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    clear();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(DL_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  return p;
}

void Pool::put(void* p, size_t bytes) {
  free_.emplace(bytes, p);
  cached_bytes += bytes;
}

void Pool::clear() {
  for (auto& kv : free_) (void)hipFree(kv.second);
  free_.clear();
  cached_bytes = 0;
}

void stream_enter(dl_ctx* c) {
  HIPCHECK(hipSetDevice(c->device));
  HIPCHECK(hipEventRecord(c->ev, c->user_stream));
  HIPCHECK(hipStreamWaitEvent(c->st, c->ev, 0));
}

void stream_exit(dl_ctx* c) {
  HIPCHECK(hipEventRecord(c->ev, c->st));
  HIPCHECK(hipStreamWaitEvent(c->user_stream, c->ev, 0));
}

int tier_prec(int tier) {
  switch (tier) {
    case DL_TIER_FP64: return P64;
    case DL_TIER_LP_BF16: return PB16;
    case DL_TIER_LP_FP16: return PH16;
    case DL_TIER_HP_FP32: return P32;
  }
  throw Error(DL_EINVAL, "unknown tier " + std::to_string(tier));
}

// ---------------------------------------------------------------------------
// gamma insertions: Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3, chiral basis
// ---------------------------------------------------------------------------
void gamma_basis(std::complex<double> (&G)[16][4][4]) {
  using C = std::complex<double>;
  const C I(0, 1);
  C g[4][4][4] = {};
  // gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]]
  const C sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[k][a][2 + b] = -I * sig[k][a][b];
        g[k][2 + a][b] = I * sig[k][a][b];
      }
  for (int a = 0; a < 2; ++a) g[3][a][2 + a] = g[3][2 + a][a] = 1;
  for (int n = 0; n < 16; ++n) {
    C m[4][4] = {};
    for (int a = 0; a < 4; ++a) m[a][a] = 1;
    for (int k = 0; k < 4; ++k) {
      if (!((n >> k) & 1)) continue;
      C t[4][4] = {};
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          for (int c = 0; c < 4; ++c) t[a][b] += m[a][c] * g[k][c][b];
      std::memcpy(m, t, sizeof(m));
    }
    std::memcpy(G[n], m, sizeof(m));
  }
}

void init_gamma_table() {
  using C = std::complex<double>;
  C G[16][4][4];
  gamma_basis(G);
  int col[16][4];
  double ph[16][4][2];
  for (int n = 0; n < 16; ++n) {
    const C (&m)[4][4] = G[n];
    for (int a = 0; a < 4; ++a) {
      int found = -1;
      for (int b = 0; b < 4; ++b)
        if (std::abs(m[a][b]) > 0.5) found = b;
      col[n][a] = found;
      ph[n][a][0] = m[a][found].real();
      ph[n][a][1] = m[a][found].imag();
    }
  }
  set_gamma_table(col, ph);
}

// ---------------------------------------------------------------------------
// per-slot spin coefficients of the dslash-type launches
// ---------------------------------------------------------------------------
enum CoefKind : int {
  CK_MHAT1 = 0,   // u_e = A^-1(mu) H_eo p_o
  CK_MHAT2,       // t_o = p_o - kappa^2 A^-1(mu) H_oe u_e
  CK_MDAG1,       // u_e = A^-1(-mu) H_eo gamma5 A^-1(-mu) w_o
  CK_MDAG2,       // out_o = w_o - kappa^2 gamma5 H_oe u_e
  CK_PREP,        // bhat_o = A^-1(eta_o + kappa H_oe A^-1 eta_e)
  CK_RECON,       // s_e = A^-1(eta_e + kappa H_eo s_o)
  CK_XI,          // xi_p = s_p - kappa H s
  CK_RECON_XI,    // s_e as CK_RECON and (g) xi_e = s_e - kappa H_eo s_o from one hop
  CK_MFULL,       // (M psi)_p = A psi_p - kappa H psi
  CK_MDAGFULL,    // (M^dag psi)_p = A(-mu) psi_p - kappa gamma5 H gamma5 psi
  CK_HOP,         // H psi
  CK_G5V,         // gamma5 C_p - kappa H gamma5 A  (backward pass)
  CK_KBH,         // kappa A^-1(mu) H psi  (one order of the hopping parameter expansion)
  // CG-loop forms: the M-hat result is stored as t' = D t with
  // D = gamma5 A^-1(-mu), which is exactly the input M-hat^dag needs at every
  // neighbour, so its hop needs no per-neighbour factor; t = D^-1 t' is
  // rebuilt per site where M-hat^dag adds it back.
  CK_MHAT2P,      // t'_o = D (p_o - kappa^2 A^-1(mu) H_oe u_e), norm of t
  CK_MDAG1P,      // u_e = A^-1(-mu) H_eo t'_o
  CK_MDAG2P,      // out_o = D^-1 t'_o - kappa^2 gamma5 H_oe u_e
  CK_COUNT
};

using Cd = std::complex<double>;

static void put(double (&dst)[4][2], float (&dst32)[4][2], const Cd (&v)[4]) {
  for (int s = 0; s < 4; ++s) {
    dst[s][0] = v[s].real();
    dst[s][1] = v[s].imag();
    dst32[s][0] = (float)v[s].real();
    dst32[s][1] = (float)v[s].imag();
  }
}

// Coefficients with a clover term: the twist factors A, A^-1 become site
// matrices (CloverKind) applied before a per-spin constant (gamma_5 signs and
// scalars, which commute with them); see csrc/clover.hip for the operator.
static Coef make_coef_clover(int kind, double kappa) {
  const double g5[4] = {1, 1, -1, -1};
  const double k2 = kappa * kappa;
  Cd d[4], e[4], f[4], g[4];
  int m[4] = {-1, -1, -1, -1};
  for (int s = 0; s < 4; ++s) {
    d[s] = 1.0;
    e[s] = 1.0;
    f[s] = 0.0;
    g[s] = 1.0;
    const double G5 = g5[s];
    switch (kind) {
      case CK_MHAT2P: e[s] = -k2; m[1] = CLV_AINV; f[s] = 1.0; g[s] = G5; m[3] = CLV_AINV_M; break;
      case CK_MDAG1P: m[1] = CLV_AINV_M; break;
      case CK_MDAG2P: e[s] = -k2 * G5; f[s] = G5; m[2] = CLV_A_M; break;
      case CK_MHAT1: m[1] = CLV_AINV; break;
      case CK_MHAT2: e[s] = -k2; m[1] = CLV_AINV; f[s] = 1.0; break;
      case CK_MDAG1: d[s] = G5; m[0] = CLV_AINV_M; m[1] = CLV_AINV_M; break;
      case CK_MDAG2: e[s] = -k2 * G5; f[s] = 1.0; break;
      case CK_PREP: m[0] = CLV_AINV; e[s] = kappa; m[1] = CLV_AINV; f[s] = 1.0; m[2] = CLV_AINV; break;
      case CK_RECON: e[s] = kappa; m[1] = CLV_AINV; f[s] = 1.0; m[2] = CLV_AINV; break;
      case CK_XI: e[s] = -kappa; f[s] = 1.0; m[2] = CLV_AC; break;
      case CK_MFULL: e[s] = -kappa; f[s] = 1.0; m[2] = CLV_A; break;
      case CK_MDAGFULL: d[s] = G5; e[s] = -kappa * G5; f[s] = 1.0; m[2] = CLV_A_M; break;
      case CK_HOP: break;
      default:
        // the expansion's kernels, the gradient insertions and the fused
        // reconstruction of s_e and xi_e are not built for clover lattices
        break;
    }
  }
  Coef c;
  put(c.d, c.d32, d);
  put(c.e, c.e32, e);
  put(c.f, c.f32, f);
  put(c.g, c.g32, g);
  for (int k = 0; k < 4; ++k) c.m[k] = m[k];
  return c;
}

static Coef make_coef(int kind, double kappa, double mu) {
  const double g5[4] = {1, 1, -1, -1};
  Cd one[4], zero[4], A[4], Am[4], Ai[4], Ami[4], G5[4];
  for (int s = 0; s < 4; ++s) {
    one[s] = 1.0;
    zero[s] = 0.0;
    A[s] = Cd(1.0, 2.0 * kappa * mu * g5[s]);
    Am[s] = Cd(1.0, -2.0 * kappa * mu * g5[s]);
    Ai[s] = 1.0 / A[s];
    Ami[s] = 1.0 / Am[s];
    G5[s] = g5[s];
  }
  Cd d[4], e[4], f[4], g[4];
  for (int s = 0; s < 4; ++s) {
    d[s] = one[s];
    e[s] = one[s];
    f[s] = zero[s];
    g[s] = one[s];
  }
  const double k2 = kappa * kappa;
  for (int s = 0; s < 4; ++s) {
    const Cd D = G5[s] * Ami[s];
    switch (kind) {
      case CK_MHAT2P: e[s] = -k2 * Ai[s]; f[s] = 1.0; g[s] = D; break;
      case CK_MDAG1P: e[s] = Ami[s]; break;
      case CK_MDAG2P: e[s] = -k2 * G5[s]; f[s] = 1.0 / D; break;
      case CK_MHAT1: e[s] = Ai[s]; break;
      case CK_MHAT2: e[s] = -k2 * Ai[s]; f[s] = 1.0; break;
      case CK_MDAG1: d[s] = G5[s] * Ami[s]; e[s] = Ami[s]; break;
      case CK_MDAG2: e[s] = -k2 * G5[s]; f[s] = 1.0; break;
      case CK_PREP: d[s] = Ai[s]; e[s] = kappa * Ai[s]; f[s] = Ai[s]; break;
      case CK_RECON: e[s] = kappa * Ai[s]; f[s] = Ai[s]; break;
      case CK_XI: e[s] = -kappa; f[s] = 1.0; break;
      case CK_RECON_XI: e[s] = kappa * Ai[s]; f[s] = Ai[s]; g[s] = kappa * Ai[s] - kappa; break;
      case CK_MFULL: e[s] = -kappa; f[s] = A[s]; break;
      case CK_MDAGFULL: d[s] = G5[s]; e[s] = -kappa * G5[s]; f[s] = Am[s]; break;
      case CK_HOP: break;
      case CK_G5V: d[s] = G5[s]; e[s] = -kappa; f[s] = G5[s]; break;
      case CK_KBH: e[s] = kappa * Ai[s]; break;
    }
  }
  Coef c;
  put(c.d, c.d32, d);
  put(c.e, c.e32, e);
  put(c.f, c.f32, f);
  put(c.g, c.g32, g);
  for (int k = 0; k < 4; ++k) c.m[k] = -1;
  return c;
}

// Block shape of the LDS-staged hop for a lattice (16-bit storage, no clover
// term, option "block_hop"): bby | Y, bbz | Z with 64 <= bby * bbz * X/2 <= 256
// threads and at most 48 KiB of LDS (three or more workgroups per CU), the
// fewest halo rows per centre row, then the most threads; one time slice per
// workgroup.  It depends on the lattice shape only, so a source's iterates do
// not depend on what else shares its batch.  false: no such shape.
static bool blk_shape(const int dims[4], int& by, int& bz, int& seg, size_t& lds) {
  const int X = dims[0], Y = dims[1], Z = dims[2], Xh = X / 2;
  double best = 1e30;
  int best_n = 0;
  by = bz = 0;
  for (int b = 1; b <= Y; ++b) {
    if (Y % b) continue;
    for (int c = 1; c <= Z; ++c) {
      if (Z % c) continue;
      const int n = b * c * Xh;
      if (n < 64 || n > 256) continue;
      const size_t bytes = (size_t)2 * (b * c + 2 * (b + c)) * 3 * Xh * 16;
      if (bytes > 48 * 1024) continue;
      const double ratio = 2.0 * (b + c) / (b * c);
      if (ratio < best - 1e-12 || (ratio < best + 1e-12 && n > best_n)) {
        best = ratio;
        best_n = n;
        by = b;
        bz = c;
        lds = bytes;
      }
    }
  }
  if (!by) return false;
  seg = 1;   // one time slice per workgroup
  return true;
}

// ---------------------------------------------------------------------------
// batch state
// ---------------------------------------------------------------------------
struct Batch {
  dl_ctx* ctx;
  int prec;
  std::vector<SlotDesc> hs, hs_tile;
  std::vector<Coef> coefs;     // host copies stay alive while their uploads are in flight
  DevBuf dslots, dcoef;
  int nslots = 0, nrhs = 0, u_rhs = 0, u_site = 0, u_deriv = 0, u_grp2 = 0, u_grp4 = 0;
  long long sites = 0;
  DevBuf partial, partial2, scal;
  CgScalars cs{};
  bool has_clover = false;     // some slot's lattice has a clover term
  bool has_plain = false;      // some slot's lattice has none
  // LDS-staged hop (16-bit storage): its units, workgroup size and LDS bytes;
  // the tile kernel's slots (UK_GRP2 units of the other slots only) when the
  // batch mixes shapes
  int u_blk = 0, blk_threads = 0, u_grp2_tile = 0;
  size_t blk_lds = 0;
  DevBuf dslots_tile;
  DevBuf fd_tmp;               // clover batches: input of a hop after its site factor d
  int* h_int = nullptr;        // pinned: active / status / iters mirrors
  double* h_dbl = nullptr;     // pinned: rr / cc / out mirrors

  Batch(dl_ctx* c, int prec_, const std::vector<SlotPlan>& plan, const std::vector<dl_job>* jobs)
      : ctx(c), prec(prec_) {
    int ur = 0, us = 0, ud = 0, ug2 = 0, ug4 = 0, rb = 0;
    long long fo = 0;
    for (const SlotPlan& sp : plan) {
      const dl_lattice* L = sp.lat;
      SlotDesc d{};
      d.X = L->dims[0]; d.Y = L->dims[1]; d.Z = L->dims[2]; d.T = L->dims[3];
      d.Xh = d.X / 2;
      d.Vh = (int)L->Vh;
      d.ntile = (d.Vh + TILE - 1) / TILE;
      d.Vp = (int)pad_half(d.Vh);
      d.tblk = sp.tblk > 0 ? sp.tblk : TBLK_DEFAULT;
      d.nrhs = sp.nrhs;
      d.ubeg[UK_RHS] = ur; d.ubeg[UK_SITE] = us; d.ubeg[UK_DERIV] = ud;
      d.ubeg[UK_GRP2] = ug2; d.ubeg[UK_GRP4] = ug4;
      d.rhs_begin = rb;
      d.fo = fo;
      d.bc = (double)L->bc;
      d.two_row = L->two_row;
      for (int p = 0; p < 4; ++p) d.gauge[p] = L->gauge[p];
      d.clv64 = L->csw != 0.0 ? L->clv64 : nullptr;
      d.clv32 = L->csw != 0.0 ? L->clv32 : nullptr;
      if (d.clv64) has_clover = true;
      else has_plain = true;
      d.acc = sp.acc;
      d.acc_ops = 0;
      if (jobs && sp.acc) d.acc_ops = (*jobs)[sp.job].accum->ops;
      if (jobs) {
        const dl_job& j = (*jobs)[sp.job];
        d.seed = j.seed;
        d.noise = j.noise;
      } else {
        d.noise = DL_NOISE_USER;
      }
      d.src0 = sp.src0;
      d.tdil = sp.tdil;
      d.tclen = sp.tclen;
      d.tentry = sp.job_first;
      d.job = sp.job;
      d.src_user = sp.src_user;
      d.sol_user = sp.sol_user;
      d.gsave = sp.gsave;
      d.gload = sp.gload;
      d.gprec = sp.gprec;
      ur += d.ntile * d.nrhs;
      us += 2 * d.ntile;
      ud += 8 * d.ntile;
      ug2 += d.ntile * ((d.nrhs + 1) / 2);
      ug4 += d.ntile * ((d.nrhs + 3) / 4);
      rb += d.nrhs;
      fo += (long long)d.nrhs * d.Vp;
      hs.push_back(d);
    }
    // LDS-staged hop for 16-bit storage, per lattice shape
    if ((prec == PB16 || prec == PH16) && ctx->block_hop) {
      int ub = 0;
      for (size_t i = 0; i < hs.size(); ++i) {
        SlotDesc& d = hs[i];
        d.ubeg[UK_BLK] = ub;
        int by = 0, bz = 0, seg = 0;
        size_t lds = 0;
        const int dims[4] = {d.X, d.Y, d.Z, d.T};
        if (!d.clv64 && blk_shape(dims, by, bz, seg, lds)) {
          d.bby = by;
          d.bbz = bz;
          d.bseg = seg;
          ub += (d.Y / by) * (d.Z / bz) * (d.T / seg) * ((d.nrhs + 1) / 2);
          blk_threads = std::max(blk_threads, (by * bz * d.Xh + 63) / 64 * 64);
          blk_lds = std::max(blk_lds, lds);
        }
      }
      u_blk = ub;
    }
    nslots = (int)hs.size();
    nrhs = rb;
    u_rhs = ur; u_site = us; u_deriv = ud; u_grp2 = ug2; u_grp4 = ug4;
    sites = fo;
    dslots = DevBuf(ctx, sizeof(SlotDesc) * nslots);
    HIPCHECK(hipMemcpyAsync(dslots.p, hs.data(), sizeof(SlotDesc) * nslots, hipMemcpyHostToDevice, ctx->st));
    if (u_blk > 0) {
      // the tile kernel covers the slots without a block shape only
      hs_tile = hs;
      int ut = 0;
      for (SlotDesc& d : hs_tile) {
        d.ubeg[UK_GRP2] = ut;
        if (!d.bby) ut += d.ntile * ((d.nrhs + 1) / 2);
      }
      u_grp2_tile = ut;
      dslots_tile = DevBuf(ctx, sizeof(SlotDesc) * nslots);
      HIPCHECK(hipMemcpyAsync(dslots_tile.p, hs_tile.data(), sizeof(SlotDesc) * nslots, hipMemcpyHostToDevice,
                              ctx->st));
    }
    coefs.resize((size_t)CK_COUNT * nslots);
    for (int k = 0; k < CK_COUNT; ++k)
      for (int i = 0; i < nslots; ++i) {
        const dl_lattice* L = plan[i].lat;
        coefs[(size_t)k * nslots + i] = L->csw != 0.0 ? make_coef_clover(k, L->kappa) : make_coef(k, L->kappa, L->mu);
      }
    dcoef = DevBuf(ctx, sizeof(Coef) * coefs.size());
    HIPCHECK(hipMemcpyAsync(dcoef.p, coefs.data(), sizeof(Coef) * coefs.size(), hipMemcpyHostToDevice, ctx->st));
    partial = DevBuf(ctx, sizeof(double) * std::max(u_rhs, 1));
    partial2 = DevBuf(ctx, sizeof(double) * std::max(u_rhs, 1));
    // scalars: 6 double arrays + 5 int arrays
    const size_t nd = 6 * (size_t)nrhs, ni = 5 * (size_t)nrhs;
    scal = DevBuf(ctx, sizeof(double) * nd + sizeof(int) * ni + 16);
    double* db = scal.as<double>();
    cs.rr = db; cs.cc = db + nrhs; cs.alpha = db + 2 * nrhs; cs.beta = db + 3 * nrhs;
    cs.tol2 = db + 4 * nrhs; cs.out = db + 5 * nrhs;
    int* ib = (int*)(db + nd);
    cs.active = ib; cs.iters = ib + nrhs; cs.maxiter = ib + 2 * nrhs; cs.status = ib + 3 * nrhs;
    cs.upd = ib + 4 * nrhs;
    if (has_clover) fd_tmp = DevBuf(ctx, std::max<size_t>(field_bytes(P64), 16));
    HIPCHECK(hipHostMalloc((void**)&h_int, sizeof(int) * 4 * std::max(nrhs, 1), hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&h_dbl, sizeof(double) * 6 * std::max(nrhs, 1), hipHostMallocDefault));
  }
  ~Batch() {
    if (h_int) (void)hipHostFree(h_int);
    if (h_dbl) (void)hipHostFree(h_dbl);
  }
  const SlotDesc* slots() const { return dslots.as<SlotDesc>(); }
  const Coef* coef(int kind) const { return dcoef.as<Coef>() + (size_t)kind * nslots; }
  size_t field_bytes(int p) const { return (size_t)sites * chunks_of(p) * 16; }
  DevBuf field(int p) { return DevBuf(ctx, std::max<size_t>(field_bytes(p), 16)); }

  void dslash(int p, int flags, int ck, int p_out, const void* in, void* out, const void* y,
              const int* gate, void* x = nullptr, void* r = nullptr, const void* pp = nullptr,
              void* out2 = nullptr, double* part = nullptr) {
    DslashArgs a{};
    a.slots = slots(); a.nslots = nslots; a.coef = coef(ck); a.p_out = p_out;
    const int g = rhs_per_wave_prec(p);
    a.total_units = g == 1 ? u_rhs : (g == 2 ? u_grp2 : u_grp4);
    a.in = in; a.out = out; a.y = y; a.partial = part ? part : partial.as<double>(); a.active = gate;
    a.x = x; a.r = r; a.p = pp; a.alpha = cs.alpha; a.out2 = out2;
    if (has_clover) {
      if (flags & F_DUAL) throw Error(DL_EINVAL, "fused reconstruction is not built for clover lattices");
      if ((flags & F_D) && clover_d(ck)) {
        // d is a site matrix on clover slots: apply it to the input first
        // (plain slots get a bit copy and keep their d in the hop)
        launch_site_factor(p, slots(), nslots, u_rhs, coef(ck), 1 - p_out, in, fd_tmp.p, gate, ctx->st);
        a.in = fd_tmp.p;
      }
      launch_dslash(p, flags | F_CLV, a, ctx->st);   // the clover slots
      if (!has_plain) return;
    }
    // the slots without a clover term
    if (u_blk > 0 && p == prec && dslash_blk_supports(p, flags)) {
      DslashArgs ab = a;
      ab.total_units = u_blk;
      launch_dslash_blk(p, flags, ab, blk_threads, blk_lds, ctx->st);
      if (u_grp2_tile > 0) {
        a.slots = dslots_tile.as<SlotDesc>();
        a.total_units = u_grp2_tile;
        launch_dslash(p, flags, a, ctx->st);
      }
      return;
    }
    launch_dslash(p, flags, a, ctx->st);
  }
  // some clover slot's coefficient d of kind ck is a site matrix
  bool clover_d(int ck) const {
    for (int i = 0; i < nslots; ++i)
      if (hs[i].clv64 && coefs[(size_t)ck * nslots + i].m[0] >= 0) return true;
    return false;
  }
  void finalize(int kind, const double* part = nullptr) {
    launch_finalize(kind, slots(), nslots, nrhs, part ? part : partial.as<double>(), cs, ctx->st);
  }
  void finalize_store(double* dst, const int* gate, const double* part) {
    CgScalars c = cs;
    c.out = dst;
    c.active = const_cast<int*>(gate);
    launch_finalize(FK_STORE, slots(), nslots, nrhs, part, c, ctx->st);
  }
  void to_host_int(const int* dev, int* host) {
    HIPCHECK(hipMemcpyAsync(host, dev, sizeof(int) * nrhs, hipMemcpyDeviceToHost, ctx->st));
  }
  void to_host_dbl(const double* dev, double* host) {
    HIPCHECK(hipMemcpyAsync(host, dev, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ctx->st));
  }
  void sync() { HIPCHECK(hipStreamSynchronize(ctx->st)); }
};

// All-ones gate (every rhs selected) for FK_STORE of reports.
static DevBuf ones_gate(Batch& b) {
  DevBuf g(b.ctx, sizeof(int) * std::max(b.nrhs, 1));
  std::vector<int> h(std::max(b.nrhs, 1), 1);
  HIPCHECK(hipMemcpyAsync(g.p, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, b.ctx->st));
  HIPCHECK(hipStreamSynchronize(b.ctx->st));
  return g;
}

// ---------------------------------------------------------------------------
// CG on Mhat^dag Mhat: one iteration (7 launches), gated by the active mask
// ---------------------------------------------------------------------------
struct CgFields {
  void *x, *r, *p, *t, *u;
};

static void cg_iteration(Batch& b, int P, const CgFields& f, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  const int* act = b.cs.active;
  if (t0) HIPCHECK(hipEventRecord(t0, b.ctx->st));
  b.dslash(P, 0, CK_MHAT1, 0, f.p, f.u, nullptr, act);
  if (t1) HIPCHECK(hipEventRecord(t1, b.ctx->st));
  b.dslash(P, F_Y | F_NORM | F_POST, CK_MHAT2P, 1, f.u, f.t, f.p, act);   // t' = D t
  b.finalize(FK_ALPHA);
  b.dslash(P, 0, CK_MDAG1P, 0, f.t, f.u, nullptr, act);
  b.dslash(P, F_Y | F_XR | F_NORM, CK_MDAG2P, 1, f.u, nullptr, f.t, act, nullptr, f.r);
  b.finalize(FK_BETA);
  launch_update_p(P, b.slots(), b.nslots, b.u_rhs, f.p, f.r, f.x, b.cs.alpha, b.cs.beta, act, b.cs.upd,
                  b.ctx->st);
}

// c = Mhat^dag bhat with bhat from eta; r = p = c, x = 0, scalars initialised.
static void cg_start(Batch& b, int P, const void* eta_e, const void* eta_o, const CgFields& f) {
  b.dslash(P, F_D | F_Y, CK_PREP, 1, eta_e, f.t, eta_o, nullptr);
  b.dslash(P, F_D, CK_MDAG1, 0, f.t, f.u, nullptr, nullptr);
  b.dslash(P, F_Y | F_NORM | F_OUT2, CK_MDAG2, 1, f.u, f.r, f.t, nullptr, nullptr, nullptr, nullptr, f.p);
  b.finalize(FK_INIT);
  launch_zero(P, b.slots(), b.nslots, b.u_rhs, f.x, nullptr, b.ctx->st);
}

// Contractions add into per-site accumulators with plain read-modify-writes,
// so no two units of one launch may own the same accumulator.  Consecutive
// slots of one lattice that feed one accumulator are contiguous in every batch
// field and merge into one contraction slot (its right-hand sides are summed in
// registers, in order); accumulators that still appear in several merged slots
// are handled in successive launches.
// Contractions of the batch's solutions into their accumulators.  Slots that
// share an accumulator go to different launches (no two waves of one launch
// add to the same site); slots whose accumulator uses the hopping parameter
// expansion run the HPE kernels (xi = eta, phi_loc / phi_der the expanded
// fields for local / derivative insertions).
struct HpeFields {
  const void* eta[2] = {nullptr, nullptr};
  const void* loc[2] = {nullptr, nullptr};
  const void* der[2] = {nullptr, nullptr};
};

static void contract_passes(Batch& b, int P, const void* s_e, const void* s_o, const void* xi_e, const void* xi_o,
                            const HpeFields& h) {
  std::vector<SlotDesc> merged;
  for (const SlotDesc& d : b.hs) {
    if (!d.acc) continue;
    if (!merged.empty()) {
      SlotDesc& m = merged.back();
      // contiguous slots of one accumulator and lattice contract as one; time-diluted
      // slots only as consecutive entries of one job (the component of an rhs
      // follows from its entry)
      const bool dil_ok = (m.tdil <= 1 && d.tdil <= 1) ||
                          (m.tdil == d.tdil && m.job == d.job && m.tentry + m.nrhs == d.tentry);
      if (m.acc == d.acc && m.gauge[0] == d.gauge[0] && m.fo + (long long)m.nrhs * m.Vp == d.fo && dil_ok) {
        m.nrhs += d.nrhs;
        continue;
      }
    }
    merged.push_back(d);
  }
  std::vector<std::vector<SlotDesc>> passes;
  std::map<std::pair<double*, bool>, int> seen;
  for (const SlotDesc& d : merged) {
    const bool hpe = DL_OPS_HPE_ORDER(d.acc_ops) != 0;
    const int k = 2 * seen[{d.acc, hpe}]++ + (hpe ? 1 : 0);
    if ((int)passes.size() <= k) passes.resize(k + 1);
    passes[k].push_back(d);
  }
  for (size_t k = 0; k < passes.size(); ++k) {
    auto& pass = passes[k];
    if (pass.empty()) continue;
    const bool hpe = k & 1;
    bool dil = false;
    int us = 0, ud = 0;
    for (SlotDesc& d : pass) {
      dil = dil || d.tdil > 1;
      d.tblk = b.ctx->contract_tblk;
      d.ubeg[UK_SITE] = us;
      d.ubeg[UK_DERIV] = ud;
      us += 2 * d.ntile;
      ud += 8 * d.ntile;
    }
    DevBuf ds(b.ctx, sizeof(SlotDesc) * pass.size());
    HIPCHECK(hipMemcpyAsync(ds.p, pass.data(), sizeof(SlotDesc) * pass.size(), hipMemcpyHostToDevice, b.ctx->st));
    const SlotDesc* dptr = ds.as<SlotDesc>();
    if (hpe) {
      launch_contract_local(P, dptr, (int)pass.size(), us, s_e, s_o, h.eta[0], h.eta[1], h.loc[0], h.loc[1], dil,
                            b.ctx->st);
      launch_contract_deriv(P, dptr, (int)pass.size(), ud, s_e, s_o, h.eta[0], h.eta[1], h.der[0], h.der[1], dil,
                            b.ctx->st);
    } else {
      launch_contract_local(P, dptr, (int)pass.size(), us, s_e, s_o, xi_e, xi_o, nullptr, nullptr, false, b.ctx->st);
      launch_contract_deriv(P, dptr, (int)pass.size(), ud, s_e, s_o, xi_e, xi_o, nullptr, nullptr, false, b.ctx->st);
    }
    // the descriptor buffer returns to the pool only after the stream passed it
    HIPCHECK(hipStreamSynchronize(b.ctx->st));
  }
}

static int count_active(Batch& b) {
  b.to_host_int(b.cs.active, b.h_int);
  b.sync();
  int n = 0;
  for (int i = 0; i < b.nrhs; ++i) n += b.h_int[i] != 0;
  return n;
}

// Plain CG (FP64 and low-precision tiers): iterations replayed from a HIP
// graph, convergence polled on the host between bursts.
// Compulsory HBM bytes of one hopping launch (u_e = A^-1 H_eo p_o) for the
// given active mask: every lattice's links once (8 links of 18 reals per
// output site) plus input and output spinor (24 reals each) per active rhs.
static double hop_launch_bytes(const Batch& b, int P, const int* active) {
  const double breal = P == P64 ? 8.0 : (P == P32 ? 4.0 : 2.0);
  double bytes = 0.0;
  std::vector<const void*> seen;
  for (const SlotDesc& d : b.hs) {
    int na = 0;
    for (int r = 0; r < d.nrhs; ++r) na += active[d.rhs_begin + r] != 0;
    if (!na) continue;
    bytes += na * 48.0 * breal * d.Vh;
    if (std::find(seen.begin(), seen.end(), d.gauge[0]) == seen.end()) {
      seen.push_back(d.gauge[0]);
      bytes += 144.0 * breal * d.Vh;
    }
  }
  return bytes;
}

static void run_cg_plain(Batch& b, int P, const CgFields& f, int maxiter_all, int first_burst) {
  if (count_active(b) == 0) return;
  dl_ctx* c = b.ctx;
  if (c->profile || !c->use_graph) {
    // plain launches; with profiling, HIP events bracket each hopping launch
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profile) {
      HIPCHECK(hipEventCreate(&e0));
      HIPCHECK(hipEventCreate(&e1));
    }
    std::vector<int> act(b.h_int, b.h_int + b.nrhs);
    try {
      for (int it = 0; it < maxiter_all; ++it) {
        cg_iteration(b, P, f, e0, e1);
        const int n = count_active(b);
        if (c->profile) {
          float ms = 0.f;
          HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
          double* pr = c->prof[P];
          int na = 0;
          for (int g = 0; g < b.nrhs; ++g) na += act[g] != 0;
          pr[0] += 1;
          pr[1] += ms;
          pr[2] += hop_launch_bytes(b, P, act.data());
          pr[3] += na;
        }
        act.assign(b.h_int, b.h_int + b.nrhs);
        if (n == 0) break;
      }
    } catch (...) {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      throw;
    }
    if (e0) HIPCHECK(hipEventDestroy(e0));
    if (e1) HIPCHECK(hipEventDestroy(e1));
    return;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIPCHECK(hipStreamBeginCapture(b.ctx->st, hipStreamCaptureModeThreadLocal));
  try {
    cg_iteration(b, P, f);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(b.ctx->st, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(b.ctx->st, &graph));
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);
    HIPCHECK(ie);
  }
  int it = 0;
  int burst = std::max(1, first_burst);
  try {
    while (it < maxiter_all) {
      const int n = std::min(burst, maxiter_all - it);
      for (int k = 0; k < n; ++k) HIPCHECK(hipGraphLaunch(exec, b.ctx->st));
      it += n;
      if (count_active(b) == 0) break;
      burst = 1;
    }
  } catch (...) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    throw;
  }
  HIPCHECK(hipGraphExecDestroy(exec));
  HIPCHECK(hipGraphDestroy(graph));
}

// High-precision tier, replayed from a graph: one step = decide (per rhs: a
// reliable update, a verification of a converged residual, or nothing), the
// FP64 update of the flagged rhs, its bookkeeping (restart from the true
// residual where the verification failed: p = r), then one CG iteration of
// every active rhs.  Each rhs goes through the same sequence of updates and
// iterations as with the host-driven loop, so the results are the same bit for
// bit; the host only reads the number of pending rhs between bursts.
template <class RU>
static void hp_graph_loop(Batch& b, const CgFields& f, int* flag, RU& reliable_update,
                          const std::vector<double>& rr_ru, const std::vector<int>& verified,
                          std::vector<int>& ru_count, int maxiter_all, int first_burst, double delta2) {
  dl_ctx* c = b.ctx;
  hipStream_t st = c->st;
  const int n = b.nrhs;
  DevBuf buf(c, sizeof(double) * n + sizeof(int) * (5 * (size_t)n + 1) + 16);
  HpState hp{};
  hp.rr_ru = buf.as<double>();
  int* ib = (int*)(hp.rr_ru + n);
  hp.hflag = ib;
  hp.flag = flag;
  hp.react = ib + n;
  hp.verified = ib + 2 * n;
  hp.ru_count = ib + 3 * n;
  hp.pending = ib + 4 * n;
  hp.delta2 = delta2;
  HIPCHECK(hipMemcpyAsync(hp.rr_ru, rr_ru.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(hp.verified, verified.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(hp.ru_count, ru_count.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemsetAsync(hp.hflag, 0, sizeof(int) * 2 * n, st));
  HIPCHECK(hipStreamSynchronize(st));   // the host vectors may change after this call

  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    launch_hp_decide(n, b.cs, hp, st);
    reliable_update(hp.flag);
    launch_hp_post(n, b.cs, hp, st);
    launch_convert(P32, P32, b.slots(), b.nslots, b.u_rhs, f.r, f.p, 0, hp.react, st);
    cg_iteration(b, P32, f);
    launch_hp_pending(n, b.cs, hp, st);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(st, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(st, &graph));
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);
    HIPCHECK(ie);
  }
  // the host loop's pass limit, counted in steps
  const int max_steps = 4 * maxiter_all + 16;
  int steps = 0, burst = std::max(1, first_burst);
  try {
    while (steps < max_steps) {
      const int k = std::min(burst, max_steps - steps);
      for (int i = 0; i < k; ++i) HIPCHECK(hipGraphLaunch(exec, st));
      steps += k;
      HIPCHECK(hipMemcpyAsync(b.h_int, hp.pending, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      if (b.h_int[0] == 0) break;
      burst = 1;
    }
  } catch (...) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    throw;
  }
  HIPCHECK(hipGraphExecDestroy(exec));
  HIPCHECK(hipGraphDestroy(graph));
  HIPCHECK(hipMemcpyAsync(ru_count.data(), hp.ru_count, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// the batch pipeline
// ---------------------------------------------------------------------------
static std::string hint_key(const std::vector<SlotPlan>& plan, int tier, double tol) {
  char buf[128];
  const dl_lattice* L = plan[0].lat;
  snprintf(buf, sizeof(buf), "%d:%g:%dx%dx%dx%d", tier, tol, L->dims[0], L->dims[1], L->dims[2], L->dims[3]);
  return buf;
}

static std::map<std::string, int>& iter_hints() {
  static std::map<std::string, int> m;
  return m;
}

void run_batch(dl_ctx* ctx, int tier, const std::vector<SlotPlan>& plan, const std::vector<dl_job>& jobs,
               SolveReport& rep) {
  const int P = tier_prec(tier);
  Batch b(ctx, P, plan, &jobs);
  hipStream_t st = ctx->st;
  // per-rhs tolerance and iteration cap
  {
    std::vector<double> tol2(b.nrhs);
    std::vector<int> mi(b.nrhs);
    int g = 0;
    for (const SlotPlan& sp : plan)
      for (int r = 0; r < sp.nrhs; ++r, ++g) {
        tol2[g] = jobs[sp.job].tol * jobs[sp.job].tol;
        mi[g] = jobs[sp.job].maxiter;
      }
    HIPCHECK(hipMemcpyAsync(b.cs.tol2, tol2.data(), sizeof(double) * b.nrhs, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(b.cs.maxiter, mi.data(), sizeof(int) * b.nrhs, hipMemcpyHostToDevice, st));
    b.sync();   // the host vectors end with this scope
  }
  int maxiter_all = 0;
  double tol_min = 1.0;
  bool want_true = false;
  for (const SlotPlan& sp : plan) {
    maxiter_all = std::max(maxiter_all, jobs[sp.job].maxiter);
    tol_min = std::min(tol_min, jobs[sp.job].tol);
    want_true = want_true || jobs[sp.job].report_true_resid;
  }
  const std::string hk = hint_key(plan, tier, tol_min);
  const int first_burst = iter_hints().count(hk) ? iter_hints()[hk] : 1;

  DevBuf eta_e = b.field(P), eta_o = b.field(P);
  launch_sources(P, b.slots(), b.nslots, b.u_rhs, 0, eta_e.p, st);
  launch_sources(P, b.slots(), b.nslots, b.u_rhs, 1, eta_o.p, st);
  DevBuf x = b.field(P), r = b.field(P), p = b.field(P), t = b.field(P), u = b.field(P);
  CgFields f{x.p, r.p, p.p, t.p, u.p};
  std::vector<int> ru_count(b.nrhs, 0);
  // s_e / s_o / xi fields in the contraction precision
  // The high-precision tier contracts its FP64 solution with FP64 products and
  // per-source FP64 sums (the correction term of the estimator carries the HP
  // accuracy into the loops); the other tiers contract in their storage type.
  const int PC = tier == DL_TIER_HP_FP32 ? P64 : P;
  DevBuf s64_e, s64_o;   // FP64 solution when the solve keeps one (HP tier)
  DevBuf e64_e, e64_o;   // FP64 sources (HP tier)

  if (tier != DL_TIER_HP_FP32) {
    cg_start(b, P, eta_e.p, eta_o.p, f);
    run_cg_plain(b, P, f, maxiter_all, first_burst);
    bool any_gsave = false;
    for (const SlotPlan& sp : plan) any_gsave = any_gsave || sp.gsave;
    if (any_gsave) launch_guess_store(P, b.slots(), b.nslots, b.u_rhs, x.p, st);
  } else {
    // High precision: FP32 CG with FP64 reliable updates (true residual of
    // the normal equations recomputed in FP64, solution accumulated in FP64).
    e64_e = b.field(P64);
    e64_o = b.field(P64);
    DevBuf c64 = b.field(P64), xhi = b.field(P64),
           t64 = b.field(P64), u64 = b.field(P64), ap64 = b.field(P64);
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 0, e64_e.p, st);
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 1, e64_o.p, st);
    b.dslash(P64, F_D | F_Y, CK_PREP, 1, e64_e.p, t64.p, e64_o.p, nullptr);
    b.dslash(P64, F_D, CK_MDAG1, 0, t64.p, u64.p, nullptr, nullptr);
    b.dslash(P64, F_Y | F_NORM, CK_MDAG2, 1, u64.p, c64.p, t64.p, nullptr);
    b.finalize(FK_INIT);
    launch_convert(P64, P32, b.slots(), b.nslots, b.u_rhs, c64.p, r.p, 0, nullptr, st);
    launch_convert(P64, P32, b.slots(), b.nslots, b.u_rhs, c64.p, p.p, 0, nullptr, st);
    launch_zero(P32, b.slots(), b.nslots, b.u_rhs, x.p, nullptr, st);
    launch_zero(P64, b.slots(), b.nslots, b.u_rhs, xhi.p, nullptr, st);
    DevBuf flag(ctx, sizeof(int) * std::max(b.nrhs, 1));
    std::vector<int> hflag(b.nrhs, 0), verified(b.nrhs, 0);
    std::vector<double> rr_ru(b.nrhs), cc(b.nrhs);
    b.to_host_dbl(b.cs.rr, b.h_dbl);
    b.sync();
    for (int g = 0; g < b.nrhs; ++g) rr_ru[g] = b.h_dbl[g];
    b.to_host_dbl(b.cs.cc, b.h_dbl);
    b.sync();
    for (int g = 0; g < b.nrhs; ++g) cc[g] = b.h_dbl[g];
    std::vector<double> tol2v(b.nrhs);
    std::vector<int> maxit(b.nrhs);
    {
      int g = 0;
      for (const SlotPlan& sp : plan)
        for (int q = 0; q < sp.nrhs; ++q, ++g) {
          tol2v[g] = jobs[sp.job].tol * jobs[sp.job].tol;   // as cs.tol2
          maxit[g] = jobs[sp.job].maxiter;
        }
    }
    const double delta2 = 1e-5;   // reliable update when ||r|| fell by ~300x since the last one
    // FP64 reliable update of the flagged right-hand sides: fold the FP32
    // correction into the FP64 solution, recompute the normal-equation
    // residual c - Mhat^dag Mhat xhi in FP64 and restart the FP32 residual
    // from it; leaves <r, r> of the flagged ones in cs.rr
    auto reliable_update = [&](const int* fl) {
      launch_convert(P32, P64, b.slots(), b.nslots, b.u_rhs, x.p, xhi.p, 1, fl, st);
      launch_zero(P32, b.slots(), b.nslots, b.u_rhs, x.p, fl, st);
      b.dslash(P64, 0, CK_MHAT1, 0, xhi.p, u64.p, nullptr, fl);
      b.dslash(P64, F_Y, CK_MHAT2, 1, u64.p, t64.p, xhi.p, fl);
      b.dslash(P64, F_D, CK_MDAG1, 0, t64.p, u64.p, nullptr, fl);
      b.dslash(P64, F_Y, CK_MDAG2, 1, u64.p, ap64.p, t64.p, fl);
      launch_residual_replace(b.slots(), b.nslots, b.u_rhs, c64.p, ap64.p, u64.p, r.p, b.partial.as<double>(), fl,
                              st);
      b.finalize_store(b.cs.rr, fl, b.partial.as<double>());
    };
    bool any_x0 = false;
    for (const SlotPlan& sp : plan) any_x0 = any_x0 || sp.gload;
    if (any_x0) {
      // initial guesses (odd sites) into the FP64 solution, then one reliable
      // update gives the starting residual, and p = r
      launch_guess_load(P64, b.slots(), b.nslots, b.u_rhs, xhi.p, st);
      std::vector<int> ones(b.nrhs, 1);
      HIPCHECK(hipMemcpyAsync(flag.p, ones.data(), sizeof(int) * b.nrhs, hipMemcpyHostToDevice, st));
      reliable_update(flag.as<int>());
      launch_convert(P32, P32, b.slots(), b.nslots, b.u_rhs, r.p, p.p, 0, nullptr, st);
      b.to_host_dbl(b.cs.rr, b.h_dbl);
      b.sync();
      const int zero = 0;
      for (int g = 0; g < b.nrhs; ++g) {
        rr_ru[g] = b.h_dbl[g];
        if (cc[g] > 0 && b.h_dbl[g] <= tol2v[g] * cc[g]) {   // the guess already converged
          verified[g] = 1;
          HIPCHECK(hipMemcpyAsync(b.cs.active + g, &zero, sizeof(int), hipMemcpyHostToDevice, st));
          HIPCHECK(hipMemcpyAsync(b.cs.status + g, &zero, sizeof(int), hipMemcpyHostToDevice, st));
        }
      }
      b.sync();
    }
    // The graph replays the update kernels every step, gated off for the rhs
    // not flagged; a gated-off launch still dispatches all its waves (about
    // 60 us for 50 rhs at 24^3 x 48, nine of them per step) while a host round
    // trip costs about 0.1 ms, so batches above HP_GRAPH_MAX_UNITS tiles x rhs
    // run the host-driven loop (the same bits either way).
    constexpr int HP_GRAPH_MAX_UNITS = 65536;
    if (ctx->profile || !ctx->use_graph || b.u_rhs > HP_GRAPH_MAX_UNITS) {
      // host-driven: the state goes to the host after every step, each step is
      // either the flagged rhs' reliable updates or one CG iteration
      int guard = 0;
      while (true) {
        // state after the previous step
        int* act = b.h_int;
        int* status = b.h_int + b.nrhs;
        int* iters = b.h_int + 2 * b.nrhs;
        b.to_host_int(b.cs.active, act);
        b.to_host_int(b.cs.status, status);
        b.to_host_int(b.cs.iters, iters);
        b.to_host_dbl(b.cs.rr, b.h_dbl);
        b.sync();
        bool any_flag = false, any_active = false;
        for (int g = 0; g < b.nrhs; ++g) {
          hflag[g] = 0;
          if (act[g]) {
            any_active = true;
            // no update within 100x (in |r|^2) of the target: the convergence
            // check's own FP64 residual follows shortly
            if (b.h_dbl[g] < delta2 * rr_ru[g] && b.h_dbl[g] > 1e2 * (tol2v[g] * cc[g])) hflag[g] = 1;
          } else if (status[g] == 0 && !verified[g] && cc[g] > 0) {
            hflag[g] = 2;   // iterated residual converged: verify with the true residual
          }
          any_flag = any_flag || hflag[g];
        }
        if (!any_active && !any_flag) break;
        if (++guard > 4 * maxiter_all + 16) break;
        if (any_flag) {
          std::vector<int> f01(b.nrhs);
          for (int g = 0; g < b.nrhs; ++g) f01[g] = hflag[g] != 0;
          HIPCHECK(hipMemcpyAsync(flag.p, f01.data(), sizeof(int) * b.nrhs, hipMemcpyHostToDevice, st));
          reliable_update(flag.as<int>());
          b.to_host_dbl(b.cs.rr, b.h_dbl);
          b.sync();
          std::vector<int> react;
          for (int g = 0; g < b.nrhs; ++g) {
            if (!hflag[g]) continue;
            ru_count[g]++;
            rr_ru[g] = b.h_dbl[g];
            if (hflag[g] == 2) {
              if (b.h_dbl[g] <= tol2v[g] * cc[g]) {
                verified[g] = 1;
              } else if (iters[g] < maxit[g]) {
                react.push_back(g);       // restart CG from the true residual
              } else {
                verified[g] = 1;
                status[g] = 1;
                HIPCHECK(hipMemcpyAsync(b.cs.status + g, &status[g], sizeof(int), hipMemcpyHostToDevice, st));
                b.sync();
              }
            }
          }
          if (!react.empty()) {
            std::vector<int> ga(b.nrhs, 0);
            for (int g : react) ga[g] = 1;
            HIPCHECK(hipMemcpyAsync(flag.p, ga.data(), sizeof(int) * b.nrhs, hipMemcpyHostToDevice, st));
            launch_convert(P32, P32, b.slots(), b.nslots, b.u_rhs, r.p, p.p, 0, flag.as<int>(), st);
            const int one = 1;
            for (int g : react) {
              HIPCHECK(hipMemcpyAsync(b.cs.active + g, &one, sizeof(int), hipMemcpyHostToDevice, st));
              HIPCHECK(hipMemcpyAsync(b.cs.status + g, &one, sizeof(int), hipMemcpyHostToDevice, st));
            }
            b.sync();
          }
          continue;
        }
        if (ctx->profile) {
          // time this iteration's hopping launch (u_e = A^-1 H_eo p_o) as the plain CG does
          std::vector<int> act(b.nrhs);
          b.to_host_int(b.cs.active, act.data());
          b.sync();
          hipEvent_t e0, e1;
          HIPCHECK(hipEventCreate(&e0));
          HIPCHECK(hipEventCreate(&e1));
          cg_iteration(b, P32, f, e0, e1);
          HIPCHECK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          double* pr = ctx->prof[P32];
          int na = 0;
          for (int g = 0; g < b.nrhs; ++g) na += act[g] != 0;
          pr[0] += 1;
          pr[1] += ms;
          pr[2] += hop_launch_bytes(b, P32, act.data());
          pr[3] += na;
        } else {
          cg_iteration(b, P32, f);
        }
      }
    } else {
      hp_graph_loop(b, f, flag.as<int>(), reliable_update, rr_ru, verified, ru_count, maxiter_all, first_burst,
                    delta2);
    }
    // fold the last FP32 correction; reconstruct in FP64
    launch_convert(P32, P64, b.slots(), b.nslots, b.u_rhs, x.p, xhi.p, 1, nullptr, st);
    s64_o = std::move(xhi);
    s64_e = b.field(P64);
    b.dslash(P64, F_Y, CK_RECON, 0, s64_o.p, s64_e.p, e64_e.p, nullptr);
  }

  // ---- solution, xi fields, contractions ---------------------------------
  // fields in the contraction precision: s_o, s_e, xi_e, xi_o (LP / FP64
  // tiers reuse x, r, p, t; the HP tier its FP64 solution and two FP64 fields)
  bool any_acc = false, any_sol = false;
  for (const SlotPlan& sp : plan) {
    any_acc = any_acc || sp.acc;
    any_sol = any_sol || sp.sol_user;
  }
  void *so_f = x.p, *se_f = r.p, *xe_f = p.p, *xo_f = t.p;
  const void *eta_ef = eta_e.p, *eta_of = eta_o.p;
  DevBuf xi64_e, xi64_o;
  bool xi_e_done = false;
  if (tier == DL_TIER_HP_FP32) {
    so_f = s64_o.p;
    se_f = s64_e.p;
    eta_ef = e64_e.p;
    eta_of = e64_o.p;
    if (any_acc) {
      xi64_e = b.field(P64);
      xi64_o = b.field(P64);
      xe_f = xi64_e.p;
      xo_f = xi64_o.p;
    }
  } else if (any_acc && !b.has_clover) {
    // s_e and xi_e = s_e - kappa H_eo s_o share the hop H_eo s_o (with a clover
    // term xi_e = (1 + C) s_e - kappa H_eo s_o: two launches below)
    b.dslash(P, F_Y | F_DUAL, CK_RECON_XI, 0, x.p, r.p, eta_e.p, nullptr, nullptr, nullptr, nullptr, p.p);
    xi_e_done = true;
  } else {
    b.dslash(P, F_Y, CK_RECON, 0, x.p, r.p, eta_e.p, nullptr);
  }
  if (any_acc) {
    int hpe = 0;
    bool any_plain = false;
    for (const SlotPlan& sp : plan) {
      if (!sp.acc) continue;
      const int o = DL_OPS_HPE_ORDER(jobs[sp.job].accum->ops);
      if (o) hpe = o;
      else any_plain = true;
    }
    if (any_plain) {
      if (!xi_e_done) b.dslash(PC, F_Y, CK_XI, 0, so_f, xe_f, se_f, nullptr);
      b.dslash(PC, F_Y, CK_XI, 1, se_f, xo_f, so_f, nullptr);
    }
    HpeFields h;
    DevBuf fa_e, fa_o, fb_e, fb_o;
    if (hpe) {
      // phi_k = (kappa B H)^k s, k = 1..n, alternating between two fields;
      // the source eta (still intact) is the other vector
      fa_e = b.field(PC); fa_o = b.field(PC); fb_e = b.field(PC); fb_o = b.field(PC);
      const void* in_e = se_f;
      const void* in_o = so_f;
      for (int k = 1; k <= hpe; ++k) {
        void* oe = (k & 1) ? fa_e.p : fb_e.p;
        void* oo = (k & 1) ? fa_o.p : fb_o.p;
        b.dslash(PC, 0, CK_KBH, 0, in_o, oe, nullptr, nullptr);
        b.dslash(PC, 0, CK_KBH, 1, in_e, oo, nullptr, nullptr);
        in_e = oe;
        in_o = oo;
      }
      const int nd = std::min(hpe, 3);
      h.eta[0] = eta_ef; h.eta[1] = eta_of;
      h.loc[0] = (hpe & 1) ? fa_e.p : fb_e.p; h.loc[1] = (hpe & 1) ? fa_o.p : fb_o.p;
      h.der[0] = (nd & 1) ? fa_e.p : fb_e.p; h.der[1] = (nd & 1) ? fa_o.p : fb_o.p;
    }
    contract_passes(b, PC, se_f, so_f, xe_f, xo_f, h);
  }
  if (any_sol) {
    if (tier == DL_TIER_HP_FP32) {
      launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 0, s64_e.p, st);
      launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 1, s64_o.p, st);
    } else {
      launch_unpack(P, b.slots(), b.nslots, b.u_rhs, 0, r.p, st);
      launch_unpack(P, b.slots(), b.nslots, b.u_rhs, 1, x.p, st);
    }
  }

  // ---- report ---------------------------------------------------------------
  rep.iters.assign(b.nrhs, 0);
  rep.status.assign(b.nrhs, 0);
  rep.ru = ru_count;
  rep.rel.assign(b.nrhs, 0.0);
  rep.truer.assign(b.nrhs, -1.0);
  b.to_host_int(b.cs.iters, b.h_int);
  b.to_host_int(b.cs.status, b.h_int + b.nrhs);
  b.to_host_dbl(b.cs.rr, b.h_dbl);
  b.to_host_dbl(b.cs.cc, b.h_dbl + b.nrhs);
  b.sync();
  int min_it = 1 << 30;
  for (int g = 0; g < b.nrhs; ++g) {
    rep.iters[g] = b.h_int[g];
    rep.status[g] = b.h_int[b.nrhs + g];
    const double cc = b.h_dbl[b.nrhs + g];
    rep.rel[g] = cc > 0 ? std::sqrt(b.h_dbl[g] / cc) : 0.0;
    if (rep.status[g] == 0) min_it = std::min(min_it, rep.iters[g]);
  }
  if (min_it < (1 << 30)) iter_hints()[hk] = std::max(1, min_it);

  if (want_true) {
    // ||eta - M s|| / ||eta|| with the FP64 operator
    DevBuf se = b.field(P64), so = b.field(P64), ee = b.field(P64), eo = b.field(P64), me = b.field(P64),
           mo = b.field(P64);
    if (tier == DL_TIER_HP_FP32) {
      launch_convert(P64, P64, b.slots(), b.nslots, b.u_rhs, s64_e.p, se.p, 0, nullptr, st);
      launch_convert(P64, P64, b.slots(), b.nslots, b.u_rhs, s64_o.p, so.p, 0, nullptr, st);
    } else {
      launch_convert(P, P64, b.slots(), b.nslots, b.u_rhs, r.p, se.p, 0, nullptr, st);
      launch_convert(P, P64, b.slots(), b.nslots, b.u_rhs, x.p, so.p, 0, nullptr, st);
    }
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 0, ee.p, st);
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 1, eo.p, st);
    b.dslash(P64, F_Y, CK_MFULL, 0, so.p, me.p, se.p, nullptr);
    b.dslash(P64, F_Y, CK_MFULL, 1, se.p, mo.p, so.p, nullptr);
    DevBuf gate = ones_gate(b);
    DevBuf out4(ctx, sizeof(double) * 4 * std::max(b.nrhs, 1));
    double* o = out4.as<double>();
    launch_diff_norms(b.slots(), b.nslots, b.u_rhs, me.p, ee.p, b.partial.as<double>(), b.partial2.as<double>(), st);
    b.finalize_store(o, gate.as<int>(), b.partial.as<double>());
    b.finalize_store(o + b.nrhs, gate.as<int>(), b.partial2.as<double>());
    launch_diff_norms(b.slots(), b.nslots, b.u_rhs, mo.p, eo.p, b.partial.as<double>(), b.partial2.as<double>(), st);
    b.finalize_store(o + 2 * b.nrhs, gate.as<int>(), b.partial.as<double>());
    b.finalize_store(o + 3 * b.nrhs, gate.as<int>(), b.partial2.as<double>());
    std::vector<double> h(4 * b.nrhs);
    HIPCHECK(hipMemcpyAsync(h.data(), o, sizeof(double) * 4 * b.nrhs, hipMemcpyDeviceToHost, st));
    b.sync();
    int g = 0;
    for (const SlotPlan& sp : plan)
      for (int q = 0; q < sp.nrhs; ++q, ++g)
        if (jobs[sp.job].report_true_resid) {
          const double den = h[b.nrhs + g] + h[3 * b.nrhs + g];
          rep.truer[g] = den > 0 ? std::sqrt((h[g] + h[2 * b.nrhs + g]) / den) : 0.0;
        }
  }
  b.sync();
}

// ---------------------------------------------------------------------------
// single operators (verification entry point)
// ---------------------------------------------------------------------------
void apply_op(dl_lattice* lat, int op, int tier, const double* in, double* out, int nrhs) {
  dl_ctx* ctx = lat->ctx;
  const int P = tier_prec(tier);
  std::vector<SlotPlan> plan;
  const long long V = lat->V;
  SlotPlan sp{};
  sp.lat = lat;
  sp.nrhs = nrhs;
  sp.src_user = in;
  sp.sol_user = out;
  plan.push_back(sp);
  Batch b(ctx, P, plan, nullptr);
  hipStream_t st = ctx->st;
  DevBuf ie = b.field(P), io = b.field(P), oe = b.field(P), oo = b.field(P), tmp = b.field(P);
  launch_sources(P, b.slots(), b.nslots, b.u_rhs, 0, ie.p, st);
  launch_sources(P, b.slots(), b.nslots, b.u_rhs, 1, io.p, st);
  switch (op) {
    case DL_OP_HOP:
      b.dslash(P, 0, CK_HOP, 0, io.p, oe.p, nullptr, nullptr);
      b.dslash(P, 0, CK_HOP, 1, ie.p, oo.p, nullptr, nullptr);
      break;
    case DL_OP_M:
      b.dslash(P, F_Y, CK_MFULL, 0, io.p, oe.p, ie.p, nullptr);
      b.dslash(P, F_Y, CK_MFULL, 1, ie.p, oo.p, io.p, nullptr);
      break;
    case DL_OP_MDAG:
      b.dslash(P, F_D | F_Y, CK_MDAGFULL, 0, io.p, oe.p, ie.p, nullptr);
      b.dslash(P, F_D | F_Y, CK_MDAGFULL, 1, ie.p, oo.p, io.p, nullptr);
      break;
    case DL_OP_MHAT:
      b.dslash(P, 0, CK_MHAT1, 0, io.p, tmp.p, nullptr, nullptr);
      b.dslash(P, F_Y, CK_MHAT2, 1, tmp.p, oo.p, io.p, nullptr);
      launch_zero(P, b.slots(), b.nslots, b.u_rhs, oe.p, nullptr, st);
      break;
    case DL_OP_MHAT_DAG:
      b.dslash(P, F_D, CK_MDAG1, 0, io.p, tmp.p, nullptr, nullptr);
      b.dslash(P, F_Y, CK_MDAG2, 1, tmp.p, oo.p, io.p, nullptr);
      launch_zero(P, b.slots(), b.nslots, b.u_rhs, oe.p, nullptr, st);
      break;
    default:
      throw Error(DL_EINVAL, "unknown operator " + std::to_string(op));
  }
  launch_unpack(P, b.slots(), b.nslots, b.u_rhs, 0, oe.p, st);
  launch_unpack(P, b.slots(), b.nslots, b.u_rhs, 1, oo.p, st);
  (void)V;
  b.sync();
}

void fill_noise_fields(dl_ctx* ctx, const std::vector<SlotPlan>& plan, const std::vector<dl_job>& jobs) {
  Batch b(ctx, P64, plan, &jobs);
  DevBuf e = b.field(P64), o = b.field(P64);
  launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 0, e.p, ctx->st);
  launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 1, o.p, ctx->st);
  launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 0, e.p, ctx->st);
  launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 1, o.p, ctx->st);
  b.sync();
}

// ---------------------------------------------------------------------------
// autotuner: slot shape of the hopping kernel
// ---------------------------------------------------------------------------
// Within a slot the hopping kernel walks tile-major over its right-hand
// sides, so one tile's links are fetched once for all of them; but the larger
// the block, the more data the neighbour tiles (z: ~4.5 tb tiles away, t:
// next block) need L2 to hold.  The time-block depth tb of the tile order
// trades t- against z-neighbour distance.  Both depend on lattice, precision
// and batch size and are measured: the hopping launch is timed on a scratch
// batch for every (block, tb) candidate and the fastest kept, in memory and in
// a JSON cache (DL_TUNE_CACHE, default ~/.cache/discloop/tune-gfx950.json).
static std::string tune_file() {
  const char* e = getenv("DL_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/discloop/tune-gfx950.json";
}

static void tune_load(dl_ctx* ctx) {
  if (ctx->tune_loaded) return;
  ctx->tune_loaded = true;
  ctx->tune_path = tune_file();
  FILE* f = fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  // a flat JSON object {"key": value, ...}: every quoted key followed by ':'
  // and a positive integer is taken, whatever the line breaks
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  fclose(f);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    size_t q = end + 1;
    while (q < text.size() && isspace((unsigned char)text[q])) ++q;
    if (q < text.size() && text[q] == ':') {
      char* stop = nullptr;
      const long v = strtol(text.c_str() + q + 1, &stop, 10);
      if (stop != text.c_str() + q + 1 && v >= 1 && v < (1 << 30)) ctx->tune[key] = (int)v;
    }
    pos = end + 1;
  }
}

static void tune_save(dl_ctx* ctx) {
  const std::string& p = ctx->tune_path;
  const size_t slash = p.find_last_of('/');
  if (slash != std::string::npos) {
    std::string dir = p.substr(0, slash), acc;
    for (size_t i = 0; i <= dir.size(); ++i) {
      if (i == dir.size() || dir[i] == '/') {
        if (!acc.empty()) (void)mkdir(acc.c_str(), 0755);
      }
      if (i < dir.size()) acc += dir[i];
    }
  }
  FILE* f = fopen(p.c_str(), "w");
  if (!f) return;   // an unwritable cache only costs a re-tune
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : ctx->tune) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < ctx->tune.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

TuneChoice autotune_block(dl_ctx* ctx, dl_lattice* lat, int prec, int nsrc_hint) {
  if (nsrc_hint <= 1) return {1, TBLK_DEFAULT};
  tune_load(ctx);
  // batch size class of the measurement: the next power of two of the job's
  // sources, between 16 and 128
  int total = 16;
  while (total < nsrc_hint && total < 128) total *= 2;
  static const char* pname[4] = {"fp64", "fp32", "bf16", "fp16"};
  char key[96], tkey[100];
  // the LDS-staged hop has its own best slot shape
  int bb_y, bb_z, bb_s;
  size_t bb_l;
  const bool blk = (prec == PB16 || prec == PH16) && ctx->block_hop && lat->csw == 0.0 &&
                   blk_shape(lat->dims, bb_y, bb_z, bb_s, bb_l);
  snprintf(key, sizeof(key), "%dx%dx%dx%d:%s:%d%s", lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3],
           pname[prec], total, blk ? ":blk" : "");
  snprintf(tkey, sizeof(tkey), "%s:t", key);
  auto it = ctx->tune.find(key);
  auto jt = ctx->tune.find(tkey);
  if (it == ctx->tune.end() || jt == ctx->tune.end()) {
    const int cands[] = {1, 2, 4, 8, 16, 32, 64, 128};
    const int tbs[] = {1, 2, 4, 8};
    double best_t = 1e300;
    int best = 16, best_tb = TBLK_DEFAULT;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    for (int N : cands) {
      if (N > total) break;
      for (int tb : tbs) {
        std::vector<SlotPlan> plan;
        for (int k = 0; k < total; k += N) {
          SlotPlan sp{};
          sp.lat = lat;
          sp.nrhs = std::min(N, total - k);
          sp.tblk = tb;
          plan.push_back(sp);
        }
        Batch b(ctx, prec, plan, nullptr);
        DevBuf in = b.field(prec), out = b.field(prec);
        HIPCHECK(hipMemsetAsync(in.p, 0, b.field_bytes(prec), ctx->st));
        b.dslash(prec, 0, CK_MHAT1, 0, in.p, out.p, nullptr, nullptr);
        HIPCHECK(hipEventRecord(e0, ctx->st));
        for (int rep = 0; rep < 3; ++rep) b.dslash(prec, 0, CK_MHAT1, 0, in.p, out.p, nullptr, nullptr);
        HIPCHECK(hipEventRecord(e1, ctx->st));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_t * 0.98) {   // prefer the earlier candidate unless a later one is clearly faster
          best_t = ms;
          best = N;
          best_tb = tb;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tune[key] = best;
    ctx->tune[tkey] = best_tb;
    tune_save(ctx);
    it = ctx->tune.find(key);
    jt = ctx->tune.find(tkey);
  }
  ctx->last_tune_block = it->second;
  return {std::max(1, std::min(nsrc_hint, it->second)), jt->second};
}

bool solve_jobs(dl_ctx* ctx, const std::vector<dl_job>& J, dl_src_stats* stats) {
  const int njobs = (int)J.size();
  std::vector<long long> first_stat(njobs + 1, 0);
  auto ncomp = [](const dl_job& q) { return std::max(q.tdil, 1); };
  for (int j = 0; j < njobs; ++j) first_stat[j + 1] = first_stat[j] + (long long)J[j].nsrc * ncomp(J[j]);
  bool all_ok = true;
  const double budget = ctx->inflight_mb * 1048576.0;
  // solutions that HP jobs start from: the caller's sol_out, or a library
  // buffer kept for this call (the lower tiers run first)
  std::vector<void*> gbuf(njobs, nullptr);
  std::vector<DevBuf> keep;
  for (int j = 0; j < njobs; ++j) {
    const int g = J[j].guess_from - 1;
    if (g < 0 || gbuf[g] || J[g].nsrc == 0) continue;
    const size_t per = (size_t)chunks_of(tier_prec(J[g].tier)) * pad_half(J[g].lat->Vh) * 16;
    keep.emplace_back(ctx, (size_t)J[g].nsrc * ncomp(J[g]) * per);
    gbuf[g] = keep.back().p;
  }
  const int max_rhs = ctx->inflight_rhs;
  const int tiers[4] = {DL_TIER_FP64, DL_TIER_LP_BF16, DL_TIER_LP_FP16, DL_TIER_HP_FP32};
  for (int tier : tiers) {
    const int P = tier_prec(tier);
    std::vector<SlotPlan> all;
    for (int j = 0; j < njobs; ++j) {
      const dl_job& q = J[j];
      if (q.tier != tier || q.nsrc == 0) continue;
      const TuneChoice tc =
          q.rhs_block > 0 ? TuneChoice{q.rhs_block, TBLK_DEFAULT} : autotune_block(ctx, q.lat, P, q.nsrc * ncomp(q));
      const int N = tc.block;
      const long long V = q.lat->V;
      // job entries e (time dilution: component-major, e = c * nsrc + vector),
      // N per slot; a diluted slot may span components (each rhs finds its
      // component and noise vector from its entry)
      const bool dil = q.tdil > 1;
      const long long nent = (long long)q.nsrc * ncomp(q);
      for (long long e = 0; e < nent; e += N) {
        SlotPlan sp{};
        sp.lat = q.lat;
        sp.job = j;
        sp.job_first = (int)e;
        sp.nrhs = (int)std::min<long long>(N, nent - e);
        sp.src0 = dil ? q.first_src : q.first_src + e;
        sp.src_user = q.src_in ? q.src_in + (dil ? 0 : (size_t)e * V * 24) : nullptr;
        sp.sol_user = q.sol_out ? q.sol_out + (size_t)e * V * 24 : nullptr;
        sp.tdil = dil ? q.tdil : 0;
        sp.tclen = q.nsrc;
        if (gbuf[j]) {
          const size_t per = (size_t)chunks_of(P) * pad_half(q.lat->Vh) * 16;
          sp.gsave = (char*)gbuf[j] + (size_t)e * per;
        }
        if (q.guess_from) {
          const dl_job& h = J[q.guess_from - 1];
          const int PG = tier_prec(h.tier);
          const size_t per = (size_t)chunks_of(PG) * pad_half(h.lat->Vh) * 16;
          sp.gload = (const char*)gbuf[q.guess_from - 1] + (size_t)e * per;
          sp.gprec = PG;
        }
        sp.acc = q.accum ? q.accum->acc[q.accum_set] : nullptr;
        sp.tblk = tc.tblk;
        all.push_back(sp);
      }
    }
    // batches bounded by device memory and right-hand-side count
    size_t i = 0;
    while (i < all.size()) {
      std::vector<SlotPlan> wave;
      double bytes = 0;
      int nrhs = 0;
      while (i < all.size()) {
        const SlotPlan& sp = all[i];
        const double vp = (double)pad_half(sp.lat->Vh);
        double per = vp * sp.nrhs * (7.0 * chunks_of(P) * 16);
        if (tier == DL_TIER_HP_FP32) per += vp * sp.nrhs * 11.0 * 192;
        if (J[sp.job].report_true_resid) per += vp * sp.nrhs * 6.0 * 192;
        const int PCk = tier == DL_TIER_HP_FP32 ? P64 : P;
        if (J[sp.job].accum && DL_OPS_HPE_ORDER(J[sp.job].accum->ops)) per += vp * sp.nrhs * (4.0 * chunks_of(PCk) * 16);
        if (!wave.empty() && (bytes + per > budget || nrhs + sp.nrhs > max_rhs)) break;
        wave.push_back(sp);
        bytes += per;
        nrhs += sp.nrhs;
        ++i;
      }
      SolveReport rep;
      run_batch(ctx, tier, wave, J, rep);
      int g = 0;
      for (const SlotPlan& sp : wave) {
        for (int r = 0; r < sp.nrhs; ++r, ++g) {
          if (rep.status[g] != 0) all_ok = false;
          if (stats) {
            dl_src_stats& s = stats[first_stat[sp.job] + sp.job_first + r];
            s.iters = rep.iters[g];
            s.status = rep.status[g];
            s.rel_resid = rep.rel[g];
            s.true_resid = rep.truer[g];
            s.reliable_updates = rep.ru[g];
            s.pad = 0;
          }
        }
        const dl_job& q = J[sp.job];
        if (q.accum)   // noise vectors: the entries of component 0
          q.accum->count[q.accum_set] += std::max(0, std::min(sp.job_first + sp.nrhs, q.nsrc) - sp.job_first);
      }
    }
  }
  return all_ok;
}

// ---------------------------------------------------------------------------
// backward pass: one adjoint solve per source
// (gradients of a real loss F as dF/dRe + i dF/dIm for complex quantities)
//   grad_eta = M^-dag (B + B^dag) s,  M^-dag = gamma5 M(-mu)^-1 gamma5
//   dF/dmu   = (1/mu) Re sum_r s^dag gamma5 Q_t3 s - 2 kappa Im sum_r <s, gamma5 z>
// ---------------------------------------------------------------------------
void loops_backward(dl_ctx* ctx, const dl_job& job, int p2max, const double* grad_loops, double* grad_eta,
                    double* grad_mu) {
  dl_lattice* L = job.lat;
  if (!L || !L->gauge_set || !L->params_set) throw Error(DL_EINVAL, "dl_loops_backward: lattice not ready");
  if (job.nsrc < 1) throw Error(DL_EINVAL, "dl_loops_backward: nsrc must be >= 1");
  if (p2max < 0) throw Error(DL_EINVAL, "dl_loops_backward: p2max must be >= 0");
  if (!(job.tol > 0) || job.maxiter < 1) throw Error(DL_EINVAL, "dl_loops_backward: bad tol / maxiter");
  if (job.noise == DL_NOISE_USER && !job.src_in) throw Error(DL_EINVAL, "dl_loops_backward: USER noise needs src_in");
  if (grad_mu && L->mu == 0)   // the tau_3 term of dF/dmu is taken as (1/mu) x its mu-weighted sum
    throw Error(DL_EINVAL, "dl_loops_backward: dF/dmu needs mu != 0");
  (void)tier_prec(job.tier);
  hipStream_t st = ctx->st;
  const int ops = job.accum ? job.accum->ops : (job.grad_ops ? job.grad_ops : DL_OPS_LOCAL | DL_OPS_DERIV);
  const int nops = (ops & DL_OPS_DERIV) ? 5 : 1;
  const int N = job.nsrc;
  const long long V = L->V;
  const int X = L->dims[0], Y = L->dims[1], Z = L->dims[2], T = L->dims[3];
  // 1. solutions: the caller's checkpoint (job.sol_out) or recomputed
  DevBuf s_buf;
  const double* s_lex = job.sol_out;
  if (!s_lex) {
    s_buf = DevBuf(ctx, (size_t)N * V * 192);
    std::vector<dl_job> J(1, job);
    J[0].sol_out = s_buf.as<double>();
    J[0].accum = nullptr;
    J[0].report_true_resid = 0;
    solve_jobs(ctx, J, nullptr);
    s_lex = s_buf.as<double>();
  }
  // 2. Omega fields from the upstream gradient
  std::vector<std::array<int, 3>> moms;
  {
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = -(L->dims[k] / 2) + 1;
      hi[k] = L->dims[k] / 2;
    }
    for (int a = lo[0]; a <= hi[0]; ++a)
      for (int b = lo[1]; b <= hi[1]; ++b)
        for (int c = lo[2]; c <= hi[2]; ++c)
          if (a * a + b * b + c * c <= p2max) moms.push_back({a, b, c});
    std::sort(moms.begin(), moms.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
      const int nx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2], ny = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
      return nx != ny ? nx < ny : x < y;
    });
  }
  const int np = (int)moms.size();
  std::vector<double> ph[3];
  const int ext[3] = {X, Y, Z};
  for (int k = 0; k < 3; ++k) {
    ph[k].resize((size_t)np * ext[k] * 2);
    for (int p = 0; p < np; ++p)
      for (int x = 0; x < ext[k]; ++x) {
        const double ang = -2.0 * M_PI * (double)moms[p][k] * x / ext[k];
        ph[k][2 * ((size_t)p * ext[k] + x)] = std::cos(ang);
        ph[k][2 * ((size_t)p * ext[k] + x) + 1] = std::sin(ang);
      }
  }
  DevBuf dph[3];
  for (int k = 0; k < 3; ++k) {
    dph[k] = DevBuf(ctx, std::max<size_t>(ph[k].size() * sizeof(double), 16));
    HIPCHECK(hipMemcpyAsync(dph[k].p, ph[k].data(), ph[k].size() * sizeof(double), hipMemcpyHostToDevice, st));
  }
  const size_t gbytes = sizeof(double) * 2 * 2 * nops * 16 * (size_t)T * np;
  DevBuf dg(ctx, std::max<size_t>(gbytes, 16));
  HIPCHECK(hipMemcpyAsync(dg.p, grad_loops, gbytes, hipMemcpyHostToDevice, st));
  DevBuf omega(ctx, sizeof(double) * 2 * 2 * nops * 16 * (size_t)V);
  launch_omega(dg.as<double>(), nops, X, Y, Z, T, np, dph[0].as<double>(), dph[1].as<double>(), dph[2].as<double>(),
               L->kappa, L->mu, N, omega.as<double>(), st);
  // 3. (B + B^dag) s, multiplied by gamma5: the right-hand side of M(-mu) z' = gamma5 v
  DevBuf v_lex(ctx, (size_t)N * V * 192), z_lex(ctx, (size_t)N * V * 192);
  std::vector<dl_job> J(1, job);
  J[0].noise = DL_NOISE_USER;
  std::vector<SlotPlan> plan;
  const int blk = std::max(1, std::min(N, 64));
  for (int k = 0; k < N; k += blk) {
    SlotPlan sp{};
    sp.lat = L;
    sp.job = 0;
    sp.job_first = k;
    sp.nrhs = std::min(blk, N - k);
    sp.src_user = s_lex + (size_t)k * V * 24;
    sp.sol_user = v_lex.as<double>() + (size_t)k * V * 24;
    plan.push_back(sp);
  }
  double sums[4] = {0, 0, 0, 0};
  {
    Batch b(ctx, P64, plan, &J);
    DevBuf se = b.field(P64), so = b.field(P64), me = b.field(P64), mo = b.field(P64), ae = b.field(P64),
           ao = b.field(P64), ce = b.field(P64), co = b.field(P64);
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 0, se.p, st);
    launch_sources(P64, b.slots(), b.nslots, b.u_rhs, 1, so.p, st);
    b.dslash(P64, F_Y, CK_XI, 0, so.p, me.p, se.p, nullptr);
    b.dslash(P64, F_Y, CK_XI, 1, se.p, mo.p, so.p, nullptr);
    DevBuf parts(ctx, sizeof(double) * 4 * std::max(b.u_rhs, 1)), red(ctx, sizeof(double) * 8);
    double* pr = parts.as<double>();
    const long long nu = std::max(b.u_rhs, 1);
    launch_insert_apply(b.slots(), b.nslots, b.u_rhs, 0, nops, omega.as<double>(), se.p, so.p, me.p, mo.p, ae.p,
                        ce.p, pr, pr + nu, st);
    launch_insert_apply(b.slots(), b.nslots, b.u_rhs, 1, nops, omega.as<double>(), se.p, so.p, me.p, mo.p, ao.p,
                        co.p, pr + 2 * nu, pr + 3 * nu, st);
    // gamma5 v = gamma5 C - kappa H gamma5 A
    b.dslash(P64, F_D | F_Y, CK_G5V, 0, ao.p, se.p, ce.p, nullptr);
    b.dslash(P64, F_D | F_Y, CK_G5V, 1, ae.p, so.p, co.p, nullptr);
    launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 0, se.p, st);
    launch_unpack(P64, b.slots(), b.nslots, b.u_rhs, 1, so.p, st);
    for (int k = 0; k < 4; ++k) launch_sum(pr + k * nu, b.u_rhs, red.as<double>() + k, st);
    double h[4];
    HIPCHECK(hipMemcpyAsync(h, red.p, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    sums[0] = h[0] + h[2];   // Re sum s^dag gamma5 Q_t3 s
    sums[1] = h[1] + h[3];
  }
  // 4. adjoint solves M(-mu) z' = gamma5 v
  dl_lattice Lm = *L;
  Lm.mu = -L->mu;
  {
    std::vector<dl_job> A(1, job);
    A[0].lat = &Lm;
    A[0].noise = DL_NOISE_USER;
    A[0].src_in = v_lex.as<double>();
    A[0].sol_out = z_lex.as<double>();
    A[0].accum = nullptr;
    A[0].report_true_resid = 0;
    A[0].first_src = 0;
    solve_jobs(ctx, A, nullptr);
  }
  // 5. grad_eta = gamma5 z', and <s, z'> for the mu-derivative
  const long long nsite = (long long)N * V;
  const long long nblk = (nsite + 255) / 256;
  DevBuf parts(ctx, sizeof(double) * 2 * nblk), red(ctx, sizeof(double) * 2);
  DevBuf gtmp;
  double* gout = grad_eta;
  if (!gout) {
    gtmp = DevBuf(ctx, (size_t)nsite * 192);
    gout = gtmp.as<double>();
  }
  launch_g5_lex(z_lex.as<double>(), gout, s_lex, nsite, parts.as<double>(), parts.as<double>() + nblk, st);
  launch_sum(parts.as<double>(), nblk, red.as<double>(), st);
  launch_sum(parts.as<double>() + nblk, nblk, red.as<double>() + 1, st);
  double h[2];
  HIPCHECK(hipMemcpyAsync(h, red.p, sizeof(h), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (grad_mu) *grad_mu = sums[0] / L->mu - 2.0 * L->kappa * h[1];
}

}  // namespace dl
