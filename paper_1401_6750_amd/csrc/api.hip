// The C ABI (include/discloop.h): argument checks, job planning and error
// translation.  No C++ exception crosses this boundary.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

using namespace dl;

// Device scratch of dl_loops_noalloc: the projection's tables and partial
// sums live here instead of in pool memory.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code this name is only
// a stand-in for the symbol: the device address of a GPU's copy comes from
// hipGetSymbolAddress with that GPU current (scratch_address, called by
// dl_create), and only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[DL_LOOPS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_ptr;   // device -> address of its copy

// Address of `device`'s copy of the scratch array; `device` must be current.
static unsigned char* scratch_address(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(DL_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_ptr[device] = (unsigned char*)ptr;
  return (unsigned char*)ptr;
}

static thread_local std::string g_last_error;

template <class F>
static int guarded(F&& f) {
  try {
    int rc = f();
    if (rc >= 0) g_last_error.clear();
    return rc;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DL_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DL_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    return DL_EHIP;
  }
}

static void require(bool ok, const std::string& msg) {
  if (!ok) throw Error(DL_EINVAL, msg);
}

extern "C" {

const char* dl_last_error(void) { return g_last_error.c_str(); }

const char* dl_version(void) { return "discloop-gfx950 0.1"; }

int dl_create(dl_ctx** out, int device, void* hip_stream) {
  return guarded([&] {
    require(out != nullptr, "dl_create: out is NULL");
    int n = 0;
    HIPCHECK(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, "dl_create: no HIP device " + std::to_string(device));
    HIPCHECK(hipSetDevice(device));
    auto* c = new dl_ctx();
    c->device = device;
    c->user_stream = (hipStream_t)hip_stream;
    try {
      HIPCHECK(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
      init_gamma_table();
      c->scratch = scratch_address(device);
    } catch (...) {
      if (c->st) (void)hipStreamDestroy(c->st);
      if (c->ev) (void)hipEventDestroy(c->ev);
      delete c;
      throw;
    }
    *out = c;
    return 0;
  });
}

int dl_destroy(dl_ctx* ctx) {
  return guarded([&] {
    if (!ctx) return 0;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->st);
    ctx->pool.clear();
    (void)hipEventDestroy(ctx->ev);
    (void)hipStreamDestroy(ctx->st);
    delete ctx;
    return 0;
  });
}

int dl_lattice_create(dl_ctx* ctx, const int dims[4], int t_bc, dl_lattice** out) {
  return guarded([&] {
    require(ctx && dims && out, "dl_lattice_create: NULL argument");
    for (int k = 0; k < 4; ++k)
      require(dims[k] >= 2 && dims[k] % 2 == 0, "dl_lattice_create: every extent must be even and >= 2");
    require(t_bc == 1 || t_bc == -1, "dl_lattice_create: t_bc must be +1 or -1");
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    // kernels address a row of per-parity 16-byte entries with a 32-bit byte
    // offset: at most 2^28 entries per row
    require(pad_half(V / 2) < (1ll << 28), "dl_lattice_create: lattice too large (more than 2^28 sites per parity)");
    HIPCHECK(hipSetDevice(ctx->device));
    auto* L = new dl_lattice();
    L->ctx = ctx;
    std::memcpy(L->dims, dims, sizeof(L->dims));
    L->bc = t_bc;
    L->V = V;
    L->Vh = V / 2;
    try {
      for (int p = 0; p < 4; ++p) {
        const size_t bytes = (size_t)pad_half(V / 2) * link_rows(p) * 16;
        if (hipMalloc(&L->gauge[p], bytes) != hipSuccess) {
          (void)hipGetLastError();
          throw Error(DL_ENOMEM, "dl_lattice_create: gauge allocation failed");
        }
      }
    } catch (...) {
      for (int p = 0; p < 4; ++p)
        if (L->gauge[p]) (void)hipFree(L->gauge[p]);
      delete L;
      throw;
    }
    *out = L;
    return 0;
  });
}

static void clover_free(dl_lattice* lat) {
  if (lat->clv64) (void)hipFree(lat->clv64);
  if (lat->clv32) (void)hipFree(lat->clv32);
  lat->clv64 = lat->clv32 = nullptr;
}

int dl_lattice_destroy(dl_lattice* lat) {
  return guarded([&] {
    if (!lat) return 0;
    (void)hipSetDevice(lat->ctx->device);
    (void)hipStreamSynchronize(lat->ctx->st);
    for (int p = 0; p < 4; ++p)
      if (lat->gauge[p]) (void)hipFree(lat->gauge[p]);
    clover_free(lat);
    delete lat;
    return 0;
  });
}

// (Re)build the clover site matrices of a lattice with a clover term once its
// gauge field and kappa, mu are set (they depend on all three).
static void clover_rebuild(dl_lattice* lat) {
  if (lat->csw == 0.0 || !lat->gauge_set || !lat->params_set) return;
  dl_ctx* c = lat->ctx;
  HIPCHECK(hipSetDevice(c->device));
  const long long vp = pad_half(lat->Vh);
  if (!lat->clv64) {
    const size_t b64 = (size_t)CLV_KINDS * 2 * clover_rows(P64) * vp * 16;
    const size_t b32 = (size_t)CLV_KINDS * 2 * clover_rows(P32) * vp * 16;
    if (hipMalloc(&lat->clv64, b64) != hipSuccess || hipMalloc(&lat->clv32, b32) != hipSuccess) {
      (void)hipGetLastError();
      clover_free(lat);
      throw Error(DL_ENOMEM, "clover term: allocation of the site matrices failed");
    }
  }
  // sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu], gamma_mu = Gamma_{2^mu}
  std::complex<double> G[16][4][4];
  gamma_basis(G);
  double sg[6][4][4][2];
  int plane = 0;
  for (int m = 0; m < 4; ++m)
    for (int n = m + 1; n < 4; ++n, ++plane)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          std::complex<double> v = 0.0;
          for (int k = 0; k < 4; ++k) v += G[1 << m][a][k] * G[1 << n][k][b] - G[1 << n][a][k] * G[1 << m][k][b];
          v *= std::complex<double>(0.0, 0.5);
          sg[plane][a][b][0] = v.real();
          sg[plane][a][b][1] = v.imag();
        }
  stream_enter(c);
  launch_clover_build(lat->gauge[P64], lat->dims, vp, lat->kappa, lat->mu, lat->csw, sg, lat->clv64, lat->clv32,
                      c->st);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(c->st));
  stream_exit(c);
}

static void gauge_upload(dl_lattice* lat, const double* links, int on_device) {
  dl_ctx* c = lat->ctx;
  lat->two_row = 0;   // nine-entry reads unless this upload's check passes
  stream_enter(c);
  const size_t bytes = (size_t)lat->V * 4 * 9 * 16;
  DevBuf stage;
  const double* src = links;
  if (!on_device) {
    stage = DevBuf(c, bytes);
    HIPCHECK(hipMemcpyAsync(stage.p, links, bytes, hipMemcpyHostToDevice, c->st));
    src = stage.as<double>();
  }
  DevBuf flag(c, sizeof(int));
  HIPCHECK(hipMemsetAsync(flag.p, 0, sizeof(int), c->st));
  launch_pack_gauge(src, lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3], lat->gauge[0], lat->gauge[1],
                    lat->gauge[2], lat->gauge[3], flag.as<int>(), c->st);
  HIPCHECK(hipGetLastError());
  int not_su3 = TWO_ROW_16 | TWO_ROW_32;
  HIPCHECK(hipMemcpyAsync(&not_su3, flag.p, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  stream_exit(c);
  lat->two_row = (TWO_ROW_16 | TWO_ROW_32) & ~not_su3;
  lat->gauge_set = true;
  clover_rebuild(lat);
}

int dl_gauge_set(dl_lattice* lat, const double* links, int on_device) {
  return guarded([&] {
    require(lat && links, "dl_gauge_set: NULL argument");
    gauge_upload(lat, links, on_device);
    return 0;
  });
}

int dl_gauge_random_host(const int dims[4], uint64_t seed, double eps, double* links) {
  return guarded([&] {
    require(dims && links, "dl_gauge_random_host: NULL argument");
    for (int k = 0; k < 4; ++k) require(dims[k] >= 1, "dl_gauge_random_host: extents must be >= 1");
    require(std::isfinite(eps), "dl_gauge_random_host: eps must be finite");
    random_gauge_host(dims, seed, eps, links);
    return 0;
  });
}

int dl_gauge_random(dl_lattice* lat, uint64_t seed, double eps) {
  return guarded([&] {
    require(lat != nullptr, "dl_gauge_random: NULL lattice");
    require(std::isfinite(eps), "dl_gauge_random: eps must be finite");
    std::vector<double> links((size_t)lat->V * 4 * 18);
    random_gauge_host(lat->dims, seed, eps, links.data());
    gauge_upload(lat, links.data(), 0);
    return 0;
  });
}

int dl_set_params(dl_lattice* lat, double kappa, double mu) {
  return guarded([&] {
    require(lat != nullptr, "dl_set_params: NULL lattice");
    require(std::isfinite(kappa) && kappa > 0, "dl_set_params: kappa must be > 0");
    require(std::isfinite(mu), "dl_set_params: mu must be finite");
    lat->kappa = kappa;
    lat->mu = mu;
    lat->params_set = true;
    clover_rebuild(lat);
    return 0;
  });
}

int dl_set_clover(dl_lattice* lat, double csw) {
  return guarded([&] {
    require(lat != nullptr, "dl_set_clover: NULL lattice");
    require(std::isfinite(csw), "dl_set_clover: c_sw must be finite");
    lat->csw = csw;
    if (csw == 0.0) {
      (void)hipSetDevice(lat->ctx->device);
      (void)hipStreamSynchronize(lat->ctx->st);
      clover_free(lat);
    } else {
      clover_rebuild(lat);
    }
    return 0;
  });
}

int dl_accum_create(dl_lattice* lat, int ops, dl_accum** out) {
  return guarded([&] {
    require(lat && out, "dl_accum_create: NULL argument");
    const int base = ops & ~DL_OPS_HPE(7), hpe = DL_OPS_HPE_ORDER(ops);
    require(base == DL_OPS_LOCAL || base == (DL_OPS_LOCAL | DL_OPS_DERIV),
            "dl_accum_create: ops must be LOCAL or LOCAL|DERIV, optionally with DL_OPS_HPE(n)");
    require(hpe <= 4, "dl_accum_create: HPE order must be 1..4");
    if (hpe)
      for (int d = 0; d < 4; ++d)
        require(lat->dims[d] >= 4, "dl_accum_create: the hopping parameter expansion needs every extent >= 4");
    HIPCHECK(hipSetDevice(lat->ctx->device));
    auto* a = new dl_accum();
    a->lat = lat;
    a->ops = ops;
    a->nq = acc_components(ops);
    const size_t bytes = sizeof(double) * (size_t)a->nq * 2 * pad_half(lat->Vh);
    for (int s = 0; s < 3; ++s) {
      if (hipMalloc((void**)&a->acc[s], bytes) != hipSuccess) {
        (void)hipGetLastError();
        for (int k = 0; k < s; ++k) (void)hipFree(a->acc[k]);
        delete a;
        throw Error(DL_ENOMEM, "dl_accum_create: allocation failed");
      }
      HIPCHECK(hipMemset(a->acc[s], 0, bytes));
    }
    *out = a;
    return 0;
  });
}

int dl_accum_reset(dl_accum* a) {
  return guarded([&] {
    require(a != nullptr, "dl_accum_reset: NULL");
    dl_ctx* c = a->lat->ctx;
    stream_enter(c);
    const size_t bytes = sizeof(double) * (size_t)a->nq * 2 * pad_half(a->lat->Vh);
    for (int s = 0; s < 3; ++s) {
      HIPCHECK(hipMemsetAsync(a->acc[s], 0, bytes, c->st));
      a->count[s] = 0;
    }
    stream_exit(c);
    return 0;
  });
}

int dl_accum_destroy(dl_accum* a) {
  return guarded([&] {
    if (!a) return 0;
    (void)hipStreamSynchronize(a->lat->ctx->st);
    for (int s = 0; s < 3; ++s)
      if (a->acc[s]) (void)hipFree(a->acc[s]);
    delete a;
    return 0;
  });
}

int dl_accum_counts(const dl_accum* a, int64_t counts[3]) {
  return guarded([&] {
    require(a && counts, "dl_accum_counts: NULL argument");
    for (int s = 0; s < 3; ++s) counts[s] = a->count[s];
    return 0;
  });
}

static std::vector<std::array<int, 3>> momentum_list(const int dims[4], int p2max) {
  std::vector<std::array<int, 3>> v;
  int lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = -(dims[k] / 2) + 1;
    hi[k] = dims[k] / 2;
  }
  for (int a = lo[0]; a <= hi[0]; ++a)
    for (int b = lo[1]; b <= hi[1]; ++b)
      for (int c = lo[2]; c <= hi[2]; ++c)
        if (a * a + b * b + c * c <= p2max) v.push_back({a, b, c});
  std::sort(v.begin(), v.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
    const int nx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2], ny = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    if (nx != ny) return nx < ny;
    return x < y;
  });
  return v;
}

int dl_momenta(const int dims[4], int p2max, int* n_xyz, int cap, int* np_out) {
  return guarded([&] {
    require(dims && np_out, "dl_momenta: NULL argument");
    require(p2max >= 0, "dl_momenta: p2max must be >= 0");
    auto v = momentum_list(dims, p2max);
    *np_out = (int)v.size();
    if (n_xyz)
      for (int i = 0; i < (int)v.size() && i < cap; ++i)
        for (int k = 0; k < 3; ++k) n_xyz[3 * i + k] = v[i][k];
    return 0;
  });
}

int dl_solve_batch(dl_ctx* ctx, const dl_job* jobs, int njobs, dl_src_stats* stats) {
  return guarded([&] {
    require(ctx != nullptr, "dl_solve_batch: NULL context");
    require(njobs >= 0 && (njobs == 0 || jobs), "dl_solve_batch: bad job array");
    std::vector<dl_job> J(jobs, jobs + njobs);
    std::vector<long long> first_stat(njobs + 1, 0);
    for (int j = 0; j < njobs; ++j) {
      const dl_job& q = J[j];
      require(q.lat != nullptr, "dl_solve_batch: job without lattice");
      require(q.lat->ctx == ctx, "dl_solve_batch: lattice of another context");
      require(q.lat->gauge_set, "dl_solve_batch: gauge field not set");
      require(q.lat->params_set, "dl_solve_batch: kappa / mu not set");
      require(q.nsrc >= 0, "dl_solve_batch: nsrc < 0");
      require(q.maxiter > 0, "dl_solve_batch: maxiter must be > 0");
      require(std::isfinite(q.tol) && q.tol > 0, "dl_solve_batch: tol must be > 0");
      require(q.noise == DL_NOISE_Z2 || q.noise == DL_NOISE_Z4 || q.noise == DL_NOISE_USER,
              "dl_solve_batch: unknown noise");
      require(q.noise != DL_NOISE_USER || q.src_in, "dl_solve_batch: USER noise needs src_in");
      require(q.first_src >= 0, "dl_solve_batch: first_src < 0");
      (void)tier_prec(q.tier);
      require(q.rhs_block >= 0, "dl_solve_batch: rhs_block < 0");
      require(q.tdil >= 0 && q.tdil <= q.lat->dims[3], "dl_solve_batch: tdil must be 0..T");
      if (q.accum) {
        require(q.accum->lat == q.lat, "dl_solve_batch: accumulator of another lattice");
        require(q.accum_set >= 0 && q.accum_set < 3, "dl_solve_batch: bad accum_set");
        require(q.lat->csw == 0.0 || DL_OPS_HPE_ORDER(q.accum->ops) == 0,
                "dl_solve_batch: the hopping parameter expansion is not built for clover lattices");
      }
      first_stat[j + 1] = first_stat[j] + (long long)q.nsrc * std::max(q.tdil, 1);
    }
    int hpe_order = 0;
    for (const dl_job& q : J) {
      if (!q.accum || q.nsrc == 0) continue;
      const int o = DL_OPS_HPE_ORDER(q.accum->ops);
      if (!o) continue;
      require(hpe_order == 0 || hpe_order == o,
              "dl_solve_batch: jobs of one call must use one hopping parameter expansion order");
      hpe_order = o;
    }
    for (int j = 0; j < njobs; ++j) {
      const dl_job& q = J[j];
      if (q.guess_from == 0) continue;
      const int g = q.guess_from - 1;
      require(g >= 0 && g < njobs && g != j, "dl_solve_batch: guess_from out of range");
      const dl_job& h = J[g];
      require(q.tier == DL_TIER_HP_FP32, "dl_solve_batch: guess_from is for HP jobs");
      require(h.tier != DL_TIER_HP_FP32, "dl_solve_batch: guess_from must name a lower-tier job");
      require(h.lat == q.lat && h.noise == q.noise && h.seed == q.seed && h.first_src == q.first_src &&
                  h.nsrc == q.nsrc && h.src_in == q.src_in && std::max(h.tdil, 1) == std::max(q.tdil, 1),
              "dl_solve_batch: guess_from job must solve the same sources on the same lattice");
    }
    stream_enter(ctx);
    const bool all_ok = solve_jobs(ctx, J, stats);
    HIPCHECK(hipGetLastError());
    stream_exit(ctx);
    return all_ok ? 0 : DL_NOT_CONVERGED;
  });
}

// Projection, Gamma rebuild and prefactors of weighted combinations of the
// accumulator's three sets: output k (complex128 [2][nops][16][T][Np], device)
// is the loops of sum_s w[k][s] S_s.  Runs on the context stream.
// Exact part of the hopping parameter expansion per site, before the
// prefactor: half the sum over both flavours (mu_f = +mu, -mu, B = A(mu_f)^-1)
// of the colour-traced orders k < n of M^-1 = sum_k (kappa B H)^k B, with the
// insertion's Gamma.  Extents >= 4 leave, on the diagonal, B (k = 0) and the
// hops forth and back, kappa^2 B Q B with Q = sum_nu [(1 - g_nu) B (1 + g_nu) +
// (1 + g_nu) B (1 - g_nu)] (k = 2, used for n >= 3); odd k vanish there.  For
// the derivative insertions (orders k < min(n, 3)) only the single hop k = 1
// survives: its four terms combine to kappa B g_nu B (used for n >= 2).
// Colour traces of the retraced links give 3.  out [nops][16].
static std::vector<std::complex<double>> hpe_exact_table(double kappa, double mu, int n, int nops) {
  using C = std::complex<double>;
  C G[16][4][4];
  gamma_basis(G);
  std::vector<C> out((size_t)nops * 16, C(0, 0));
  const double g5[4] = {1, 1, -1, -1};
  auto trace_with = [&](int m, const C (&S)[4][4]) {
    C t(0, 0);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) t += G[m][a][b] * S[b][a];
    return t;
  };
  for (const double muf : {mu, -mu}) {
    C B[4];
    for (int s = 0; s < 4; ++s) B[s] = 1.0 / C(1.0, 2.0 * kappa * muf * g5[s]);
    // local: S = B + kappa^2 B Q B
    C S[4][4] = {};
    for (int a = 0; a < 4; ++a) S[a][a] = B[a];
    if (n >= 3) {
      C Q[4][4] = {};
      for (int nu = 0; nu < 4; ++nu) {
        const C (&g)[4][4] = G[1 << nu];
        for (const double sg : {1.0, -1.0}) {
          // (1 - sg g) B (1 + sg g)
          C L[4][4], R[4][4];
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
              L[a][b] = (a == b ? 1.0 : 0.0) - sg * g[a][b];
              R[a][b] = (a == b ? 1.0 : 0.0) + sg * g[a][b];
            }
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
              for (int c = 0; c < 4; ++c) Q[a][b] += L[a][c] * B[c] * R[c][b];
        }
      }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) S[a][b] += kappa * kappa * B[a] * Q[a][b] * B[b];
    }
    for (int m = 0; m < 16; ++m) out[m] += 1.5 * trace_with(m, S);
    if (nops > 1 && n >= 2) {
      for (int nu = 0; nu < 4; ++nu) {
        C D[4][4];
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) D[a][b] = kappa * B[a] * G[1 << nu][a][b] * B[b];
        for (int m = 0; m < 16; ++m) out[(size_t)(1 + nu) * 16 + m] += 1.5 * trace_with(m, D);
      }
    }
  }
  return out;
}

// Device buffers of one projection: carved from `scratch` (the no-allocation
// entry point) or taken from the context pool.
struct LoopsWork {
  dl_ctx* ctx;
  unsigned char* scratch;
  size_t cap, used = 0;
  std::vector<DevBuf> held;
  LoopsWork(dl_ctx* c, unsigned char* s, size_t cp) : ctx(c), scratch(s), cap(cp) {}
  void* get(size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);
    if (!scratch) {
      held.emplace_back(ctx, bytes);
      return held.back().p;
    }
    void* p = scratch + used;
    used += (bytes + 255) & ~(size_t)255;
    return p;
  }
};

static size_t round256(size_t b) { return (std::max<size_t>(b, 16) + 255) & ~(size_t)255; }

static int loops_device(dl_ctx* ctx, dl_accum* a, int p2max, const double (*w)[3], int nw, double* target,
                        unsigned char* scratch, size_t scratch_cap) {
  dl_lattice* L = a->lat;
  auto moms = momentum_list(L->dims, p2max);
  const int np = (int)moms.size();
  const int X = L->dims[0], Y = L->dims[1], Z = L->dims[2], T = L->dims[3];
  // tables of the separable projection: distinct kx, distinct (kx, ky)
  std::vector<int> kxs, pair_ix, pj(np);
  std::vector<std::array<int, 2>> pairs;
  for (int p = 0; p < np; ++p) {
    const int kx = moms[p][0], ky = moms[p][1];
    int ix = (int)(std::find(kxs.begin(), kxs.end(), kx) - kxs.begin());
    if (ix == (int)kxs.size()) kxs.push_back(kx);
    const std::array<int, 2> pr{kx, ky};
    int j = (int)(std::find(pairs.begin(), pairs.end(), pr) - pairs.begin());
    if (j == (int)pairs.size()) {
      pairs.push_back(pr);
      pair_ix.push_back(ix);
    }
    pj[p] = j;
  }
  const int nkx = (int)kxs.size(), nkxy = (int)pairs.size();
  // distinct kz values, and the z-sum's thread order (kz, then pair)
  std::vector<int> kzs, pk(np), order(np);
  for (int p = 0; p < np; ++p) {
    const int kz = moms[p][2];
    int k = (int)(std::find(kzs.begin(), kzs.end(), kz) - kzs.begin());
    if (k == (int)kzs.size()) kzs.push_back(kz);
    pk[p] = k;
    order[p] = p;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return pk[a] != pk[b] ? pk[a] < pk[b] : pj[a] < pj[b]; });
  const int nkz = (int)kzs.size();
  auto phase = [](double n, int x, int ext, double* out) {
    const double ang = -2.0 * M_PI * n * x / ext;
    out[0] = std::cos(ang);
    out[1] = std::sin(ang);
  };
  std::vector<double> tabs;   // roots x | roots y | pz | shift, complex
  const size_t o_px = 0, o_py = o_px + 2ull * X, o_pz = o_py + 2ull * Y,
               o_sh = o_pz + 2ull * nkz * Z, n_tab = o_sh + 6ull * np;
  tabs.resize(std::max<size_t>(n_tab, 2));
  for (int x = 0; x < X; ++x) phase(1, x, X, &tabs[o_px + 2 * (size_t)x]);
  for (int y = 0; y < Y; ++y) phase(1, y, Y, &tabs[o_py + 2 * (size_t)y]);
  std::vector<int> kx_mod(nkx), ky_mod(nkxy);
  for (int k = 0; k < nkx; ++k) kx_mod[k] = ((kxs[k] % X) + X) % X;
  for (int k = 0; k < nkxy; ++k) ky_mod[k] = ((pairs[k][1] % Y) + Y) % Y;
  const int ext[3] = {X, Y, Z};
  for (int k = 0; k < nkz; ++k)
    for (int z = 0; z < Z; ++z) phase(kzs[k], z, Z, &tabs[o_pz + 2 * ((size_t)k * Z + z)]);
  for (int p = 0; p < np; ++p) {
    for (int nu = 0; nu < 3; ++nu) {
      double* f = &tabs[o_sh + 2 * ((size_t)p * 3 + nu)];
      phase(moms[p][nu], 1, ext[nu], f);
      f[0] += 1.0;
    }
  }
  std::vector<int> itab(pair_ix);
  itab.insert(itab.end(), pj.begin(), pj.end());
  itab.insert(itab.end(), pk.begin(), pk.end());
  itab.insert(itab.end(), order.begin(), order.end());
  itab.insert(itab.end(), kx_mod.begin(), kx_mod.end());
  itab.insert(itab.end(), ky_mod.begin(), ky_mod.end());
  const int nops = (a->ops & DL_OPS_DERIV) ? 5 : 1;
  const int hpe = DL_OPS_HPE_ORDER(a->ops);
  const size_t per_out = (size_t)2 * 2 * nops * 16 * T * np;   // doubles
  const size_t tab_bytes = tabs.size() * sizeof(double), itab_bytes = std::max<size_t>(itab.size(), 1) * sizeof(int);
  const size_t pbytes = std::max<size_t>(sizeof(double) * 2 * (size_t)a->nq * T * np, 16);
  const size_t r2_bytes = sizeof(double) * 2 * (size_t)a->nq * T * Z * nkxy;
  const size_t ex_bytes = hpe ? sizeof(double) * 2 * (size_t)nw * nops * 16 : 0;
  if (scratch) {
    const size_t need = round256(tab_bytes) + round256(itab_bytes) + round256(pbytes) + round256(r2_bytes) +
                        (hpe ? round256(ex_bytes) : 0);
    if (need > scratch_cap)
      throw Error(DL_EINVAL, "dl_loops_noalloc: this projection needs " + std::to_string(need) +
                                 " bytes of device scratch, the limit is " + std::to_string(scratch_cap));
  }
  LoopsWork wk(ctx, scratch, scratch_cap);
  double* dtab = (double*)wk.get(tab_bytes);
  int* ditab = (int*)wk.get(itab_bytes);
  HIPCHECK(hipMemcpyAsync(dtab, tabs.data(), tab_bytes, hipMemcpyHostToDevice, ctx->st));
  if (!itab.empty())
    HIPCHECK(hipMemcpyAsync(ditab, itab.data(), itab.size() * sizeof(int), hipMemcpyHostToDevice, ctx->st));
  ProjTables tb{};
  tb.np = np; tb.nkx = nkx; tb.nkxy = nkxy;
  const double* dt = dtab;
  tb.roots_x = dt + o_px; tb.roots_y = dt + o_py; tb.pz = dt + o_pz; tb.shift = dt + o_sh;
  tb.pair_ix = ditab; tb.pj = ditab + nkxy;
  tb.pk = tb.pj + np; tb.order = tb.pk + np;
  tb.kx_mod = tb.order + np; tb.ky_mod = tb.kx_mod + nkx;
  double* proj = (double*)wk.get(pbytes);
  double* r2 = (double*)wk.get(r2_bytes);
  // exact part of the hopping parameter expansion: per output, the spatial
  // volume (momentum 0) times the weighted source count of the sets used
  double* dex = nullptr;
  if (hpe) {
    const auto ex = hpe_exact_table(L->kappa, L->mu, hpe, nops);
    std::vector<double> h((size_t)nw * nops * 16 * 2);
    for (int k = 0; k < nw; ++k) {
      double wsum = 0.0;
      for (int s = 0; s < 3; ++s)
        if (w[k][s] != 0.0 && a->count[s] > 0) wsum += w[k][s] * (double)a->count[s];
      const double f = wsum * (double)X * Y * Z;
      for (int i = 0; i < nops * 16; ++i) {
        h[((size_t)k * nops * 16 + i) * 2] = f * ex[i].real();
        h[((size_t)k * nops * 16 + i) * 2 + 1] = f * ex[i].imag();
      }
    }
    dex = (double*)wk.get(ex_bytes);
    HIPCHECK(hipMemcpyAsync(dex, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ctx->st));
    HIPCHECK(hipStreamSynchronize(ctx->st));   // h ends with this scope
  }
  for (int k = 0; k < nw; ++k) {
    const double* sets[3];
    for (int s = 0; s < 3; ++s) sets[s] = (w[k][s] != 0.0 && a->count[s] > 0) ? a->acc[s] : nullptr;
    if (sets[0] || sets[1] || sets[2]) {
      // derivative rows (q >= 48) hold link-centred sums
      launch_project(sets, w[k], a->nq, 48, X, Y, Z, T, tb, r2, proj, ctx->st);
    } else {
      launch_fill_zero(proj, pbytes / sizeof(double), ctx->st);
    }
    const double* exk = hpe ? dex + (size_t)k * nops * 16 * 2 : nullptr;
    launch_loops_finalize(proj, nops, T, np, L->kappa, L->mu, exk, target + k * per_out, ctx->st);
  }
  HIPCHECK(hipGetLastError());
  return np;
}

static void loops_common(dl_ctx* ctx, dl_accum* a, int p2max, const double (*w)[3], int nw, double* out,
                         int out_on_device, int* np_out) {
  dl_lattice* L = a->lat;
  const int np = (int)momentum_list(L->dims, p2max).size();
  if (np_out) *np_out = np;
  const int nops = (a->ops & DL_OPS_DERIV) ? 5 : 1;
  const size_t obytes = sizeof(double) * 2 * 2 * nops * 16 * (size_t)L->dims[3] * np * nw;
  stream_enter(ctx);
  DevBuf dout;
  double* target = out;
  if (!out_on_device) {
    dout = DevBuf(ctx, std::max<size_t>(obytes, 16));
    target = dout.as<double>();
  }
  loops_device(ctx, a, p2max, w, nw, target, nullptr, 0);
  if (!out_on_device) {
    HIPCHECK(hipMemcpyAsync(out, target, obytes, hipMemcpyDeviceToHost, ctx->st));
    HIPCHECK(hipStreamSynchronize(ctx->st));
  }
  stream_exit(ctx);
}

// Checks of dl_loops / dl_loops_noalloc and the TSM weights of the three sets.
static void tsm_weights(dl_ctx* ctx, dl_accum* a, int p2max, const double* out, const char* fn, double w[3]) {
  const std::string f(fn);
  require(ctx && a && out, f + ": NULL argument");
  require(p2max >= 0, f + ": p2max must be >= 0");
  dl_lattice* L = a->lat;
  require(L->ctx == ctx, f + ": accumulator of another context");
  require(L->params_set, f + ": kappa / mu not set");
  require(a->count[DL_SET_LPC] == 0 || a->count[DL_SET_LPC] == a->count[DL_SET_HP],
          f + ": the LPC set must hold the same sources as the HP set");
  // with both LP and HP sources the estimate is the TSM one, which needs the
  // LP solves of the HP sources; S_LP / N_LP + S_HP / N_HP would count the loop twice
  require(a->count[DL_SET_LP] == 0 || a->count[DL_SET_HP] == 0 || a->count[DL_SET_LPC] == a->count[DL_SET_HP],
          f + ": LP and HP sets without the LPC set (the LP solves of the HP sources) form no estimator");
  // TSM combination L = S_LP / N_LP + (S_HP - S_LPC) / N_HP, taken on the
  // accumulators so one projection serves all three sets
  const double w_lp = a->count[DL_SET_LP] > 0 ? 1.0 / (double)a->count[DL_SET_LP] : 0.0;
  const double w_hp = a->count[DL_SET_HP] > 0 ? 1.0 / (double)a->count[DL_SET_HP] : 0.0;
  w[0] = w_lp;
  w[1] = w_hp;
  w[2] = -w_hp;
}

int dl_loops(dl_ctx* ctx, dl_accum* a, int p2max, double* out, int out_on_device, int* np_out) {
  return guarded([&] {
    double w[1][3];
    tsm_weights(ctx, a, p2max, out, "dl_loops", w[0]);
    loops_common(ctx, a, p2max, w, 1, out, out_on_device, np_out);
    return 0;
  });
}

int dl_loops_noalloc(dl_ctx* ctx, dl_accum* a, int p2max, double* out, int* np_out) {
  return guarded([&] {
    double w[1][3];
    tsm_weights(ctx, a, p2max, out, "dl_loops_noalloc", w[0]);
    require(ctx->scratch != nullptr, "dl_loops_noalloc: context has no scratch address");
    const int np = (int)momentum_list(a->lat->dims, p2max).size();
    if (np_out) *np_out = np;
    stream_enter(ctx);
    loops_device(ctx, a, p2max, w, 1, out, ctx->scratch, DL_LOOPS_NOALLOC_SCRATCH_BYTES);
    stream_exit(ctx);
    return 0;
  });
}

int dl_loops_sets(dl_ctx* ctx, dl_accum* a, int p2max, double* out, int out_on_device, int* np_out) {
  return guarded([&] {
    require(ctx && a && out, "dl_loops_sets: NULL argument");
    require(p2max >= 0, "dl_loops_sets: p2max must be >= 0");
    dl_lattice* L = a->lat;
    require(L->ctx == ctx, "dl_loops_sets: accumulator of another context");
    require(L->params_set, "dl_loops_sets: kappa / mu not set");
    const double w[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    loops_common(ctx, a, p2max, w, 3, out, out_on_device, np_out);
    return 0;
  });
}

int dl_set_option(dl_ctx* ctx, const char* name, double value) {
  return guarded([&] {
    require(ctx && name, "dl_set_option: NULL argument");
    const std::string n(name);
    if (n == "inflight_rhs") {
      require(value >= 1 && value < 1e9, "dl_set_option: inflight_rhs must be >= 1");
      ctx->inflight_rhs = (int)value;
    } else if (n == "inflight_mb") {
      require(value > 0, "dl_set_option: inflight_mb must be > 0");
      ctx->inflight_mb = value;
    } else if (n == "use_graph") {
      require(value == 0 || value == 1, "dl_set_option: use_graph must be 0 or 1");
      ctx->use_graph = value != 0;
    } else if (n == "contract_tblk") {
      require(value >= 1 && value <= 64, "dl_set_option: contract_tblk must be in 1..64");
      ctx->contract_tblk = (int)value;
    } else if (n == "block_hop") {
      require(value == 0 || value == 1, "dl_set_option: block_hop must be 0 or 1");
      ctx->block_hop = value != 0;
    } else if (n == "profile") {
      require(value == 0 || value == 1, "dl_set_option: profile must be 0 or 1");
      ctx->profile = value != 0;
    } else {
      throw Error(DL_EINVAL, "dl_set_option: unknown option '" + n + "'");
    }
    return 0;
  });
}

int dl_profile_read(dl_ctx* ctx, int tier, double out[4]) {
  return guarded([&] {
    require(ctx && out, "dl_profile_read: NULL argument");
    const int P = tier_prec(tier);
    for (int k = 0; k < 4; ++k) {
      out[k] = ctx->prof[P][k];
      ctx->prof[P][k] = 0;
    }
    return 0;
  });
}

int dl_autotune(dl_ctx* ctx, dl_lattice* lat, int tier, int nsrc, int* block_out, int* tblk_out) {
  return guarded([&] {
    require(ctx && lat && block_out, "dl_autotune: NULL argument");
    require(lat->ctx == ctx, "dl_autotune: lattice belongs to another context");
    require(nsrc >= 1, "dl_autotune: nsrc must be >= 1");
    const int P = tier_prec(tier);
    stream_enter(ctx);
    const TuneChoice tc = autotune_block(ctx, lat, P, nsrc);
    stream_exit(ctx);
    *block_out = tc.block;
    if (tblk_out) *tblk_out = tc.tblk;
    return 0;
  });
}

int dl_apply_op(dl_lattice* lat, int op, int tier, const double* in, double* out, int nrhs) {
  return guarded([&] {
    require(lat && in && out, "dl_apply_op: NULL argument");
    require(nrhs >= 1, "dl_apply_op: nrhs must be >= 1");
    require(lat->gauge_set, "dl_apply_op: gauge field not set");
    require(lat->params_set || op == DL_OP_HOP, "dl_apply_op: kappa / mu not set");
    require(op >= DL_OP_M && op <= DL_OP_HOP, "dl_apply_op: unknown operator");
    stream_enter(lat->ctx);
    apply_op(lat, op, tier, in, out, nrhs);
    HIPCHECK(hipGetLastError());
    stream_exit(lat->ctx);
    return 0;
  });
}

int dl_fill_noise(dl_lattice* lat, int noise, uint64_t seed, int64_t src, double* out) {
  return guarded([&] {
    require(lat && out, "dl_fill_noise: NULL argument");
    require(noise == DL_NOISE_Z2 || noise == DL_NOISE_Z4, "dl_fill_noise: noise must be Z2 or Z4");
    require(src >= 0, "dl_fill_noise: src < 0");
    dl_ctx* c = lat->ctx;
    stream_enter(c);
    std::vector<dl_job> J(1);
    std::memset(&J[0], 0, sizeof(dl_job));
    J[0].lat = lat;
    J[0].noise = noise;
    J[0].seed = seed;
    std::vector<SlotPlan> plan(1);
    plan[0] = SlotPlan{};
    plan[0].lat = lat;
    plan[0].job = 0;
    plan[0].nrhs = 1;
    plan[0].src0 = src;
    plan[0].sol_user = out;
    fill_noise_fields(c, plan, J);
    stream_exit(c);
    return 0;
  });
}

int dl_loops_backward(dl_ctx* ctx, const dl_job* job, int p2max, const double* grad_loops, double* grad_eta,
                      double* grad_mu) {
  return guarded([&] {
    require(ctx && job && grad_loops, "dl_loops_backward: NULL argument");
    require(!job->lat || job->lat->csw == 0.0, "dl_loops_backward: not built for clover lattices");
    require(!job->accum || DL_OPS_HPE_ORDER(job->accum->ops) == 0,
            "dl_loops_backward: loops with the hopping parameter expansion are not differentiated");
    require(job->tdil <= 1, "dl_loops_backward: time-diluted sources are not differentiated");
    require(job->accum || job->grad_ops == 0 || job->grad_ops == DL_OPS_LOCAL ||
                job->grad_ops == (DL_OPS_LOCAL | DL_OPS_DERIV),
            "dl_loops_backward: grad_ops must be 0, DL_OPS_LOCAL or DL_OPS_LOCAL | DL_OPS_DERIV");
    loops_backward(ctx, *job, p2max, grad_loops, grad_eta, grad_mu);
    return 0;
  });
}

}  // extern "C"
