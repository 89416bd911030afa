// Host runtime objects behind the C ABI.
#pragma once

#include <complex>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/discloop.h"
#include "kernels.h"

namespace dl {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what);
#define HIPCHECK(x) ::dl::hip_check((x), #x)

// Device memory with a size-keyed cache owned by the context.
struct Pool {
  std::multimap<size_t, void*> free_;
  size_t cached_bytes = 0;
  void* get(size_t bytes);
  void put(void* p, size_t bytes);
  void clear();
};

}  // namespace dl

struct dl_ctx {
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t st = nullptr;      // internal stream all work runs on
  hipEvent_t ev = nullptr;
  unsigned char* scratch = nullptr;   // this GPU's copy of dl_loops_noalloc's scratch array
  dl::Pool pool;
  std::map<std::string, int> tune;   // autotuned rhs block / tile-order block per (dims, precision, size)
  std::string tune_path;
  bool tune_loaded = false;
  int last_tune_block = 0;
  // options
  int inflight_rhs = 1024;
  double inflight_mb = 32768.0;
  bool use_graph = true;
  bool block_hop = false;        // LDS-staged hop for 16-bit storage where the lattice shape allows
  int contract_tblk = 8;         // time slices per block of the derivative contraction's tile order
  bool profile = false;
  // hopping-kernel profile per storage precision: launches, ms, bytes, rhs
  double prof[4][4] = {};
};

struct dl_lattice {
  dl_ctx* ctx = nullptr;
  int dims[4] = {0, 0, 0, 0};
  int bc = -1;
  long long V = 0, Vh = 0;
  void* gauge[4] = {nullptr, nullptr, nullptr, nullptr};
  bool gauge_set = false;
  // TWO_ROW_* bits (checked at upload): the hops of those storage classes
  // rebuild row 2 of the links from rows 0 and 1
  int two_row = 0;
  double kappa = 0, mu = 0;
  bool params_set = false;
  // clover term (c_sw = 0: none); its site matrices follow the gauge field,
  // kappa and mu (rebuilt by dl_gauge_set, dl_set_params and dl_set_clover)
  double csw = 0;
  void* clv64 = nullptr;
  void* clv32 = nullptr;
};

struct dl_accum {
  dl_lattice* lat = nullptr;
  int ops = 1;
  int nq = 48;
  double* acc[3] = {nullptr, nullptr, nullptr};
  int64_t count[3] = {0, 0, 0};
};

namespace dl {

// RAII device buffer from the context pool
struct DevBuf {
  dl_ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(dl_ctx* c, size_t b) : ctx(c), bytes(b) { p = b ? c->pool.get(b) : nullptr; }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    ctx = o.ctx; p = o.p; bytes = o.bytes;
    o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p && ctx) ctx->pool.put(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return (T*)p; }
};

// Entry and exit of every API call: order the internal stream after the
// caller's stream, and the caller's stream after the internal one.
void stream_enter(dl_ctx* c);
void stream_exit(dl_ctx* c);

int tier_prec(int tier);

// One-source-block slot of a batch before device upload.
struct SlotPlan {
  dl_lattice* lat;
  int job;                 // index into the job array
  int job_first;           // index of rhs 0 within the job
  int nrhs;
  long long src0;
  const double* src_user;
  double* sol_user;
  double* acc;
  int tblk;                // tile-order time block (0: default)
  // initial guesses: per job rhs a [chunk][Vp] half field (odd sites) in the
  // storage precision of the job that produced it
  void* gsave;             // store this slot's odd solutions here (rhs 0), or null
  const void* gload;       // start this slot's CG from here (rhs 0), or null
  int gprec;               // precision of gload
  int tdil = 0;            // time dilution of the job (components per noise vector)
  int tclen = 0;           // noise vectors of the job
};

struct SolveReport {
  std::vector<int> iters, status, ru;
  std::vector<double> rel, truer;
};

// Solve the slots of one precision class; returns per-rhs results in slot order.
void run_batch(dl_ctx* ctx, int tier, const std::vector<SlotPlan>& plan, const std::vector<dl_job>& jobs,
               SolveReport& rep);

// Single-operator application for verification (dl_apply_op).
void apply_op(dl_lattice* lat, int op, int tier, const double* in, double* out, int nrhs);

void set_gamma_table(const int col[16][4], const double ph[16][4][2]);
// Dense Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3 of the chiral basis (gamma_nu = Gamma_{2^nu}).
void gamma_basis(std::complex<double> (&G)[16][4][4]);
void init_gamma_table();

// Slot shape of the hopping kernel: right-hand sides per slot and the
// time-block depth of the tile order.
struct TuneChoice { int block, tblk; };
TuneChoice autotune_block(dl_ctx* ctx, dl_lattice* lat, int prec, int nsrc_hint);

// Plan validated jobs into slots (autotuned block sizes) and memory-bounded
// batches per precision class, run them, fill stats (job order) and the
// accumulator counts.  Returns whether every source converged.
bool solve_jobs(dl_ctx* ctx, const std::vector<dl_job>& J, dl_src_stats* stats);

// Write the Z2 / Z4 sources of the plan's slots to their sol_user arrays.
void fill_noise_fields(dl_ctx* ctx, const std::vector<SlotPlan>& plan, const std::vector<dl_job>& jobs);

// Synthetic links U = exp(i eps H) (gauge.hip) into host memory, complex128
// [t][z][y][x][mu][3][3]; multi-threaded.
void random_gauge_host(const int dims[4], uint64_t seed, double eps, double* links);

// Adjoint-solve gradients of the loops (dl_loops_backward).
void loops_backward(dl_ctx* ctx, const dl_job& job, int p2max, const double* grad_loops, double* grad_eta,
                    double* grad_mu);

}  // namespace dl
