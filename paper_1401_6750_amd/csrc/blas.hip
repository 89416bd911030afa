// CG scalar finalisation, BLAS-1 kernels, noise generation and layout packing.
//
// Reductions are deterministic: every unit (64 sites of one right-hand side)
// writes one FP64 partial sum (fixed butterfly), and the finalise kernel sums
// the partials of a right-hand side over tiles in a fixed order.  The tiling
// does not depend on how many right-hand sides are interleaved, so a source
// gives bit-identical iterates alone or in any batch.
#include <stdexcept>

#include "kernels.h"

namespace dl {

static inline int grid_for(int units, int wpb) { return (units + wpb - 1) / wpb; }

// ---------------------------------------------------------------------------
// finalisation of reductions: one wavefront per global right-hand side
// ---------------------------------------------------------------------------
__device__ inline int find_slot_by_rhs(const SlotDesc* slots, int nslots, int g) {
  int lo = 0, hi = nslots - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (slots[mid].rhs_begin <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(64) void k_finalize(int kind, const SlotDesc* slots, int nslots,
                                                 int nrhs_total, const double* partial, CgScalars cs) {
  const int g = blockIdx.x;
  if (g >= nrhs_total) return;
  const int lane = threadIdx.x;
  if (kind != FK_INIT && kind != FK_STORE && !cs.active[g]) {
    if (kind == FK_ALPHA && threadIdx.x == 0) cs.upd[g] = 0;   // no step this iteration
    return;
  }
  const SlotDesc& sd = slots[find_slot_by_rhs(slots, nslots, g)];
  const int r = g - sd.rhs_begin;
  double v = 0.0;
  for (int t = lane; t < sd.ntile; t += 64) v += partial[sd.ubeg[UK_RHS] + t * sd.nrhs + r];
  v = wave_sum(v);
  if (lane != 0) return;
  const bool finite = isfinite(v);
  switch (kind) {
    case FK_INIT:
      cs.cc[g] = v;
      cs.rr[g] = v;
      cs.iters[g] = 0;
      cs.upd[g] = 0;
      if (!finite) { cs.active[g] = 0; cs.status[g] = 2; }
      else if (v == 0.0) { cs.active[g] = 0; cs.status[g] = 0; }
      else { cs.active[g] = 1; cs.status[g] = 1; }
      break;
    case FK_ALPHA:
      if (!(finite && v > 0.0)) {
        cs.active[g] = 0; cs.status[g] = 2; cs.alpha[g] = 0.0; cs.upd[g] = 0;
      } else {
        cs.alpha[g] = cs.rr[g] / v;
        cs.upd[g] = 1;
      }
      break;
    case FK_BETA: {
      const int it = cs.iters[g] + 1;
      cs.iters[g] = it;
      if (!finite) { cs.active[g] = 0; cs.status[g] = 2; break; }
      if (v <= cs.tol2[g] * cs.cc[g]) {
        cs.active[g] = 0; cs.status[g] = 0; cs.rr[g] = v;
        break;
      }
      cs.beta[g] = v / cs.rr[g];
      cs.rr[g] = v;
      if (it >= cs.maxiter[g]) { cs.active[g] = 0; cs.status[g] = 1; }
      break;
    }
    case FK_STORE:
      if (!cs.active || cs.active[g]) cs.out[g] = v;   // the gate: rhs whose partials were written
      break;
  }
}

void launch_finalize(int kind, const SlotDesc* slots, int nslots, int nrhs_total, const double* partial,
                     const CgScalars& cs, hipStream_t st) {
  if (nrhs_total == 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(nrhs_total), dim3(64), 0, st, kind, slots, nslots, nrhs_total,
                     partial, cs);
}

// ---------------------------------------------------------------------------
// reliable-update decisions of the high-precision tier, one thread per rhs
// (the same rules the host applies between plain launches)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hp_decide(int nrhs, CgScalars cs, HpState hp) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrhs) return;
  int h = 0;
  const double rr = cs.rr[g];
  if (cs.active[g]) {
    // no update within 100x (in <r, r>) of the target: the verification's own
    // FP64 residual follows shortly
    if (rr < hp.delta2 * hp.rr_ru[g] && rr > 1e2 * (cs.tol2[g] * cs.cc[g])) h = 1;
  } else if (cs.status[g] == 0 && !hp.verified[g] && cs.cc[g] > 0) {
    h = 2;
  }
  hp.hflag[g] = h;
  hp.flag[g] = h != 0;
  hp.react[g] = 0;
}

__global__ __launch_bounds__(256) void k_hp_post(int nrhs, CgScalars cs, HpState hp) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrhs) return;
  const int h = hp.hflag[g];
  if (!h) return;
  hp.ru_count[g] += 1;
  const double rr = cs.rr[g];
  hp.rr_ru[g] = rr;
  if (h == 2) {
    if (rr <= cs.tol2[g] * cs.cc[g]) {
      hp.verified[g] = 1;
    } else if (cs.iters[g] < cs.maxiter[g]) {
      hp.react[g] = 1;
      cs.active[g] = 1;
      cs.status[g] = 1;
    } else {
      hp.verified[g] = 1;
      cs.status[g] = 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_hp_pending(int nrhs, CgScalars cs, HpState hp) {
  __shared__ int cnt[256];
  int n = 0;
  for (int g = threadIdx.x; g < nrhs; g += blockDim.x)
    n += cs.active[g] || (cs.status[g] == 0 && !hp.verified[g] && cs.cc[g] > 0);
  cnt[threadIdx.x] = n;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) hp.pending[0] = cnt[0];
}

void launch_hp_decide(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_hp_decide, dim3((nrhs + 255) / 256), dim3(256), 0, st, nrhs, cs, hp);
}

void launch_hp_post(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_hp_post, dim3((nrhs + 255) / 256), dim3(256), 0, st, nrhs, cs, hp);
}

void launch_hp_pending(int nrhs, const CgScalars& cs, const HpState& hp, hipStream_t st) {
  hipLaunchKernelGGL(k_hp_pending, dim3(1), dim3(256), 0, st, nrhs, cs, hp);
}

// ---------------------------------------------------------------------------
// unit decoding shared by the BLAS kernels (UK_RHS units)
// ---------------------------------------------------------------------------
struct UnitRhs {
  int si, r, g, s;
  bool valid;
  long long off;
};

__device__ inline bool decode_rhs_unit(const SlotDesc* slots, int nslots, int total_units, UnitRhs& w) {
  const int u = wave_unit();
  if (u >= total_units) return false;
  w.si = find_slot(slots, nslots, UK_RHS, u);
  const SlotDesc& sd = slots[w.si];
  const int ul = u - sd.ubeg[UK_RHS];
  const int tile = ul / sd.nrhs;
  w.r = ul - tile * sd.nrhs;
  w.g = sd.rhs_begin + w.r;
  w.s = tile * TILE + (threadIdx.x & 63);
  w.valid = w.s < sd.Vh;
  w.off = sd.fo + (long long)w.r * sd.Vp;
  return true;
}

template <class S>
__global__ __launch_bounds__(256) void k_update_p(const SlotDesc* slots, int nslots, int total_units, void* p,
                                                  const void* r, void* x, const double* alpha,
                                                  const double* beta, const int* active, const int* upd) {
  using R = typename Traits<S>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  const bool ux = upd[w.g] != 0, up = active[w.g] != 0;
  if (!(ux || up) || !w.valid) return;
  const long vp = slots[w.si].Vp;
  cx<R> pv[12];
  load_spinor<S>(field_at<S>(p, w.off), vp, w.s, pv);
  if (ux) {
    const R al = (R)alpha[w.g];
    cx<R> xv[12];
    load_spinor<S>(field_at<S>(x, w.off), vp, w.s, xv);
#pragma unroll
    for (int k = 0; k < 12; ++k) xv[k] = xv[k] + al * pv[k];
    store_spinor<S>(field_at<S>(x, w.off), vp, w.s, xv);
  }
  if (up) {
    const R b = (R)beta[w.g];
    cx<R> rv[12];
    load_spinor<S>(field_at<S>(r, w.off), vp, w.s, rv);
#pragma unroll
    for (int k = 0; k < 12; ++k) pv[k] = rv[k] + b * pv[k];
    store_spinor<S>(field_at<S>(p, w.off), vp, w.s, pv);
  }
}

template <class S>
__global__ __launch_bounds__(256) void k_zero(const SlotDesc* slots, int nslots, int total_units, void* f,
                                              const int* active) {
  using R = typename Traits<S>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  if ((active && !active[w.g]) || !w.valid) return;
  cx<R> z[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) z[k] = mk<R>(0, 0);
  store_spinor<S>(field_at<S>(f, w.off), slots[w.si].Vp, w.s, z);
}

#define DISPATCH_PREC(prec, KERNEL, ...)                                                     \
  switch (prec) {                                                                            \
    case P64: hipLaunchKernelGGL((KERNEL<double>), __VA_ARGS__); break;                      \
    case P32: hipLaunchKernelGGL((KERNEL<float>), __VA_ARGS__); break;                       \
    case PB16: hipLaunchKernelGGL((KERNEL<bf16s>), __VA_ARGS__); break;                      \
    case PH16: hipLaunchKernelGGL((KERNEL<f16s>), __VA_ARGS__); break;                       \
    default: throw std::runtime_error("bad precision");                                     \
  }

void launch_update_p(int prec, const SlotDesc* slots, int nslots, int total_units, void* p, const void* r,
                     void* x, const double* alpha, const double* beta, const int* active, const int* upd,
                     hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_update_p, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots,
                total_units, p, r, x, alpha, beta, active, upd);
}

void launch_zero(int prec, const SlotDesc* slots, int nslots, int total_units, void* f, const int* active,
                 hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_zero, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots, total_units,
                f, active);
}

// ---------------------------------------------------------------------------
// volume sources
// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: output i
// of the stream seeded with `seed` is mix(seed + (i + 1) * golden).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class S>
__global__ __launch_bounds__(256) void k_sources(const SlotDesc* slots, int nslots, int total_units, int parity,
                                                 void* eta) {
  using R = typename Traits<S>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  if (!w.valid) return;
  const SlotDesc& sd = slots[w.si];
  const Coords c = eo_coords(sd, w.s, parity);
  const long long lex = c.x + (long long)sd.X * (c.y + (long long)sd.Y * (c.z + (long long)sd.Z * c.t));
  const long long V = 2ll * sd.Vh;
  cx<R> v[12];
  if (sd.noise == 2 && !sd.src_user) {  // no caller field for this slot: zeros
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = mk<R>(0, 0);
  } else if (sd.noise == 2) {          // caller sources, complex128 [rhs][V][12]
    const double2* src = (const double2*)sd.src_user + ((long long)src_vector(sd, w.r) * V + lex) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 q = src[k];
      v[k] = mk<R>((R)q.x, (R)q.y);
    }
  } else {
    const uint64_t base = ((uint64_t)(sd.src0 + src_vector(sd, w.r)) * (uint64_t)V + (uint64_t)lex) * 12ull;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const uint64_t b = splitmix64_at(sd.seed, base + k);
      if (sd.noise == 0) {
        v[k] = mk<R>((b & 1ull) ? (R)-1 : (R)1, (R)0);
      } else {
        const int q = (int)(b & 3ull);          // 0 -> 1, 1 -> i, 2 -> -1, 3 -> -i
        const R re = q == 0 ? (R)1 : (q == 2 ? (R)-1 : (R)0);
        const R im = q == 1 ? (R)1 : (q == 3 ? (R)-1 : (R)0);
        v[k] = mk<R>(re, im);
      }
    }
  }
  if (sd.tdil > 1 && c.t % sd.tdil != tdil_comp(sd, w.r)) {   // time dilution: other component's slice
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = mk<R>(0, 0);
  }
  store_spinor<S>(field_at<S>(eta, w.off), sd.Vp, w.s, v);
}

void launch_sources(int prec, const SlotDesc* slots, int nslots, int total_units, int parity, void* eta,
                    hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_sources, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots, total_units,
                parity, eta);
}

template <class S>
__global__ __launch_bounds__(256) void k_unpack(const SlotDesc* slots, int nslots, int total_units, int parity,
                                                const void* f) {
  using R = typename Traits<S>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  if (!w.valid) return;
  const SlotDesc& sd = slots[w.si];
  if (!sd.sol_user) return;
  const Coords c = eo_coords(sd, w.s, parity);
  const long long lex = c.x + (long long)sd.X * (c.y + (long long)sd.Y * (c.z + (long long)sd.Z * c.t));
  const long long V = 2ll * sd.Vh;
  cx<R> v[12];
  load_spinor<S>(field_at<S>(f, w.off), sd.Vp, w.s, v);
  double2* dst = (double2*)sd.sol_user + ((long long)w.r * V + lex) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2((double)v[k].re, (double)v[k].im);
}

void launch_unpack(int prec, const SlotDesc* slots, int nslots, int total_units, int parity, const void* f,
                   hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_unpack, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots, total_units,
                parity, f);
}

// ---------------------------------------------------------------------------
// initial guesses kept between the solves of one call
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_guess_store(const SlotDesc* slots, int nslots, int total_units,
                                                     const void* f) {
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  const SlotDesc& sd = slots[w.si];
  if (!sd.gsave || !w.valid) return;
  constexpr int NC = Traits<S>::NC;
  const uint4* src = (const uint4*)field_at<S>(f, w.off);
  uint4* dst = (uint4*)sd.gsave + (long long)w.r * NC * sd.Vp;
#pragma unroll
  for (int k = 0; k < NC; ++k) dst[(long long)k * sd.Vp + w.s] = src[(long long)k * sd.Vp + w.s];
}

template <class SO, class SI>
__device__ inline void guess_load_one(const SlotDesc& sd, const UnitRhs& w, void* f) {
  using RI = typename Traits<SI>::R;
  using RO = typename Traits<SO>::R;
  cx<RI> a[12];
  load_spinor<SI>((const char*)sd.gload + (long long)w.r * Traits<SI>::NC * sd.Vp * 16, sd.Vp, w.s, a);
  cx<RO> b[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = mk<RO>((RO)a[k].re, (RO)a[k].im);
  store_spinor<SO>(field_at<SO>(f, w.off), sd.Vp, w.s, b);
}

template <class SO>
__global__ __launch_bounds__(256) void k_guess_load(const SlotDesc* slots, int nslots, int total_units, void* f) {
  using RO = typename Traits<SO>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  const SlotDesc& sd = slots[w.si];
  if (!w.valid) return;
  switch (sd.gload ? sd.gprec : -1) {
    case P64: guess_load_one<SO, double>(sd, w, f); break;
    case P32: guess_load_one<SO, float>(sd, w, f); break;
    case PB16: guess_load_one<SO, bf16s>(sd, w, f); break;
    case PH16: guess_load_one<SO, f16s>(sd, w, f); break;
    default: {
      cx<RO> z[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) z[k] = mk<RO>(0, 0);
      store_spinor<SO>(field_at<SO>(f, w.off), sd.Vp, w.s, z);
    }
  }
}

void launch_guess_store(int prec, const SlotDesc* slots, int nslots, int total_units, const void* f,
                        hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_guess_store, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots, total_units,
                f);
}

void launch_guess_load(int prec, const SlotDesc* slots, int nslots, int total_units, void* f, hipStream_t st) {
  if (!total_units) return;
  DISPATCH_PREC(prec, k_guess_load, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots, total_units,
                f);
}

// ---------------------------------------------------------------------------
// precision conversion and reliable-update helpers
// ---------------------------------------------------------------------------
template <class SI, class SO>
__global__ __launch_bounds__(256) void k_convert(const SlotDesc* slots, int nslots, int total_units,
                                                 const void* in, void* out, int add, const int* active) {
  using RI = typename Traits<SI>::R;
  using RO = typename Traits<SO>::R;
  UnitRhs w;
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  if ((active && !active[w.g]) || !w.valid) return;
  const long vp = slots[w.si].Vp;
  cx<RI> a[12];
  load_spinor<SI>(field_at<SI>(in, w.off), vp, w.s, a);
  cx<RO> b[12];
  if (add) {
    load_spinor<SO>(field_at<SO>(out, w.off), vp, w.s, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = mk<RO>(b[k].re + (RO)a[k].re, b[k].im + (RO)a[k].im);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = mk<RO>((RO)a[k].re, (RO)a[k].im);
  }
  store_spinor<SO>(field_at<SO>(out, w.off), vp, w.s, b);
}

template <class SI>
static void convert_to(int prec_out, dim3 g, hipStream_t st, const SlotDesc* slots, int nslots, int tu,
                       const void* in, void* out, int add, const int* active) {
  switch (prec_out) {
    case P64: hipLaunchKernelGGL((k_convert<SI, double>), g, dim3(256), 0, st, slots, nslots, tu, in, out, add, active); break;
    case P32: hipLaunchKernelGGL((k_convert<SI, float>), g, dim3(256), 0, st, slots, nslots, tu, in, out, add, active); break;
    case PB16: hipLaunchKernelGGL((k_convert<SI, bf16s>), g, dim3(256), 0, st, slots, nslots, tu, in, out, add, active); break;
    case PH16: hipLaunchKernelGGL((k_convert<SI, f16s>), g, dim3(256), 0, st, slots, nslots, tu, in, out, add, active); break;
    default: throw std::runtime_error("bad precision");
  }
}

void launch_convert(int prec_in, int prec_out, const SlotDesc* slots, int nslots, int total_units,
                    const void* in, void* out, int add, const int* active, hipStream_t st) {
  if (!total_units) return;
  dim3 g(grid_for(total_units, 4));
  switch (prec_in) {
    case P64: convert_to<double>(prec_out, g, st, slots, nslots, total_units, in, out, add, active); break;
    case P32: convert_to<float>(prec_out, g, st, slots, nslots, total_units, in, out, add, active); break;
    case PB16: convert_to<bf16s>(prec_out, g, st, slots, nslots, total_units, in, out, add, active); break;
    case PH16: convert_to<f16s>(prec_out, g, st, slots, nslots, total_units, in, out, add, active); break;
    default: throw std::runtime_error("bad precision");
  }
}

__global__ __launch_bounds__(256) void k_residual_replace(const SlotDesc* slots, int nslots, int total_units,
                                                          const void* c64, const void* ap64, void* r64,
                                                          void* r32, double* partial, const int* flag) {
  UnitRhs w;
  const int u = wave_unit();
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  if (!flag[w.g]) return;
  double n = 0.0;
  if (w.valid) {
    const long vp = slots[w.si].Vp;
    cx<double> c[12], ap[12];
    load_spinor<double>(field_at<double>(c64, w.off), vp, w.s, c);
    load_spinor<double>(field_at<double>(ap64, w.off), vp, w.s, ap);
    cx<float> rf[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      c[k] = c[k] - ap[k];
      rf[k] = mk<float>((float)c[k].re, (float)c[k].im);
    }
    store_spinor<double>(field_at<double>(r64, w.off), vp, w.s, c);
    store_spinor<float>(field_at<float>(r32, w.off), vp, w.s, rf);
    n = norm2(c);
  }
  n = wave_sum(n);
  if ((threadIdx.x & 63) == 0) partial[u] = n;
}

void launch_residual_replace(const SlotDesc* slots, int nslots, int total_units, const void* c64,
                             const void* ap64, void* r64, void* r32, double* partial, const int* flag,
                             hipStream_t st) {
  if (!total_units) return;
  hipLaunchKernelGGL(k_residual_replace, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots,
                     total_units, c64, ap64, r64, r32, partial, flag);
}

__global__ __launch_bounds__(256) void k_diff_norms(const SlotDesc* slots, int nslots, int total_units,
                                                    const void* a, const void* b, double* pd, double* pb) {
  UnitRhs w;
  const int u = wave_unit();
  if (!decode_rhs_unit(slots, nslots, total_units, w)) return;
  double nd = 0.0, nb = 0.0;
  if (w.valid) {
    const long vp = slots[w.si].Vp;
    cx<double> x[12], y[12];
    load_spinor<double>(field_at<double>(a, w.off), vp, w.s, x);
    load_spinor<double>(field_at<double>(b, w.off), vp, w.s, y);
    nb = norm2(y);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = x[k] - y[k];
    nd = norm2(x);
  }
  nd = wave_sum(nd);
  nb = wave_sum(nb);
  if ((threadIdx.x & 63) == 0) {
    pd[u] = nd;
    pb[u] = nb;
  }
}

void launch_diff_norms(const SlotDesc* slots, int nslots, int total_units, const void* a, const void* b,
                       double* partial_diff, double* partial_b, hipStream_t st) {
  if (!total_units) return;
  hipLaunchKernelGGL(k_diff_norms, dim3(grid_for(total_units, 4)), dim3(256), 0, st, slots, nslots,
                     total_units, a, b, partial_diff, partial_b);
}

// ---------------------------------------------------------------------------
// gauge packing
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_gauge(const double* src, int X, int Y, int Z, int T, void* g64,
                                                    void* g32, void* gb16, void* gh16, int* not_su3) {
  const long long V = (long long)X * Y * Z * T;
  const long long vp = pad_half(V / 2);   // row stride of the link chunk rows
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * 4) return;
  const int mu = (int)(i / V);
  const long long lex = i - (long long)mu * V;
  const int x = (int)(lex % X);
  long long rest = lex / X;
  const int y = (int)(rest % Y);
  rest /= Y;
  const int z = (int)(rest % Z);
  const int t = (int)(rest / Z);
  const int par = (x + y + z + t) & 1;
  const long long s = lex >> 1;
  const double2* u = (const double2*)src + (lex * 4 + mu) * 9;
  // a special unitary matrix has orthonormal rows and unit determinant, so
  // its row 2 is the complex conjugate of the cross product of rows 0 and 1:
  // the identity the two-row hops use; flag the storage classes for which a
  // link misses it: by > 1e-6 (16-bit and FP32), by > 1e-7 (FP32)
  {
    double dev = 0.0;
    for (int k = 0; k < 3; ++k) {
      const int ki = (k + 1) % 3, kj = (k + 2) % 3;
      const double2 ai = u[ki], aj = u[kj], bi = u[3 + ki], bj = u[3 + kj];
      const double re = ai.x * bj.x - ai.y * bj.y - (aj.x * bi.x - aj.y * bi.y);
      const double im = ai.x * bj.y + ai.y * bj.x - (aj.x * bi.y + aj.y * bi.x);
      dev = fmax(dev, fmax(fabs(u[6 + k].x - re), fabs(u[6 + k].y + im)));
    }
    if (!(dev <= 1e-6)) atomicOr(not_su3, TWO_ROW_16 | TWO_ROW_32);
    else if (!(dev <= 1e-7)) atomicOr(not_su3, TWO_ROW_32);
  }
  // chunk rows [mu][parity][chunk][site] of vp sites (common.h)
  const long long row = (long long)(mu * 2 + par);
  double2* r64 = (double2*)g64;
  float2* r32 = (float2*)g32;        // 5 chunks of 2 complex
  uint32_t* rb = (uint32_t*)gb16;    // 3 chunks of 4 complex
  uint32_t* rh = (uint32_t*)gh16;
  // the site x + mu, which this link reaches from behind
  int xn[4] = {x, y, z, t};
  const int ext[4] = {X, Y, Z, T};
  xn[mu] = xn[mu] + 1 == ext[mu] ? 0 : xn[mu] + 1;
  const long long sn = (xn[0] + (long long)X * (xn[1] + (long long)Y * (xn[2] + (long long)Z * xn[3]))) >> 1;
  for (int e = 0; e < 12; ++e) {
    const double2 q = e < 9 ? u[e] : make_double2(0.0, 0.0);  // zero padding
    if (e < 9) r64[(row * 9 + e) * vp + s] = q;
    if (e < 10) r32[((row * 5 + e / 2) * vp + s) * 2 + e % 2] = make_float2((float)q.x, (float)q.y);
    const cx<float> qf = mk<float>((float)q.x, (float)q.y);
    const long long w16 = ((row * 3 + e / 4) * vp + s) * 4 + e % 4;
    rb[w16] = pack2<bf16s>(qf);
    rh[w16] = pack2<f16s>(qf);
    if (e == 8) {   // the ninth entry again, beside those of the site's other forward links
      const long long n16 = ((long long)(LINK_ROW_NINTH + par) * vp + s) * 4 + mu;
      rb[n16] = pack2<bf16s>(qf);
      rh[n16] = pack2<f16s>(qf);
      // and at x + mu, among the links reaching that site from behind
      const long long b16 = ((long long)(LINK_ROW_NINTH_BWD + 1 - par) * vp + sn) * 4 + mu;
      rb[b16] = pack2<bf16s>(qf);
      rh[b16] = pack2<f16s>(qf);
    }
    if (e < 6) {    // rows 0 and 1 again, site-centred, at x and at x + mu
      const int j = 6 * (mu & 1) + e;
      const long long cf = (long long)LINK_ROW_R12 + 12 * par + 3 * (mu >> 1) + j / 4;
      const long long cb = (long long)LINK_ROW_R12 + 12 * (1 - par) + 6 + 3 * (mu >> 1) + j / 4;
      rb[(cf * vp + s) * 4 + j % 4] = pack2<bf16s>(qf);
      rh[(cf * vp + s) * 4 + j % 4] = pack2<f16s>(qf);
      rb[(cb * vp + sn) * 4 + j % 4] = pack2<bf16s>(qf);
      rh[(cb * vp + sn) * 4 + j % 4] = pack2<f16s>(qf);
    }
  }
}

void launch_pack_gauge(const double* src, int X, int Y, int Z, int T, void* g64, void* g32, void* gb16,
                       void* gh16, int* not_su3, hipStream_t st) {
  const long long n = (long long)X * Y * Z * T * 4;
  hipLaunchKernelGGL(k_pack_gauge, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, X, Y, Z, T, g64,
                     g32, gb16, gh16, not_su3);
}

}  // namespace dl
