/*
 * discloop.h -- C ABI of the MI355X (gfx950) stochastic fermion-loop library.
 *
 * The library computes disconnected fermion loops of twisted-mass Wilson
 * fermions the way the paper "A QUDA-branch to compute disconnected diagrams
 * in GPUs" (LATTICE 2013) describes them:
 *   - many stochastic inversions M s_r = eta_r (Section 2, eq. (1)) with
 *     volume noise generated on the GPU (Section 2.3 draws it on the host;
 *     Section 2.4 names that as a bottleneck and plans GPU generation);
 *   - the truncated solver method (Section 2.1): many low-precision solves
 *     plus a few high-precision corrections;
 *   - one-end-trick contractions for all ultra-local and one-derivative
 *     insertions, with and without tau_3 (Section 2.1.1, Section 2.2),
 *     accumulated over sources on the GPU (the all-GPU scheme of Section 2.4,
 *     Fig. 4) and projected to momenta with a p^2 cut (Section 2.3);
 *   - the options the interfaces combine with them: per-set partial sums for
 *     base-2 storage (Section 2.1.1, Fig. 2; dl_loops_sets), the hopping
 *     parameter expansion of the loops without tau_3 (Section 2.3;
 *     DL_OPS_HPE), time-diluted sources (Section 2.2; dl_job.tdil), and the
 *     Wilson operator as mu = 0 (Section 2.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice dims are {X, Y, Z, T}, every extent even and >= 2.  The site index
 * is lexicographic, x fastest: site = x + X (y + Y (z + Z t)).
 * Operator (kappa normalised, u flavour):
 *     M = 1 - kappa H + 2 i kappa mu gamma_5,
 *     (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                       + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu),
 * chiral gamma basis (gamma_5 = diag(1, 1, -1, -1)), periodic in space, and
 * a factor t_bc on every hop across the time boundary.  The d flavour is
 * M(-mu).
 * Host/device spinor fields at the boundary are complex128, laid out
 * [site][spin 4][colour 3] (interleaved re, im).  Gauge fields are complex128
 * [t][z][y][x][mu 4][3][3] (row-major 3x3, mu = 0..3 for x, y, z, t).
 * Pointers documented "device" must be device memory of the context's GPU;
 * the library never takes ownership of caller memory.
 *
 * Every call returns an int status: 0 OK; 1 DL_NOT_CONVERGED (results were
 * written, per-source flags tell which ones); negative values are errors
 * (see DL_E*).  dl_last_error() returns a thread-local message for the last
 * failing call on the calling thread.  No C++ exception crosses this ABI.
 * All GPU work is ordered on the context's stream; calls that return host
 * results synchronise that stream before returning.
 */
#ifndef DISCLOOP_H
#define DISCLOOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DL_OK 0
#define DL_NOT_CONVERGED 1
#define DL_EINVAL (-1)
#define DL_ENOMEM (-2)
#define DL_EHIP (-3)
#define DL_ESTATE (-4)
#define DL_EBREAKDOWN (-5)

/* noise of the volume sources (Section 2): Z2 = real +-1, Z4 = {1, i, -1, -i};
 * USER = caller-provided sources (dl_job.src_in). */
#define DL_NOISE_Z2 0
#define DL_NOISE_Z4 1
#define DL_NOISE_USER 2

/* solver tiers of the truncated solver method (Section 2.1).
 *   FP64     plain method: fields, links and arithmetic in FP64.
 *   LP_BF16  low precision: bf16-stored spinors and links, FP32 arithmetic,
 *            FP64 dot products.
 *   LP_FP16  as LP_BF16 with IEEE half storage.
 *   HP_FP32  high precision: FP32 fields and arithmetic with FP64 reliable
 *            updates (true residual and solution accumulated in FP64). */
#define DL_TIER_FP64 0
#define DL_TIER_LP_BF16 1
#define DL_TIER_LP_FP16 2
#define DL_TIER_HP_FP32 3

/* accumulator sets of the TSM estimator
 *   L = S_LP / N_LP + (S_HP - S_LPC) / N_HP
 * LP: low-precision solves of the LP sources; HP: high-precision solves of
 * the correction sources; LPC: low-precision solves of those same sources. */
#define DL_SET_LP 0
#define DL_SET_HP 1
#define DL_SET_LPC 2

/* insertion sets: LOCAL = 16 ultra-local Gamma; DERIV adds the 4 x 16
 * one-derivative insertions (Section 2.1.1: 160 with both flavours). */
#define DL_OPS_LOCAL 1
#define DL_OPS_DERIV 2
/* Hopping parameter expansion of the loops without tau_3 (one of the variance
 * reductions of the interfaces, Section 2.3), order n = 1..4, or'ed into the
 * ops of dl_accum_create.  With B = A^-1, A = 1 + 2 i kappa mu gamma_5 and
 * M = A - kappa H, M^-1 = sum_{k<n} (kappa B H)^k B + (kappa B H)^n M^-1: the
 * first sum is added exactly (its elements used here do not depend on the gauge
 * field) and only the remainder is estimated, from phi = (kappa B H)^n s and the
 * source eta, the d flavour by gamma_5-hermiticity from the same sample.
 * Derivative insertions use order min(n, 3).  Requires every lattice extent
 * >= 4.  The loops with tau_3 keep the one-end trick. */
#define DL_OPS_HPE(n) ((n) << 4)
#define DL_OPS_HPE_ORDER(ops) (((ops) >> 4) & 7)

/* per-source status in dl_src_stats.status */
#define DL_SRC_CONVERGED 0
#define DL_SRC_MAXITER 1
#define DL_SRC_BREAKDOWN 2

typedef struct dl_ctx dl_ctx;
typedef struct dl_lattice dl_lattice;
typedef struct dl_accum dl_accum;

/* One batch entry of dl_solve_batch: nsrc sources of one lattice and tier. */
typedef struct dl_job {
  dl_lattice* lat;       /* lattice (gauge field and kappa, mu set) */
  int noise;             /* DL_NOISE_* */
  int tier;              /* DL_TIER_* */
  uint64_t seed;         /* noise seed (Z2 / Z4) */
  int64_t first_src;     /* index r of the first source; source r is a pure
                            function of (seed, r) */
  int nsrc;              /* number of sources, >= 0 */
  int maxiter;           /* CG iteration cap per source, > 0 */
  double tol;            /* target relative residual rho (> 0) */
  int rhs_block;         /* sources interleaved per slot; 0 = autotuned */
  int report_true_resid; /* nonzero: also compute ||eta - M s|| / ||eta|| in FP64 */
  const double* src_in;  /* DL_NOISE_USER: device complex128 [nsrc][V][12] */
  double* sol_out;       /* optional device complex128 [nsrc][V][12]: s_r */
  dl_accum* accum;       /* optional: add the loops of every source here */
  int accum_set;         /* DL_SET_* */
  int guess_from;        /* 0: CG starts from zero.  j + 1 (HP tier only): start
                            from the solutions of job j of the same call, which
                            must be a lower tier (FP64, LP_BF16 or LP_FP16) over
                            the same lattice and sources (noise, seed,
                            first_src, nsrc, src_in).  The final accuracy is
                            unchanged; the truncated-solver correction solves
                            then start at the low-precision residual. */
  int tdil;              /* time dilution (Section 2.2 works with time-diluted
                            sources): 0 or 1 = none; D >= 2 (at most T) splits every
                            noise vector r into D sources eta_(r,c), c = 0..D-1, equal
                            to eta_r on the time slices t with t mod D == c and zero
                            elsewhere, each solved on its own.  nsrc still counts
                            noise vectors; the job's stats and sol_out hold nsrc * D
                            entries, component-major (entry c * nsrc + r - first_src);
                            src_in (USER noise) holds the nsrc undiluted vectors.  The
                            loops of one noise vector are the sum over its components,
                            so the accumulator's source count grows by nsrc.  One-end-
                            trick structures contract every component over the whole
                            lattice; the hopping parameter expansion, which pairs eta
                            with the solution, only next to the component's slices. */
  int grad_ops;          /* dl_loops_backward without an accumulator (accum NULL):
                            the insertion set of the loops, DL_OPS_LOCAL or
                            DL_OPS_LOCAL | DL_OPS_DERIV (0 = LOCAL | DERIV).
                            Ignored when accum is set; dl_solve_batch ignores it. */
} dl_job;

typedef struct dl_src_stats {
  int iters;             /* CG iterations taken */
  int status;            /* DL_SRC_* */
  double rel_resid;      /* final iterated relative residual of the normal system */
  double true_resid;     /* ||eta - M s|| / ||eta|| (FP64), or -1 if not requested */
  int reliable_updates;  /* HP tier: number of FP64 reliable updates */
  int pad;
} dl_src_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t, may
 * be NULL for the null stream) is borrowed: all work of this context is
 * ordered on it and it must outlive the context. */
int dl_create(dl_ctx** out, int device, void* hip_stream);
int dl_destroy(dl_ctx* ctx);
/* Message of the last failing call on this thread ("" if none). */
const char* dl_last_error(void);
/* Library version string. */
const char* dl_version(void);

/* ---- lattice and gauge field ------------------------------------------- */

/* Create a lattice {X, Y, Z, T} (all even, >= 2) with time boundary factor
 * t_bc (-1 antiperiodic, +1 periodic).  The library owns its device fields.
 * DL_EINVAL for an odd or too small extent, a bad t_bc, or more than 2^28
 * sites per parity (the kernels' 32-bit row offsets); DL_ENOMEM when the
 * link arrays do not fit. */
int dl_lattice_create(dl_ctx* ctx, const int dims[4], int t_bc, dl_lattice** out);
int dl_lattice_destroy(dl_lattice* lat);

/* Copy a gauge field in (layout above) and pack it into the FP64, FP32, bf16
 * and fp16 even-odd layouts.  on_device: 0 host pointer, 1 device pointer.
 * The caller keeps ownership of `links`.  Any complex 3x3 links are accepted;
 * when every link's row 2 equals the complex conjugate of the cross product
 * of rows 0 and 1 to 1e-6 (true of SU(3) matrices, the links of lattice
 * QCD), the bf16 / fp16 hopping kernels read rows 0 and 1 only and
 * rebuild row 2, otherwise they read all nine entries (checked here, on the
 * GPU, once per call). */
int dl_gauge_set(dl_lattice* lat, const double* links, int on_device);

/* Synthetic gauge field, the stand-in for the paper's twisted-mass ensembles
 * (Section 2.1.1 measures on 32^3 x 64 configurations): every link is
 * U = exp(i eps H), H = sum_a h_a lambda_a / 2 over the eight Gell-Mann
 * matrices with h_a ~ N(0, 1).  The Gaussians come from Box-Muller on a
 * SplitMix64 counter stream (Steele, Lea & Flood 2014): link l = 4 site + mu
 * (site lexicographic, x fastest) uses outputs 8 l .. 8 l + 7 of stream
 * `seed`, output i being mix(seed + (i + 1) 0x9E3779B97F4A7C15), mapped to
 * (0, 1) by its top 53 bits; pair k gives h_2k = sqrt(-2 ln u_2k) cos(2 pi
 * u_2k+1), h_2k+1 the sine.  A link is a pure function of (seed, site, mu),
 * so a C caller and the library's Python test inputs build the same field.
 *   dl_gauge_random      generates the field on the host and loads it into
 *                        the lattice as dl_gauge_set does;
 *   dl_gauge_random_host writes it to caller host memory `links`, complex128
 *                        [t][z][y][x][mu][3][3] (the dl_gauge_set layout),
 *                        dims {X, Y, Z, T} >= 1; no GPU is used.
 * Errors: DL_EINVAL (NULL argument, non-finite eps). */
int dl_gauge_random(dl_lattice* lat, uint64_t seed, double eps);
int dl_gauge_random_host(const int dims[4], uint64_t seed, double eps, double* links);

/* Set kappa (> 0) and mu of the operator.  mu = 0 is the Wilson operator
 * (Section 2.4 expects the code to carry over to Wilson-type fermions): u and
 * d coincide, the loops with tau_3 vanish and those without it are the plain
 * Wilson loops, tr Gamma 2 D_W^-1; dl_loops_backward then gives no dF/dmu. */
int dl_set_params(dl_lattice* lat, double kappa, double mu);

/* Clover term (Section 2.4 expects the package to work for Wilson and clover
 * fermions; the operator is not printed there).  With c_sw != 0 the operator
 * is the O(a)-improved one in kappa normalisation:
 *     M = 1 + C - kappa H + 2 i kappa mu gamma_5,
 *     C(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *     sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
 *     Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / 8,
 * Q the four plaquettes of the (mu, nu) plane that start and end at x, each
 * walked like U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag (links periodic in
 * every direction; t_bc acts on the fermion hops only).  C is hermitian,
 * independent of mu and commutes with gamma_5, so the d flavour is M(-mu), the
 * even-odd solves use the per-site matrices A = 1 + C + 2 i kappa mu gamma_5
 * (two 6 x 6 blocks) and the loops without tau_3 use xi = (1 + C - kappa H) s.
 * The site matrices are built on the GPU whenever the gauge field, kappa / mu
 * or c_sw change (FP64 and FP32 copies, 1.7 kB per site).  c_sw = 0 removes
 * the term.  Not built for clover lattices: the hopping parameter expansion
 * (dl_solve_batch refuses DL_OPS_HPE accumulators) and dl_loops_backward.
 * Errors: DL_EINVAL (NULL lattice, non-finite c_sw), DL_ENOMEM. */
int dl_set_clover(dl_lattice* lat, double csw);

/* ---- solves and loops -------------------------------------------------- */

/* Solve every source of every job (Section 2, eq. (1)) by even-odd CGNR at
 * the job's tier, then add the one-end-trick loops of each solution to the
 * job's accumulator set.  Jobs of the same precision class run together in
 * shared launches (different lattices and source blocks interleaved).
 * stats: optional host array of sum(nsrc * max(tdil, 1)) entries, in job order.
 * Returns DL_NOT_CONVERGED if any source missed its tolerance. */
int dl_solve_batch(dl_ctx* ctx, const dl_job* jobs, int njobs, dl_src_stats* stats);

/* Per-site FP64 loop accumulators of one lattice (three TSM sets).  ops:
 * DL_OPS_LOCAL or DL_OPS_LOCAL | DL_OPS_DERIV, optionally | DL_OPS_HPE(n).
 * The jobs of one dl_solve_batch call that accumulate into HPE accumulators
 * must all use the same order.  DL_EINVAL for other values, or for HPE on a
 * lattice with an extent below 4. */
int dl_accum_create(dl_lattice* lat, int ops, dl_accum** out);
int dl_accum_reset(dl_accum* acc);
int dl_accum_destroy(dl_accum* acc);
/* Number of sources added to each set (counts[3] = {LP, HP, LPC}). */
int dl_accum_counts(const dl_accum* acc, int64_t counts[3]);

/* Integer momenta n with |n|^2 <= p2max, components in (-L/2, L/2] of the
 * lattice's spatial extents, ordered by |n|^2 then (n_x, n_y, n_z).  Writes
 * up to cap vectors to n_xyz (host int[cap][3], may be NULL) and returns the
 * count in *np_out. */
int dl_momenta(const int dims[4], int p2max, int* n_xyz, int cap, int* np_out);

/* Project the accumulated loops (Section 2.3: Fourier transform over space
 * per time slice, cut at p^2 <= p2max), rebuild the 16 Gamma insertions from
 * the 4x4 outer products (Section 2.2), combine the TSM sets and apply the
 * one-end-trick prefactors.  out: complex128 [2][nops][16][T][Np], flavour 0
 * with tau_3, 1 without; op 0 local, 1..4 derivative along x, y, z, t
 * (nops = 1 or 5 by the accumulator's ops); host (out_on_device = 0) or
 * device pointer.  *np_out receives Np.  With DL_OPS_HPE the loops without
 * tau_3 are the expansion's estimate: exact part plus estimated remainder. */
int dl_loops(dl_ctx* ctx, dl_accum* acc, int p2max, double* out, int out_on_device,
             int* np_out);

/* The three TSM sets separately, without the division by their source counts:
 * out[s] (s = DL_SET_LP, DL_SET_HP, DL_SET_LPC) is the sum over the set's
 * sources of the loops that dl_loops normalises (same projection, Gamma
 * rebuild and prefactors), layout complex128 [3][2][nops][16][T][Np].  A set
 * without sources gives zeros.  With dl_accum_counts the TSM estimate is
 * S_LP / N_LP + (S_HP - S_LPC) / N_HP; partial sums of disjoint source blocks
 * add up, which is what base-2 storage of partial sums needs (Section 2.1.1,
 * Fig. 2).  Errors as dl_loops. */
int dl_loops_sets(dl_ctx* ctx, dl_accum* acc, int p2max, double* out, int out_on_device, int* np_out);

/* Bytes of the per-GPU device scratch array of dl_loops_noalloc. */
#define DL_LOOPS_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* dl_loops for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same projection, Gamma rebuild, TSM combination and prefactors as dl_loops,
 * through the same kernels, with out a device pointer (complex128
 * [2][nops][16][T][Np]); *np_out receives Np.  No hipMalloc, hipFree or other
 * device allocation: the projection's tables and partial sums use a file-scope
 * device array of DL_LOOPS_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the
 * library runs on holds from its first dl_create until the process ends.  A
 * projection needs about 16 (nq T Z n_xy + nq T Np) bytes of it (nq = 48
 * local, 240 with derivative insertions; n_xy distinct (n_x, n_y) pairs among
 * the Np momenta): 61 MiB for 24^3 x 48 with derivatives at p^2 <= 4.  A call
 * that needs more fails with DL_EINVAL before any GPU work.  All calls on one
 * GPU share the array and every call overwrites all of it that it reads, so
 * nothing carries over between calls; calls that overlap on one GPU (other
 * contexts' streams, other threads) race and must be ordered by the caller.
 * The small index and phase tables are uploaded from host memory with
 * hipMemcpyAsync.  Errors as dl_loops. */
int dl_loops_noalloc(dl_ctx* ctx, dl_accum* acc, int p2max, double* out, int* np_out);

/* Gradients of the loops of one job's sources with respect to the sources and
 * to mu, for a real loss F.  The loops are the plain estimator over the job's
 * nsrc sources (what dl_loops returns for an accumulator that holds only
 * them); nops is that of job->accum, or of job->grad_ops when job->accum
 * is NULL (the accumulator is read for its insertion set only, so a caller
 * may free it after dl_loops and pass grad_ops instead).
 * Complex gradients follow PyTorch's convention, dF/dRe z + i dF/dIm z:
 *   grad_loops  host complex128 [2][nops][16][T][Np], the gradient of F with
 *               respect to the loops;
 *   grad_eta    device complex128 [nsrc][V][12] (optional): gradient with
 *               respect to the sources eta (job->src_in for USER noise);
 *   grad_mu     host double (optional): dF/dmu.
 * If job->sol_out is set it must hold the solutions of the forward call
 * (checkpoint) and is read; otherwise they are recomputed.  One adjoint solve
 * per source, M^dag = gamma_5 M(-mu) gamma_5, at job->tier and job->tol.
 * DL_EINVAL if job->accum uses DL_OPS_HPE (not differentiated). */
int dl_loops_backward(dl_ctx* ctx, const dl_job* job, int p2max, const double* grad_loops,
                      double* grad_eta, double* grad_mu);

/* ---- options and kernel timing ----------------------------------------- */

/* Set a context option (name, numeric value):
 *   "inflight_rhs"  max right-hand sides solved together per launch (>= 1)
 *   "inflight_mb"   device memory budget of one batch of solves, MiB
 *   "use_graph"     1: replay CG iterations from a HIP graph; 0: plain launches
 *   "block_hop"     1: 16-bit hops through the LDS-staged kernel (a block of
 *                   whole x-rows and its y / z halo staged in LDS per time
 *                   slice) on lattices whose shape allows it; 0 (default): the
 *                   tile kernel.  Changes the norms' summation order, so the
 *                   low-precision iterates, not their accuracy.
 *   "contract_tblk" time slices per block of the derivative contraction's
 *                   tile order (1..64, default 8): the tiles at one place of
 *                   successive slices run together, so a tile's +t neighbour
 *                   rows are read while they are still cached.  Results do
 *                   not depend on it.
 *   "profile"       1: time every hopping-kernel launch of the CG (the
 *                   u_e = A^-1 H_eo p_o step) with HIP events on the context
 *                   stream and count its compulsory bytes; 0: off
 * Returns DL_EINVAL for an unknown name or value. */
int dl_set_option(dl_ctx* ctx, const char* name, double value);

/* Read and reset the profile counters of the hopping kernel for one storage
 * tier: out[0] launches, out[1] total kernel milliseconds, out[2] total
 * compulsory HBM bytes (links once per lattice and launch, input and output
 * spinor once per active right-hand side), out[3] total active rhs. */
int dl_profile_read(dl_ctx* ctx, int tier, double out[4]);

/* Slot shape that dl_solve_batch uses for a job of `nsrc` sources of `tier`
 * on `lat` when job->rhs_block is 0: *block_out right-hand sides per batch
 * slot and, if tblk_out is not NULL, *tblk_out time slices per block of the
 * hopping kernel's tile order.  The first call per (lattice shape, storage
 * precision, size class = next power of two of nsrc in [16, 128]) runs the
 * autotuner: it times the hopping kernel on size-class many scratch
 * right-hand sides for blocks 1, 2, 4, ... and tile-order depths 1, 2, 4, 8
 * and keeps the fastest (a later candidate only when more than 2% faster).
 * Results are cached in the context and in the JSON file named by the
 * environment variable DL_TUNE_CACHE (default ~/.cache/discloop/
 * tune-gfx950.json); an unwritable file only costs a re-tune.  The choice
 * never changes results, only speed.  Synchronises the context stream.
 * Errors: DL_EINVAL (NULL argument, nsrc < 1, unknown tier), DL_EHIP. */
int dl_autotune(dl_ctx* ctx, dl_lattice* lat, int tier, int nsrc, int* block_out, int* tblk_out);

/* ---- single operators, for verification -------------------------------- */

/* Operators of dl_apply_op. */
#define DL_OP_M 0        /* M psi, full lattice */
#define DL_OP_MDAG 1     /* M^dag psi */
#define DL_OP_MHAT 2     /* even-odd Schur complement on odd sites */
#define DL_OP_MHAT_DAG 3 /* its adjoint */
#define DL_OP_HOP 4      /* the hopping term H psi */

/* Apply one operator to nrhs fields through the library's kernels at
 * precision `tier` (its storage type).  in/out: device complex128
 * [nrhs][V][12]; for MHAT / MHAT_DAG only odd sites of `in` are read and the
 * even sites of `out` are set to zero. */
int dl_apply_op(dl_lattice* lat, int op, int tier, const double* in, double* out, int nrhs);

/* Write source number `src` (Z2 / Z4) to out (device complex128 [V][12]). */
int dl_fill_noise(dl_lattice* lat, int noise, uint64_t seed, int64_t src, double* out);

#ifdef __cplusplus
}
#endif

#endif /* DISCLOOP_H */
