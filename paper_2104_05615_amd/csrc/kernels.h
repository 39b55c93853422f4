// Host-side launch interface of the library's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mspcg {

enum class Prec : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, I8 = 4 };

// Size of the static device workspace of mspcg_apply_device_noalloc (one
// copy per device, held until the process ends), and its address on the
// current device (resolved once per device; call with the device current).
constexpr size_t kScratchBytes = size_t(128) << 20;
void* scratch_device_ptr();

// A single-parity 5D field in device memory, type-erased.
struct FieldPtr {
  void* data = nullptr;
  float* scale = nullptr;
  int64_t stride = 0;   // chunks per chunk-array (= n5)
  Prec prec = Prec::F32;
};

template <typename S> inline Field<S> typed(const FieldPtr& f) {
  Field<S> r;
  r.data = reinterpret_cast<typename Field<S>::chunk*>(f.data);
  r.scale = f.scale;
  r.stride = f.stride;
  return r;
}

// Fused epilogue after a hop, per 5D site (x, s) and chirality chi:
//   out(s) = E0 w(s) [or w(s) if w_identity] + E1 h(s) [or h(s) if E1 null]
// with Ls x Ls real matrices per chirality ([2][Ls][Ls], calc precision).
// If dot_partial is set, each block writes Re<dotf, out> over its sites.
struct Epilogue {
  const void* E0 = nullptr;
  const void* E1 = nullptr;
  bool w_identity = false;
  double* dot_partial = nullptr;
  const FieldPtr* dotf = nullptr;
};

// Right-hand sides of one launch.  A batched field holds its RHS one after
// another (RHS r starts r whole fields after RHS 0); solver scalars are
// [r][SLOT_COUNT], per-subdomain scalars [r][nsub] and block partials
// [r][blocks per RHS].  Every kernel skips RHS r when mask[r] == 0.
struct Batch {
  int n = 1;
  const int* mask = nullptr;
};

// Workgroup -> (site block, RHS) mapping of the hop kernels, one workgroup
// per item.  order 0 runs the RHS outermost; order 1 puts the RHS of one site
// block next to each other, so they read the block's links from one L2.
// xcd = 1 deals contiguous item ranges to each XCD (neighbouring site blocks
// share an L2), 0 leaves the hardware's round-robin order.  Partial sums are
// indexed by (RHS, site block), so no schedule changes a result.
struct Sched {
  int order = 0;
  int xcd = 1;
  int tchunk = 0;   // full-lattice hops: 0 lexicographic block order, k > 0 chunked t sweep of ~(80 << k) KB chunks
};

struct HopGeometry {
  Lattice lat;
  int out_parity;
  int Ls;
};

// slots of the outer solver's device scalar array
enum ScalarSlot { SLOT_RHO = 0, SLOT_PAP, SLOT_ALPHA, SLOT_BETA, SLOT_RR, SLOT_RZ, SLOT_RZOLD, SLOT_R64, SLOT_TMP,
                  SLOT_COUNT = 16 };
enum FinishMode { FIN_STORE = 0, FIN_ALPHA, FIN_RHO, FIN_BETA_FR, FIN_BETA_PR };

// sites per block of the site kernels (16 when the MFMA epilogue is used)
int sites_per_block(int Ls, Prec p);
bool uses_mfma(int Ls, Prec p);
// epilogue engine of every handle of the process (MFMA on by default)
void set_mfma_epilogue(bool on);
bool mfma_epilogue();
int64_t full_blocks(int64_t vh, int Ls, Prec p);

// ---------------------------------------------------------------- site kernels
// the dot partials of a hop are [rhs][site blocks]
void hop_full(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w,
              const void* gauge, const HopGeometry& geo, bool dagger, const Epilogue& epi,
              const Batch& bt = Batch(), const Sched& sc = Sched());
void hop_sub(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, const void* gauge,
             const Lattice& lat, int out_parity, const SubTables& tb, int nsub, int Ls, bool dagger,
             const Epilogue& epi, const Batch& bt = Batch(), const Sched& sc = Sched());
// site blocks per RHS of hop_full / hop_sub
int64_t hop_full_blocks(const Lattice& lat, int Ls, Prec p);
// out = E w (E null: copy); optional |out|^2 partials (one per block)
void apply5_full(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& w, const void* E, int64_t nsites,
                 int Ls, double* norm_partial, const Batch& bt = Batch());
// p <- z + beta p (beta = scal[beta_slot]);  out = E p
void xpay_apply5(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& pvec, const FieldPtr& z,
                 const double* scal, int beta_slot, const void* E, int64_t nsites, int Ls, const Batch& bt = Batch());

// ---------------------------------------------------------------- layouts
// canonical FP64 [Ls][nsites][4][3] complex <-> internal (a batch: RHS r at
// canon + r * nsites * Ls * 24)
void pack_field(hipStream_t st, const FieldPtr& out, const double* canon, int64_t nsites, int Ls,
                const Batch& bt = Batch());
void unpack_field(hipStream_t st, double* canon, const FieldPtr& in, int64_t nsites, int Ls,
                  const Batch& bt = Batch());
// p[0..n) = v (a kernel, so that graph capture records no memset)
void fill_int(hipStream_t st, int* p, int n, int v);
// zero bytes_per_rhs bytes of every masked RHS (bytes_per_rhs % 16 == 0)
void zero_batched(hipStream_t st, void* data, int64_t bytes_per_rhs, const Batch& bt);
// gauge: canonical [T][Z][Y][X][4][3][3] complex FP64 -> [parity][mu][vh][10] double2 / float2 / half2
// (bytes_per_real 8, 4 or 2)
// (9 entries of a link padded to 10)
void pack_gauge(hipStream_t st, void* out, int bytes_per_real, const double* canon, const Lattice& lat);

// ---------------------------------------------------------------- outer BLAS-1 (FP64 / FP32 fields)
int64_t blas_blocks(int64_t nchunks);
// x += alpha p ; rn = r - alpha q ; partial |rn|^2.  nreal = 24 * n5 (per RHS).
void cg_update(hipStream_t st, Prec p, void* x, const void* pv, const void* r, const void* q, void* rn, int64_t nreal,
               const double* scal, int alpha_slot, double* partial, int64_t nblocks, const Batch& bt = Batch());
// partial Re<a,b1>, Re<a,b2> (b2 nullable)
void dot2(hipStream_t st, Prec p, const void* a, const void* b1, const void* b2, int64_t nreal, double* partial1,
          double* partial2, int64_t nblocks, const Batch& bt = Batch());
// r64 = b - Ax (r64 nullable) ; partial |r64|^2 ; r_lo = (float) r64 if r_lo
void residual64(hipStream_t st, const double* b, const double* Ax, double* r64, float* r_lo, int64_t n5,
                double* partial, int64_t nblocks, const Batch& bt = Batch());
// x64 += x_lo ; x_lo = 0
void accum_lo(hipStream_t st, double* x64, float* xlo, int64_t n5, const Batch& bt = Batch());
void f64_to_f32(hipStream_t st, const double* a, float* b, int64_t n5, const Batch& bt = Batch());
// reduce partial sums (fixed order) and update solver scalars (FinishMode);
// with p1 null, S1 is taken from scal[slot].  One RHS per workgroup.
void finish(hipStream_t st, const double* p1, const double* p2, int64_t n, double* scal, int mode, int slot,
            const Batch& bt = Batch());

// ---------------------------------------------------------------- per-RHS solver control
//
// The outer iteration's decisions (convergence, reliable update, breakdown,
// iteration limit) are taken on the device, so that an iteration needs no
// host round trip and can be replayed as a captured graph.
enum RhsStatus { RHS_RUNNING = 0, RHS_OK, RHS_NOT_CONVERGED, RHS_BREAKDOWN };
struct Ctl {
  int* active;    // RHS still iterating (the mask of the iteration's kernels)
  int* ru;        // reliable update in this iteration (mask of its kernels)
  int* bzero;     // zero source: x = 0
  int* status;    // RhsStatus
  int* iters;     // outer iterations
  int* rus;       // reliable updates
  int* precs;     // preconditioner applications
  int* nactive;   // one int: number of RHS still iterating
  double* bnorm;  // |b|
  double* rmax;   // largest residual norm since the last reliable update
  double* rr;     // last |r|^2 (iterated, or true after a reliable update)
};
struct CtlParams {
  double tol, delta;
  int maxiter;
};
// from scal[TMP] = |b|^2: status, active, bnorm; scal[TMP] = 0.  With a
// join mask only the RHS r with join[r] != 0 start (the others keep their
// state), and join[r] becomes active[r]: the start-up kernels after it use
// join as their mask.
void ctl_init(hipStream_t st, const Ctl& c, double* scal, int n, int* join);
// starting residual: scal[R64] (has_x0) or |b|^2; rmax, rr (RHS of join only)
void ctl_start(hipStream_t st, const Ctl& c, const double* scal, int n, bool has_x0, const int* join);
// after the iterated |r|^2 (scal[RR]) and pAp (scal[PAP]): breakdown,
// iteration count, reliable-update decision
void ctl_iterate(hipStream_t st, const Ctl& c, const double* scal, int n, const CtlParams& p);
// after the reliable-update kernels: true residual (scal[R64]) decides
// convergence; iteration limit; scal[RR] = the current |r|^2; counts the
// RHS still active
void ctl_after_update(hipStream_t st, const Ctl& c, double* scal, int n, const CtlParams& p);

// ---------------------------------------------------------------- preconditioner (sub.hip)
//
// Per-subdomain inner CG state: rho[d], alpha[d], beta[d], active[d].
struct SubScalars {
  double* rho;      // rho of the current iteration (and the one SUB_INIT / SUB_BETA write)
  double* alpha;
  double* beta;
  int* active;
  double* rho_next; // sub_xpay5 reads rho and writes rho_next (the caller swaps them)
};

// Restrict the outer residual to the centre region of every subdomain:
//   r_s = R_s r,  p_s = r_s,  t0 = E p_s (M_phi),  partial |r_s|^2 (per block, [d][bps])
void sub_restrict(hipStream_t st, Prec outer, Prec inner, const FieldPtr& r_outer, const FieldPtr& rs,
                  const FieldPtr& ps, const FieldPtr& t0, const void* E, const Lattice& lat, const SubTables& tc,
                  int nsub, int Ls, double* partial, const Batch& bt = Batch());
// alpha_d = rho_d / <p_s, q_s> from the [d][bps] partials pq (SUB_ALPHA, computed
// by every wavefront), then z_s (+)= alpha_d p_s ; r_s -= alpha_d q_s ;
// partial |r_s|^2  (first: z_s = alpha_d p_s).  last: the k-th step, whose
// residual nothing reads: z_s only (r_s, q_s untouched, partials zero).
void sub_update(hipStream_t st, Prec inner, const FieldPtr& zs, const FieldPtr& ps, const FieldPtr& rs,
                const FieldPtr& qs, const SubScalars& sc, bool first, bool last, const SubTables& tc, int nsub,
                int Ls, const double* pq, double* partial, const Batch& bt = Batch());
// beta_d = |r_s|^2 / rho_d from the [d][bps] partials rr (SUB_BETA, computed by
// every wavefront; rho_next = |r_s|^2), then p_s = r_s + beta_d p_s ; t0 = E p_s
void sub_xpay5(hipStream_t st, Prec inner, const FieldPtr& ps, const FieldPtr& rs, const FieldPtr& t0,
               const SubScalars& sc, const double* rr, const void* E, const SubTables& tc, int nsub, int Ls,
               const Batch& bt = Batch());
// z = sum_s R_s^T z_s (outer precision); partials Re<z, r>, Re<z, r_old> (r_old nullable)
void sub_prolong(hipStream_t st, Prec outer, Prec inner, const FieldPtr& z_outer, const FieldPtr& zs,
                 const FieldPtr& r_outer, const FieldPtr* rold_outer, const Lattice& lat, const SubTables& tc,
                 int nsub, int Ls, double* partial1, double* partial2, const Batch& bt = Batch());
// per-subdomain scalar updates from [d][bps] partials:
//   SUB_INIT : rho = S, active = rho > 0
//   SUB_ALPHA: alpha = rho / S (0 and inactive if S <= 0 or not finite)
//   SUB_BETA : if S == 0 inactive; beta = S / rho; rho = S
enum SubFinish { SUB_INIT = 0, SUB_ALPHA, SUB_BETA };
void sub_finish(hipStream_t st, const double* partial, int bps, int nsub, const SubScalars& sc, int mode,
                const Batch& bt = Batch());

// ---------------------------------------------------------------- reduced-Ls preconditioner (reduced.hip)
// out(x, so, mo, c) = sum_{si, mi} W[so][mo][si][mi] in(x, si, mi, c) (+ mu r(x, so, mo, c) when r
// is given); W complex [Lo][4][Li][4] (double2 for FP64 fields, float2 for FP32).  With p1 set,
// workgroup partials of Re<out, r> (p1) and Re<out, rold> (p2, when rold is given), indexed
// [rhs][transform_blocks].
int transform_sites(int Li, int Lo, Prec p);
int64_t transform_blocks(int64_t vh, int Li, int Lo, Prec p);
void transform(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const void* W, int Li, int Lo,
               int64_t vh, double mu, const FieldPtr* r, const FieldPtr* rold, double* p1, double* p2,
               const Batch& bt = Batch());
// e = a - b over nreal reals of one layout, workgroup sums of e^2 in partial[nblocks]
void diff_norm(hipStream_t st, Prec p, void* e, const void* a, const void* b, int64_t nreal, double* partial,
               int nblocks);
// G[(s mf)(t mg)] += sum over sites and colour of f(x, s, mf, c) conj(g(x, t, mg, c)); f has Lf
// slices, g Lg; partial holds outer_sum_parts(vh) x (Lf 4 Lg 4) entries
int outer_sum_parts(int64_t vh);
void outer_sum(hipStream_t st, Prec p, const FieldPtr& f, const FieldPtr& g, int Lf, int Lg, int64_t vh,
               double2* partial, double2* G);

}  // namespace mspcg
