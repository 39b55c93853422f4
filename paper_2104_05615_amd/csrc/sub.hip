// Preconditioner kernels (Sec. 2.4-2.5): moving the outer residual into the
// centre region C of every virtual subdomain and the inner solution back, and
// the inner CG's vector updates with per-subdomain scalars.  The four hops of
// the local operator A_s run through hop_sub (kernels.hip).
//
// All kernels here map threads like the site kernels: a block owns ns sites
// of C of one subdomain and all their Ls slices, so per-block partial sums are
// grouped by subdomain as [d][bps].  Batched launches put the RHS in
// blockIdx.y: fields at RHS offsets (Field::at), per-subdomain scalars at
// r * nsub, partials at r * nsub * bps; RHS with mask[r] == 0 are skipped.
#include <stdexcept>
#include <string>

#include "kernels.h"
#include "sitekern.h"

namespace mspcg {

#define LAUNCH_CHECK()                                                                \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("kernel launch: ") +   \
                                                   hipGetErrorString(e_));            \
  } while (0)

struct CSite {
  bool inb, valid;
  int sl, s;
  int64_t blk, d, j, in5;   // in5: index in the per-subdomain C field
};

__device__ __forceinline__ CSite c_site(const SubTables& tc, int ns, int Ls) {
  CSite c;
  const int tid = threadIdx.x;
  c.inb = tid < ns * Ls;
  c.sl = c.inb ? tid / Ls : 0;
  c.s = c.inb ? tid - c.sl * Ls : 0;
  c.blk = xcd_block(blockIdx.x, gridDim.x);
  c.d = (int64_t)tc.fbps.div((uint32_t)c.blk);   // blocks < 2^31
  c.j = (c.blk - c.d * tc.bps) * ns + c.sl;
  c.valid = c.inb && c.j < tc.n_out;
  c.in5 = (c.d * tc.n_out + c.j) * Ls + c.s;
  return c;
}

// global single-parity index of centre site j of subdomain d
__device__ __forceinline__ uint32_t c_global(const SubTables& tc, const Lattice& lat, int64_t d, int64_t j) {
  const short4 o = tc.origin[d];
  const short4 lc = tc.coords[j];
  // centre sites lie inside the subdomain: no wrap needed
  const int g[4] = {o.x + lc.x, o.y + lc.y, o.z + lc.z, o.w + lc.w};
  return lat.index(g);
}

template <typename O, typename I>
__global__ void __launch_bounds__(256)
k_sub_restrict(Field<O> r, Field<I> rs, Field<I> ps, Field<I> t0, const calc_t<I>* E, Lattice lat, SubTables tc,
               int Ls, int ns, double* partial, const int* mask) {
  using T = calc_t<I>;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  r = r.at(rhs);
  rs = rs.at(rhs);
  ps = ps.at(rhs);
  t0 = t0.at(rhs);
  partial += (int64_t)rhs * gridDim.x;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* mats = reinterpret_cast<T*>(red + 16);
  T* tile = mats + 2 * Ls * Ls;
  const CSite c = c_site(tc, ns, Ls);
  for (int k = threadIdx.x; k < 2 * Ls * Ls; k += blockDim.x) mats[k] = E[k];
  T v[24];
  if (c.valid) {
    const int64_t g = c_global(tc, lat, c.d, c.j);
    load_site(r, g * Ls + c.s, v);
    store_site(rs, c.in5, v);
    store_site(ps, c.in5, v);
  } else {
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
  }
  double loc = 0;
#pragma unroll
  for (int k = 0; k < 24; ++k) loc += (double)v[k] * (double)v[k];
  T* my = tile + c.sl * tile_stride(Ls);
  if (c.inb) tile_put(my, c.s, v);
  __syncthreads();
  if (c.inb) mat5_lds(my, mats, c.s, Ls, v, false);
  if (c.valid) store_site(t0, c.in5, v);
  const double tot = block_sum(loc, red);
  if (threadIdx.x == 0) partial[c.blk] = tot;
}

// The scalar a k_sub_finish of mode SUB_ALPHA or SUB_BETA would compute for
// subdomain d, evaluated in the kernel that uses it: every wavefront sums
// the bps partials in k_sub_finish's fixed order (lane-strided, then a
// butterfly), so each gets the same value to the bit without a barrier, and
// the field loads of the kernel need not wait for it.  Thread 0 of the block
// holding the subdomain's first site block also stores the new state (alpha
// or beta, rho_next, active) as k_sub_finish does.  Other wavefronts may
// read `active` while that thread clears it, but it is cleared only where
// every reader takes the same decision from the same sum; rho is read from
// one array and written to another.  Call from every lane of the wavefront.
__device__ __forceinline__ double fused_finish(const double* partial, int bps, int64_t d, bool first_blk, int mode,
                                               const double* rho, double* rho_next, double* alpha, double* beta,
                                               int* active) {
  const int lane = threadIdx.x & 63;
  double S = 0;
  for (int b = lane; b < bps; b += 64) S += partial[d * bps + b];
  for (int off = 32; off > 0; off >>= 1) S += __shfl_xor(S, off);
  const bool act = active[d] != 0;
  const bool store = first_blk && threadIdx.x == 0;
  double v;
  if (mode == SUB_ALPHA) {
    const bool ok = act && S > 0.0 && isfinite(S);
    v = ok ? rho[d] / S : 0.0;
    if (store) {
      alpha[d] = v;
      if (!ok) active[d] = 0;
    }
  } else {
    const bool ok = act && S > 0.0;
    v = ok ? S / rho[d] : 0.0;
    if (store) {
      beta[d] = v;
      rho_next[d] = ok ? S : rho[d];
      if (!ok) active[d] = 0;
    }
  }
  return v;
}

template <typename I>
__global__ void __launch_bounds__(256)
k_sub_update(Field<I> zs, Field<I> ps, Field<I> rs, Field<I> qs, SubScalars sc, int nsub, int first, int last,
             SubTables tc, int Ls, int ns, const double* pq, double* partial, const int* mask) {
  using T = calc_t<I>;
  __shared__ double red[16];
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  zs = zs.at(rhs);
  ps = ps.at(rhs);
  rs = rs.at(rhs);
  qs = qs.at(rhs);
  const int64_t so = (int64_t)rhs * nsub;
  partial += (int64_t)rhs * gridDim.x;
  const CSite c = c_site(tc, ns, Ls);
  const double alpha_d = fused_finish(pq + so * tc.bps, tc.bps, c.d, c.blk == c.d * tc.bps, SUB_ALPHA, sc.rho + so,
                                      nullptr, sc.alpha + so, nullptr, sc.active + so);
  double loc = 0;
  if (c.valid) {
    const T a = (T)alpha_d;
    T z[24], p[24];
    load_site(ps, c.in5, p);
    if (first) {
#pragma unroll
      for (int k = 0; k < 24; ++k) z[k] = a * p[k];
    } else {
      load_site(zs, c.in5, z);
#pragma unroll
      for (int k = 0; k < 24; ++k) z[k] += a * p[k];
    }
    store_site(zs, c.in5, z);
    if (!last) {
      T r[24], q[24];
      load_site(rs, c.in5, r);
      load_site(qs, c.in5, q);
#pragma unroll
      for (int k = 0; k < 24; ++k) {
        r[k] -= a * q[k];
        loc += (double)r[k] * (double)r[k];
      }
      store_site(rs, c.in5, r);
    }
  }
  const double tot = block_sum(loc, red);
  if (threadIdx.x == 0) partial[c.blk] = tot;
}

template <typename I>
__global__ void __launch_bounds__(256)
k_sub_xpay5(Field<I> ps, Field<I> rs, Field<I> t0, SubScalars sc, const double* rr, int nsub, const calc_t<I>* E,
            SubTables tc, int Ls, int ns, const int* mask) {
  using T = calc_t<I>;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  ps = ps.at(rhs);
  rs = rs.at(rhs);
  t0 = t0.at(rhs);
  const int64_t so = (int64_t)rhs * nsub;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* mats = reinterpret_cast<T*>(red + 16);
  T* tile = mats + 2 * Ls * Ls;
  const CSite c = c_site(tc, ns, Ls);
  for (int k = threadIdx.x; k < 2 * Ls * Ls; k += blockDim.x) mats[k] = E[k];
  const double beta_d = fused_finish(rr + so * tc.bps, tc.bps, c.d, c.blk == c.d * tc.bps, SUB_BETA, sc.rho + so,
                                     sc.rho_next + so, nullptr, sc.beta + so, sc.active + so);
  T p[24];
  if (c.valid) {
    const T b = (T)beta_d;
    T r[24];
    load_site(ps, c.in5, p);
    load_site(rs, c.in5, r);
#pragma unroll
    for (int k = 0; k < 24; ++k) p[k] = r[k] + b * p[k];
    store_site(ps, c.in5, p);
  } else {
#pragma unroll
    for (int k = 0; k < 24; ++k) p[k] = 0;
  }
  T* my = tile + c.sl * tile_stride(Ls);
  if (c.inb) tile_put(my, c.s, p);
  __syncthreads();
  if (c.inb) mat5_lds(my, mats, c.s, Ls, p, false);
  if (c.valid) store_site(t0, c.in5, p);
}

template <typename O, typename I>
__global__ void __launch_bounds__(256)
k_sub_prolong(Field<O> z, Field<I> zs, Field<O> r, Field<O> rold, int has_rold, Lattice lat, SubTables tc, int Ls,
              int ns, double* partial1, double* partial2, const int* mask) {
  using T = calc_t<O>;
  __shared__ double red[16];
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  z = z.at(rhs);
  zs = zs.at(rhs);
  r = r.at(rhs);
  rold = rold.at(rhs);
  partial1 += (int64_t)rhs * gridDim.x;
  if (partial2) partial2 += (int64_t)rhs * gridDim.x;
  const CSite c = c_site(tc, ns, Ls);
  double l1 = 0, l2 = 0;
  if (c.valid) {
    const int64_t g5 = c_global(tc, lat, c.d, c.j) * Ls + c.s;
    T v[24], rv[24];
    load_site(zs, c.in5, v);
    store_site(z, g5, v);
    // the dots use z as stored in the outer precision
    load_site(z, g5, v);
    load_site(r, g5, rv);
#pragma unroll
    for (int k = 0; k < 24; ++k) l1 += (double)v[k] * (double)rv[k];
    if (has_rold) {
      load_site(rold, g5, rv);
#pragma unroll
      for (int k = 0; k < 24; ++k) l2 += (double)v[k] * (double)rv[k];
    }
  }
  const double t1 = block_sum(l1, red);
  if (threadIdx.x == 0) partial1[c.blk] = t1;
  if (has_rold) {
    const double t2 = block_sum(l2, red);
    if (threadIdx.x == 0) partial2[c.blk] = t2;
  }
}

// one wavefront per subdomain: lane l sums partials l, l+64, ... in order,
// then a fixed butterfly over the 64 lanes -- deterministic
__global__ void __launch_bounds__(64)
k_sub_finish(const double* partial, int bps, int nsub, double* rho, double* alpha, double* beta, int* active,
             int mode, const int* mask) {
  const int d = blockIdx.x;
  const int lane = threadIdx.x;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const int64_t so = (int64_t)rhs * nsub;
  partial += so * bps;
  rho += so;
  alpha += so;
  beta += so;
  active += so;
  double S = 0;
  for (int b = lane; b < bps; b += 64) S += partial[(int64_t)d * bps + b];
  for (int off = 32; off > 0; off >>= 1) S += __shfl_xor(S, off);
  if (lane != 0 || d >= nsub) return;
  switch (mode) {
    case SUB_INIT:
      rho[d] = S;
      active[d] = S > 0.0 ? 1 : 0;
      alpha[d] = 0.0;
      beta[d] = 0.0;
      break;
    case SUB_ALPHA:
      if (active[d] && S > 0.0 && isfinite(S)) alpha[d] = rho[d] / S;
      else { alpha[d] = 0.0; active[d] = 0; }
      break;
    case SUB_BETA:
      if (active[d] && S > 0.0) { beta[d] = S / rho[d]; rho[d] = S; }
      else { beta[d] = 0.0; active[d] = 0; }
      break;
  }
}

// ---------------------------------------------------------------- launchers

static int c_ns(int Ls, Prec p) { return sites_per_block(Ls, p); }

static dim3 c_grid(int nsub, const SubTables& tc, const Batch& bt) {
  return dim3((unsigned)((int64_t)nsub * tc.bps), (unsigned)bt.n);
}

template <typename O, typename I>
static void restrict_t(hipStream_t st, const FieldPtr& r, const FieldPtr& rs, const FieldPtr& ps, const FieldPtr& t0,
                       const void* E, const Lattice& lat, const SubTables& tc, int nsub, int Ls, double* partial,
                       const Batch& bt) {
  using T = calc_t<I>;
  const int ns = c_ns(Ls, rs.prec);
  const size_t lds = 16 * sizeof(double) + sizeof(T) * (size_t)(2 * Ls * Ls + ns * tile_stride(Ls));
  hipLaunchKernelGGL((k_sub_restrict<O, I>), c_grid(nsub, tc, bt), dim3(site_block_threads(ns, Ls)), lds, st,
                     typed<O>(r), typed<I>(rs), typed<I>(ps), typed<I>(t0), (const T*)E, lat, tc, Ls, ns, partial,
                     bt.mask);
  LAUNCH_CHECK();
}

template <typename O>
static void restrict_o(hipStream_t st, Prec inner, const FieldPtr& r, const FieldPtr& rs, const FieldPtr& ps,
                       const FieldPtr& t0, const void* E, const Lattice& lat, const SubTables& tc, int nsub, int Ls,
                       double* partial, const Batch& bt) {
  switch (inner) {
    case Prec::F64: restrict_t<O, double>(st, r, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt); break;
    case Prec::F32: restrict_t<O, float>(st, r, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt); break;
    case Prec::F16: restrict_t<O, __half>(st, r, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt); break;
    case Prec::BF16: restrict_t<O, __hip_bfloat16>(st, r, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt); break;
    case Prec::I8: restrict_t<O, int8_t>(st, r, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt); break;
  }
}

void sub_restrict(hipStream_t st, Prec outer, Prec inner, const FieldPtr& r_outer, const FieldPtr& rs,
                  const FieldPtr& ps, const FieldPtr& t0, const void* E, const Lattice& lat, const SubTables& tc,
                  int nsub, int Ls, double* partial, const Batch& bt) {
  if (outer == Prec::F64) restrict_o<double>(st, inner, r_outer, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt);
  else if (outer == Prec::F32) restrict_o<float>(st, inner, r_outer, rs, ps, t0, E, lat, tc, nsub, Ls, partial, bt);
  else throw std::runtime_error("sub_restrict: outer precision must be FP64 or FP32");
}

template <typename I>
static void update_t(hipStream_t st, const FieldPtr& zs, const FieldPtr& ps, const FieldPtr& rs, const FieldPtr& qs,
                     const SubScalars& sc, bool first, bool last, const SubTables& tc, int nsub, int Ls,
                     const double* pq, double* partial, const Batch& bt) {
  const int ns = c_ns(Ls, zs.prec);
  hipLaunchKernelGGL((k_sub_update<I>), c_grid(nsub, tc, bt), dim3(site_block_threads(ns, Ls)), 0, st, typed<I>(zs),
                     typed<I>(ps), typed<I>(rs), typed<I>(qs), sc, nsub, first ? 1 : 0, last ? 1 : 0, tc, Ls, ns, pq,
                     partial, bt.mask);
  LAUNCH_CHECK();
}

void sub_update(hipStream_t st, Prec inner, const FieldPtr& zs, const FieldPtr& ps, const FieldPtr& rs,
                const FieldPtr& qs, const SubScalars& sc, bool first, bool last, const SubTables& tc, int nsub,
                int Ls, const double* pq, double* partial, const Batch& bt) {
  switch (inner) {
    case Prec::F64: update_t<double>(st, zs, ps, rs, qs, sc, first, last, tc, nsub, Ls, pq, partial, bt); break;
    case Prec::F32: update_t<float>(st, zs, ps, rs, qs, sc, first, last, tc, nsub, Ls, pq, partial, bt); break;
    case Prec::F16: update_t<__half>(st, zs, ps, rs, qs, sc, first, last, tc, nsub, Ls, pq, partial, bt); break;
    case Prec::BF16: update_t<__hip_bfloat16>(st, zs, ps, rs, qs, sc, first, last, tc, nsub, Ls, pq, partial, bt); break;
    case Prec::I8: update_t<int8_t>(st, zs, ps, rs, qs, sc, first, last, tc, nsub, Ls, pq, partial, bt); break;
  }
}

template <typename I>
static void xpay5_t(hipStream_t st, const FieldPtr& ps, const FieldPtr& rs, const FieldPtr& t0, const SubScalars& sc,
                    const double* rr, const void* E, const SubTables& tc, int nsub, int Ls, const Batch& bt) {
  using T = calc_t<I>;
  const int ns = c_ns(Ls, ps.prec);
  const size_t lds = 16 * sizeof(double) + sizeof(T) * (size_t)(2 * Ls * Ls + ns * tile_stride(Ls));
  hipLaunchKernelGGL((k_sub_xpay5<I>), c_grid(nsub, tc, bt), dim3(site_block_threads(ns, Ls)), lds, st, typed<I>(ps),
                     typed<I>(rs), typed<I>(t0), sc, rr, nsub, (const T*)E, tc, Ls, ns, bt.mask);
  LAUNCH_CHECK();
}

void sub_xpay5(hipStream_t st, Prec inner, const FieldPtr& ps, const FieldPtr& rs, const FieldPtr& t0,
               const SubScalars& sc, const double* rr, const void* E, const SubTables& tc, int nsub, int Ls,
               const Batch& bt) {
  switch (inner) {
    case Prec::F64: xpay5_t<double>(st, ps, rs, t0, sc, rr, E, tc, nsub, Ls, bt); break;
    case Prec::F32: xpay5_t<float>(st, ps, rs, t0, sc, rr, E, tc, nsub, Ls, bt); break;
    case Prec::F16: xpay5_t<__half>(st, ps, rs, t0, sc, rr, E, tc, nsub, Ls, bt); break;
    case Prec::BF16: xpay5_t<__hip_bfloat16>(st, ps, rs, t0, sc, rr, E, tc, nsub, Ls, bt); break;
    case Prec::I8: xpay5_t<int8_t>(st, ps, rs, t0, sc, rr, E, tc, nsub, Ls, bt); break;
  }
}

template <typename O, typename I>
static void prolong_t(hipStream_t st, const FieldPtr& z, const FieldPtr& zs, const FieldPtr& r, const FieldPtr* rold,
                      const Lattice& lat, const SubTables& tc, int nsub, int Ls, double* p1, double* p2,
                      const Batch& bt) {
  const int ns = c_ns(Ls, zs.prec);
  Field<O> ro = rold ? typed<O>(*rold) : Field<O>{};
  hipLaunchKernelGGL((k_sub_prolong<O, I>), c_grid(nsub, tc, bt), dim3(site_block_threads(ns, Ls)), 0, st,
                     typed<O>(z), typed<I>(zs), typed<O>(r), ro, rold ? 1 : 0, lat, tc, Ls, ns, p1,
                     rold ? p2 : nullptr, bt.mask);
  LAUNCH_CHECK();
}

template <typename O>
static void prolong_o(hipStream_t st, Prec inner, const FieldPtr& z, const FieldPtr& zs, const FieldPtr& r,
                      const FieldPtr* rold, const Lattice& lat, const SubTables& tc, int nsub, int Ls, double* p1,
                      double* p2, const Batch& bt) {
  switch (inner) {
    case Prec::F64: prolong_t<O, double>(st, z, zs, r, rold, lat, tc, nsub, Ls, p1, p2, bt); break;
    case Prec::F32: prolong_t<O, float>(st, z, zs, r, rold, lat, tc, nsub, Ls, p1, p2, bt); break;
    case Prec::F16: prolong_t<O, __half>(st, z, zs, r, rold, lat, tc, nsub, Ls, p1, p2, bt); break;
    case Prec::BF16: prolong_t<O, __hip_bfloat16>(st, z, zs, r, rold, lat, tc, nsub, Ls, p1, p2, bt); break;
    case Prec::I8: prolong_t<O, int8_t>(st, z, zs, r, rold, lat, tc, nsub, Ls, p1, p2, bt); break;
  }
}

void sub_prolong(hipStream_t st, Prec outer, Prec inner, const FieldPtr& z_outer, const FieldPtr& zs,
                 const FieldPtr& r_outer, const FieldPtr* rold_outer, const Lattice& lat, const SubTables& tc,
                 int nsub, int Ls, double* partial1, double* partial2, const Batch& bt) {
  if (outer == Prec::F64) prolong_o<double>(st, inner, z_outer, zs, r_outer, rold_outer, lat, tc, nsub, Ls, partial1,
                                            partial2, bt);
  else if (outer == Prec::F32) prolong_o<float>(st, inner, z_outer, zs, r_outer, rold_outer, lat, tc, nsub, Ls,
                                                partial1, partial2, bt);
  else throw std::runtime_error("sub_prolong: outer precision must be FP64 or FP32");
}

void sub_finish(hipStream_t st, const double* partial, int bps, int nsub, const SubScalars& sc, int mode,
                const Batch& bt) {
  hipLaunchKernelGGL(k_sub_finish, dim3((unsigned)nsub, (unsigned)bt.n), dim3(64), 0, st, partial, bps, nsub, sc.rho,
                     sc.alpha, sc.beta, sc.active, mode, bt.mask);
  LAUNCH_CHECK();
}

}  // namespace mspcg
