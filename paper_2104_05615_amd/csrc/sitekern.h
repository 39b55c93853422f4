// Site kernels shared by the full-lattice operator and the subdomain
// (preconditioner) operator: one Wilson hop (Sec. 2.2) followed by a fused
// fifth-dimension epilogue (Sec. 3.1.3).
//
// Thread mapping: a block owns `ns` output 4D sites and all Ls slices of each
// (thread = (site, s), s fastest).  The hop result of the block is staged in
// LDS as [ns][Ls][24] so that the Ls x Ls matrices of the epilogue, which mix
// the fifth dimension within one chirality, read it directly.
#pragma once

#include "common.h"

namespace mspcg {

template <typename S> using calc_t = typename StoreTraits<S>::calc;

// padded row stride (elements) of one site's [Ls][24] tile in LDS
__host__ __device__ inline int tile_stride(int Ls) { return Ls * 24 + 4; }

// site kernels launch whole wavefronts: ns * Ls threads do work, the rest of
// the last wavefront idles (cross-lane reductions need every lane present)
__host__ __device__ inline int site_block_threads(int ns, int Ls) { return ((ns * Ls + 63) / 64) * 64; }

struct SiteRef {
  bool valid;
  int64_t site;   // output site: full-lattice single-parity index, or region-local index
  int64_t d;      // subdomain (0 for the full lattice)
  int64_t out5;   // 5D index of the output
  int64_t w5;     // 5D index of the centre field, or -1 when it vanishes there
};

// ---------------------------------------------------------------- full lattice

template <typename T> struct FullGeo {
  Lattice lat;
  int par;        // output parity
  Gauge<T> g;

  __device__ __forceinline__ SiteRef locate(int64_t blk, int sl, int ns, int Ls, int s) const {
    SiteRef r;
    r.site = blk * ns + sl;
    r.d = 0;
    r.valid = r.site < lat.vh;
    r.out5 = r.site * Ls + s;
    r.w5 = r.out5;
    return r;
  }

  // neighbours along mu differ in lex by the stride of mu (periodic wrap)
  template <int MU, bool DAG, typename S>
  __device__ __forceinline__ void dir(const Field<S>& in, const int* c, uint32_t lx, uint32_t site, int s, int Ls,
                                      T* acc) const {
    constexpr int SF = DAG ? +1 : -1;  // (1 - gamma) forward, (1 + gamma) backward; flipped for the adjoint
    constexpr int SB = -SF;
    const int L = lat.ext(MU);
    const uint32_t st = lat.stride(MU);
    const uint32_t lf = (c[MU] + 1 == L) ? lx - (uint32_t)(L - 1) * st : lx + st;
    const uint32_t lb = (c[MU] == 0) ? lx + (uint32_t)(L - 1) * st : lx - st;
    const uint32_t jf = lf >> 1, jb = lb >> 1;
    T psi[24], h[12], gh[12], u[18];
    load_site(in, jf * (uint32_t)Ls + (uint32_t)s, psi);
    project<MU, SF>(psi, h);
    load_link(g, par, MU, site, u);
    su3_mul_half<false>(u, h, gh);
    reconstruct_add<MU, SF>(gh, acc);
    load_site(in, jb * (uint32_t)Ls + (uint32_t)s, psi);
    project<MU, SB>(psi, h);
    load_link(g, 1 - par, MU, jb, u);
    su3_mul_half<true>(u, h, gh);
    reconstruct_add<MU, SB>(gh, acc);
  }

  template <bool DAG, typename S>
  __device__ __forceinline__ void hop(const Field<S>& in, const SiteRef& r, int s, int Ls, T* acc) const {
    int c[4];
    lat.coords(r.site, par, c);
    const uint32_t lx = lat.lex(c);
    const uint32_t site = (uint32_t)r.site;
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    dir<0, DAG>(in, c, lx, site, s, Ls, acc);
    dir<1, DAG>(in, c, lx, site, s, Ls, acc);
    dir<2, DAG>(in, c, lx, site, s, Ls, acc);
    dir<3, DAG>(in, c, lx, site, s, Ls, acc);
  }
};

// ---------------------------------------------------------------- subdomains
// (tables: SubTables in common.h)

template <typename T> struct SubGeo {
  SubTables tb;
  Lattice lat;
  int par;        // output parity (global)
  Gauge<T> g;

  __device__ __forceinline__ SiteRef locate(int64_t blk, int sl, int ns, int Ls, int s) const {
    SiteRef r;
    r.d = blk / tb.bps;
    const int64_t b = blk - r.d * tb.bps;
    r.site = b * ns + sl;
    r.valid = r.site < tb.n_out;
    r.out5 = (r.d * tb.n_out + r.site) * Ls + s;
    if (tb.wmap == nullptr) r.w5 = r.out5;
    else {
      const int m = r.valid ? tb.wmap[r.site] : -1;
      r.w5 = m >= 0 ? (r.d * tb.n_w + m) * Ls + s : -1;
    }
    return r;
  }

  template <int MU, bool DAG, typename S>
  __device__ __forceinline__ void dir(const Field<S>& in, uint32_t base_in, const int* gco, uint32_t lx,
                                      const int* nb, int s, int Ls, T* acc) const {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    T psi[24], h[12], gh[12], u[18];
    const int jf = nb[2 * MU], jb = nb[2 * MU + 1];
    if (jf >= 0) {
      load_site(in, (base_in + (uint32_t)jf) * (uint32_t)Ls + (uint32_t)s, psi);
      project<MU, SF>(psi, h);
      load_link(g, par, MU, lx >> 1, u);
      su3_mul_half<false>(u, h, gh);
      reconstruct_add<MU, SF>(gh, acc);
    }
    if (jb >= 0) {
      const int L = lat.ext(MU);
      const uint32_t st = lat.stride(MU);
      const uint32_t lb = (gco[MU] == 0) ? lx + (uint32_t)(L - 1) * st : lx - st;
      load_site(in, (base_in + (uint32_t)jb) * (uint32_t)Ls + (uint32_t)s, psi);
      project<MU, SB>(psi, h);
      load_link(g, 1 - par, MU, lb >> 1, u);
      su3_mul_half<true>(u, h, gh);
      reconstruct_add<MU, SB>(gh, acc);
    }
  }

  template <bool DAG, typename S>
  __device__ __forceinline__ void hop(const Field<S>& in, const SiteRef& r, int s, int Ls, T* acc) const {
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    const short4 o = tb.origin[r.d];          // uniform over the block
    const short4 lc = tb.coords[r.site];
    const int l[4] = {o.x + lc.x, o.y + lc.y, o.z + lc.z, o.w + lc.w};
    int gco[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int v = l[m];
      if (v < 0) v += tb.dims[m];
      if (v >= tb.dims[m]) v -= tb.dims[m];
      gco[m] = v;
    }
    const uint32_t lx = lat.lex(gco);
    const int4 n0 = reinterpret_cast<const int4*>(tb.nbr)[2 * r.site];
    const int4 n1 = reinterpret_cast<const int4*>(tb.nbr)[2 * r.site + 1];
    const int nb[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
    const uint32_t base_in = (uint32_t)r.d * (uint32_t)tb.n_in;
    dir<0, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    dir<1, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    dir<2, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    dir<3, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
  }
};

// ---------------------------------------------------------------- epilogue helpers

// y(s) (+)= E[chi][s][t] v(t) over an LDS tile [Ls][24]
template <typename T>
__device__ __forceinline__ void mat5_lds(const T* tile, const T* E, int s, int Ls, T* y, bool acc) {
  T r[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) r[k] = acc ? y[k] : (T)0;
  const T* Ep = E + s * Ls;
  const T* Em = E + Ls * Ls + s * Ls;
  for (int t = 0; t < Ls; ++t) {
    const T ep = Ep[t], em = Em[t];
    const T* v = tile + t * 24;
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] += ep * v[k];
#pragma unroll
    for (int k = 12; k < 24; ++k) r[k] += em * v[k];
  }
#pragma unroll
  for (int k = 0; k < 24; ++k) y[k] = r[k];
}

template <typename T>
__device__ __forceinline__ void tile_put(T* tile, int s, const T* v) {
#pragma unroll
  for (int k = 0; k < 24; ++k) tile[s * 24 + k] = v[k];
}

// block-wide sum of a double (fixed order: deterministic).  Result valid on
// thread 0.  Contains a barrier: call from every thread of the block.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double tot = 0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) tot += red[i];
  }
  __syncthreads();
  return tot;
}

// LDS layout of the site kernels:
//   red   [16] doubles            (block reduction scratch)
//   mats  [3][2][Ls][Ls] of T     (E0, E1, E2)
//   tileA [ns][tile_stride] of T  (hop result / second-stage input)
//   tileB [ns][tile_stride] of T  (centre field; only when E0 is dense)
template <typename T>
inline size_t site_lds_bytes(int ns, int Ls, bool tileB) {
  return 16 * sizeof(double) + sizeof(T) * (size_t)(6 * Ls * Ls + (tileB ? 2 : 1) * ns * tile_stride(Ls));
}

// One hop with the fused epilogue
//   y = E0 w (or w if w_identity) + E1 h (or h), out = E2 y (or y),
// and optionally one |y|^2 partial per block.
template <typename Geo, typename S, bool DAG, bool HASW>
__global__ void __launch_bounds__(256)
k_hop(Geo geo, Field<S> out, Field<S> in, Field<S> w, int Ls, int ns, const calc_t<S>* E0, const calc_t<S>* E1,
      const calc_t<S>* E2, int w_identity, double* norm_partial) {
  using T = calc_t<S>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* mats = reinterpret_cast<T*>(red + 16);
  T* tileA = mats + 6 * Ls * Ls;
  T* tileB = tileA + ns * tile_stride(Ls);

  const int tid = threadIdx.x;
  const bool inb = tid < ns * Ls;
  const int sl = inb ? tid / Ls : 0, s = inb ? tid - sl * Ls : 0;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const SiteRef r = geo.locate(blk, sl, ns, Ls, s);
  const bool valid = inb && r.valid;

  const int nm = 2 * Ls * Ls;
  for (int k = tid; k < nm; k += blockDim.x) {
    if (E0) mats[k] = E0[k];
    if (E1) mats[nm + k] = E1[k];
    if (E2) mats[2 * nm + k] = E2[k];
  }

  T h[24], y[24];
  if (valid) geo.template hop<DAG>(in, r, s, Ls, h);
  else {
#pragma unroll
    for (int k = 0; k < 24; ++k) h[k] = 0;
  }
  T* myA = tileA + sl * tile_stride(Ls);
  T* myB = tileB + sl * tile_stride(Ls);
  if (inb) tile_put(myA, s, h);
  T wv[24];
  if (HASW) {
    if (valid && r.w5 >= 0) load_site(w, r.w5, wv);
    else {
#pragma unroll
      for (int k = 0; k < 24; ++k) wv[k] = 0;
    }
    if (!w_identity && inb) tile_put(myB, s, wv);
  }
  __syncthreads();
  if (inb && E1) mat5_lds(myA, mats + nm, s, Ls, y, false);
  else {
#pragma unroll
    for (int k = 0; k < 24; ++k) y[k] = h[k];
  }
  if (HASW) {
    if (w_identity) {
#pragma unroll
      for (int k = 0; k < 24; ++k) y[k] += wv[k];
    } else if (inb) {
      mat5_lds(myB, mats, s, Ls, y, true);
    }
  }
  if (norm_partial) {
    T loc = 0;
    if (valid) {
#pragma unroll
      for (int k = 0; k < 24; ++k) loc += y[k] * y[k];
    }
    const double tot = block_sum((double)loc, red);
    if (tid == 0) norm_partial[blk] = tot;
  }
  if (E2) {
    __syncthreads();
    if (inb) tile_put(myA, s, y);
    __syncthreads();
    if (inb) mat5_lds(myA, mats + 2 * nm, s, Ls, y, false);
  }
  if (valid) store_site(out, r.out5, y);
}

}  // namespace mspcg
