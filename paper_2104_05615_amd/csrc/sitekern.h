// Site kernels shared by the full-lattice operator and the subdomain
// (preconditioner) operator: one Wilson hop (Sec. 2.2) followed by a fused
// fifth-dimension epilogue (Sec. 3.1.3).
//
// Thread mapping: a block owns `ns` output 4D sites and all Ls slices of each
// (thread = (site, s), s fastest).  The hop result of the block is staged in
// LDS as [ns][Ls][24] so that the Ls x Ls matrices of the epilogue, which mix
// the fifth dimension within one chirality, read it directly.
#pragma once

#include <type_traits>

#include "common.h"

namespace mspcg {

template <typename S> using calc_t = typename StoreTraits<S>::calc;

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Register fence between the directions of a hop: the 24 accumulators are
// final here and no later memory access moves above this point.  Without it
// the compiler overlaps all eight neighbour terms and needs every register.
template <typename T>
__device__ __forceinline__ void pin(T* acc) {
#pragma unroll
  for (int k = 0; k < 24; ++k) asm volatile("" : "+v"(acc[k]));
  asm volatile("" ::: "memory");
}

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

// load a neighbour and project it: h = (1 + SIGN gamma_mu) psi (upper half);
// returns the factor the reconstruction multiplies by (the 16-bit scale)
template <int MU, int SIGN, typename S, typename T>
__device__ __forceinline__ T load_project(const Field<S>& in, uint32_t i, T* h) {
  if constexpr (std::is_same<S, __half>::value) {
    uint4 q[3];
    const float sc = load_site_raw16(in, i, q);
    project_h<MU, SIGN>(q, h);
    return sc;
  } else {
    T psi[24];
    const T sc = load_site_unscaled(in, i, psi);
    project<MU, SIGN>(psi, h);
    return sc;
  }
}

template <int MU, int SIGN, typename S, typename T>
__device__ __forceinline__ void accumulate(const T* gh, T sc, T* acc) {
  if constexpr (StoreTraits<S>::scaled) reconstruct_fma<MU, SIGN>(gh, sc, acc);
  else reconstruct_add<MU, SIGN>(gh, acc);
}

// ---------------------------------------------------------------- full lattice

// Order in which the site blocks of a full-lattice hop are swept.  In
// lexicographic order the +-t neighbours of a block lie a whole time slice
// away, and at these volumes three slices exceed an XCD's L2, so every
// neighbour spinor of the t direction is fetched again.  The chunked order
// cuts each time slice into chunks of bzc z-planes by bb blocks of a plane
// and sweeps one chunk through all T slices before the next: the blocks in
// flight together are consecutive slices of one small chunk, and the t
// neighbours of a block were just read or are about to be.  chunk = 0 keeps
// the lexicographic order.  A block is the same set of sites in either order
// (only the order of the launch's workgroups changes), so no result depends
// on it.
struct BlockOrder {
  uint32_t chunk;      // blocks per chunk (bzc * bb); 0: lexicographic
  uint32_t bzc, bb;    // z-planes per chunk, blocks of one plane per chunk
  uint32_t bz;         // blocks per z-plane
  uint32_t bps;        // blocks per time slice
  FastDiv fchunk, fT, fbb, fnyc;   // division by chunk, T, bb and bz / bb

  __device__ __forceinline__ int64_t physical(int64_t blk) const {
    if (chunk == 0) return blk;
    const uint32_t L = (uint32_t)blk;
    const uint32_t q = fchunk.div(L), w = L - q * chunk;
    const uint32_t c = fT.div(q), t = q - c * fT.d;
    const uint32_t zl = fbb.div(w), k = w - zl * bb;
    const uint32_t zc = fnyc.div(c), yc = c - zc * fnyc.d;
    return (int64_t)t * bps + (int64_t)(zc * bzc + zl) * bz + yc * bb + k;
  }
};

template <typename T> struct FullGeo {
  Lattice lat;
  int par;        // output parity
  Gauge<T> g;
  BlockOrder order;

  __device__ __forceinline__ int64_t physical(int64_t blk) const { return order.physical(blk); }

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
    T h[12], gh[12], u[18];
    T sc = load_project<MU, SF>(in, jf * (uint32_t)Ls + (uint32_t)s, h);
    load_link(g, par, MU, site, u);
    su3_mul_half<false>(u, h, gh);
    accumulate<MU, SF, S>(gh, sc, acc);
    sc = load_project<MU, SB>(in, jb * (uint32_t)Ls + (uint32_t)s, h);
    load_link(g, 1 - par, MU, jb, u);
    su3_mul_half<true>(u, h, gh);
    accumulate<MU, SB, S>(gh, sc, acc);
  }

  template <bool DAG, typename S>
  __device__ __forceinline__ void hop(const Field<S>& in, const SiteRef& r, int s, int Ls, T* acc) const {
    int c[4];
    lat.coords(r.site, par, c);
    const uint32_t lx = lat.lex(c);
    const uint32_t site = (uint32_t)r.site;
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    // two directions between register fences: their four terms' loads are
    // in flight together (all eight at once need more registers than the
    // kernel has and spill)
    dir<0, DAG>(in, c, lx, site, s, Ls, acc);
    dir<1, DAG>(in, c, lx, site, s, Ls, acc);
    pin(acc);
    dir<2, DAG>(in, c, lx, site, s, Ls, acc);
    dir<3, DAG>(in, c, lx, site, s, Ls, acc);
  }
};

// ---------------------------------------------------------------- FP16 hop terms on MFMA
//
// The SU(3) products of a 16-bit hop run on v_mfma_f32_4x4x4f16: 16
// independent 4 x 4 x 4 blocks per wavefront, block b on lanes 4b .. 4b + 3;
// lane 4b + i holds row i of the block's A (4 K entries) and column i of its
// B (4 K entries), and receives column i of the product (4 rows).  With Ls a
// multiple of 4 and s fastest, the 4 lanes of a block are 4 fifth-dimension
// slices of one 4D site, so they share the link of every term and the guard
// of every term.
//
// Per spin of the projected half spinor (Sec. 2.2) a term is
//     g = U (psi_a + f psi_b),   f = +-1 or +-i,
// taken as a real 8 x 12 by 12 x 4 product per block: K runs over the real
// and imaginary parts of the three colours of psi_a and of f psi_b (the
// projection happens in the FP32 accumulation, so nothing is rounded to 16
// bits on the way), the rows are the real parts (first product) and the
// imaginary parts (second product) of the three output colours, and the
// columns are the block's 4 lanes.  Lane i supplies the rows of colour
// min(i, 2) (row 3 duplicates row 2 and its output is unused) and its own
// stored halves as B.  Multiplying a stored half pair by f only moves and
// negates halves, which is exact.

__device__ __forceinline__ half4_t hpair(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(half4_t, (u32x2){lo, hi});
}

__device__ __forceinline__ uint32_t swap_halves(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }

// a (re, im) half pair times f: F = 1, -1, 2 (+i) or -2 (-i)
template <int F> __device__ __forceinline__ uint32_t cmul_word(uint32_t w) {
  if constexpr (F == 1) return w;
  else if constexpr (F == -1) return w ^ 0x80008000u;
  else if constexpr (F == 2) return swap_halves(w) ^ 0x00008000u;   // (-im, re)
  else return swap_halves(w) ^ 0x80000000u;                         // (im, -re)
}

// The three stored words a lane needs of an FP16 link record: row `a` of U
// (DAG false) or column `a` (DAG true, for U^dag), one (re, im) half pair per
// entry.  An absent term (present false) reads past the array: zeros, no
// data moved.
template <bool DAG>
__device__ __forceinline__ u32x4 link_words(const Gauge<__half>& g, int parity, int mu, uint32_t site, int a,
                                            bool present) {
  const __amdgpu_buffer_rsrc_t r = make_rsrc(g.data, (uint64_t)80 * (uint64_t)g.vh * 4u);
  const uint32_t off = link_offset(g, parity, mu, site, present);
  u32x4 w;
  w.x = __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * (uint32_t)(DAG ? a : 3 * a), 0, 0);
  w.y = __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * (uint32_t)(DAG ? 3 + a : 3 * a + 1), 0, 0);
  w.z = __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * (uint32_t)(DAG ? 6 + a : 3 * a + 2), 0, 0);
  w.w = 0;
  return w;
}

// the 24 stored halves of a site as three 16-byte chunks, and its scale
__device__ __forceinline__ float load_site_v16(const Field<__half>& f, uint32_t i, u32x4& c0, u32x4& c1,
                                               u32x4& c2) {
  using C = typename Field<__half>::chunk;
  const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
  const uint32_t off = i * (uint32_t)sizeof(C);
  const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
  c0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  c1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + cs, 0, 0);
  c2 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 2 * cs, 0, 0);
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
}

// the 24 stored int8 values of a site as three 8-byte chunks, and its scale
__device__ __forceinline__ float load_site_v8(const Field<int8_t>& f, uint32_t i, u32x2& c0, u32x2& c1, u32x2& c2) {
  using C = typename Field<int8_t>::chunk;
  const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
  const uint32_t off = i * (uint32_t)sizeof(C);
  const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
  c0 = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  c1 = __builtin_amdgcn_raw_buffer_load_b64(r, off + cs, 0, 0);
  c2 = __builtin_amdgcn_raw_buffer_load_b64(r, off + 2 * cs, 0, 0);
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Eight int8 values (two words, component order) as four FP16 (re, im)
// pairs, exactly: each byte, biased to u = q + 128 in [0, 255], becomes the
// low mantissa bits of the FP16 number 1024 + u (exponent byte 0x64), and one
// packed FP16 subtraction of 1152 leaves q (integers below 2048 are exact).
__device__ __forceinline__ u32x4 i8_to_h16(u32x2 c) {
  const uint32_t x0 = c.x ^ 0x80808080u, x1 = c.y ^ 0x80808080u;
  const uint32_t e = 0x64646464u;
  // v_perm_b32 result bytes: (u_lo, 0x64, u_hi, 0x64) for bytes 0,1 and 2,3
  const uint32_t w[4] = {__builtin_amdgcn_perm(e, x0, 0x04010400u), __builtin_amdgcn_perm(e, x0, 0x04030402u),
                         __builtin_amdgcn_perm(e, x1, 0x04010400u), __builtin_amdgcn_perm(e, x1, 0x04030402u)};
  const half2_t off = {(_Float16)1152.0f, (_Float16)1152.0f};
  u32x4 r;
  r.x = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2_t, w[0]) - off);
  r.y = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2_t, w[1]) - off);
  r.z = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2_t, w[2]) - off);
  r.w = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2_t, w[3]) - off);
  return r;
}

// Those words as the A rows of the real-part (re: out.re = sum_b re_b . psi_b)
// and imaginary-part (im) outputs of colour a, one (re, im)-ordered pair per
// input colour b.
template <bool DAG>
__device__ __forceinline__ void link_rows(u32x4 lw, uint32_t* re, uint32_t* im) {
  const uint32_t w[3] = {lw.x, lw.y, lw.z};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if constexpr (!DAG) {             // U_ab:        (Re, -Im) and (Im, Re)
      re[b] = w[b] ^ 0x80000000u;
      im[b] = swap_halves(w[b]);
    } else {                          // conj(U_ba):  (Re, Im) and (-Im, Re)
      re[b] = w[b];
      im[b] = swap_halves(w[b]) ^ 0x00008000u;
    }
  }
}

// g (6 FP32: colour-major re, im) = U (u + F d) for one spin
template <int F>
__device__ __forceinline__ void spin_mfma(const uint32_t* u, const uint32_t* d, const uint32_t* xr,
                                          const uint32_t* xi, float* g) {
  const half4_t b0 = hpair(u[0], u[1]);
  const half4_t b1 = hpair(cmul_word<F>(d[0]), cmul_word<F>(d[1]));
  const half4_t b2 = hpair(u[2], cmul_word<F>(d[2]));
  const float4_t z = {0.f, 0.f, 0.f, 0.f};
  float4_t re = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xr[0], xr[1]), b0, z, 0, 0, 0);
  float4_t im = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xi[0], xi[1]), b0, z, 0, 0, 0);
  re = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xr[0], xr[1]), b1, re, 0, 0, 0);
  im = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xi[0], xi[1]), b1, im, 0, 0, 0);
  re = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xr[2], xr[2]), b2, re, 0, 0, 0);
  im = __builtin_amdgcn_mfma_f32_4x4x4f16(hpair(xi[2], xi[2]), b2, im, 0, 0, 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g[2 * c] = re[c];
    g[2 * c + 1] = im[c];
  }
}

// one hop term: acc += sc [ g ; SIGN G^dag g ], g = U h, h = (1 + SIGN gamma_mu) psi
// (the projection factors are those of project_h)
template <int MU, int SIGN, bool DAG>
__device__ __forceinline__ void term_mfma(u32x4 q0, u32x4 q1, u32x4 q2, u32x4 lw, float sc, float* acc) {
  uint32_t xr[3], xi[3];
  link_rows<DAG>(lw, xr, xi);
  const uint32_t w[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
  float gh[12];
  // spin 0 pairs with spin 3 (mu = x, y) or 2 (z, t); spin 1 with the other
  constexpr int D0 = MU < 2 ? 9 : 6, D1 = MU < 2 ? 6 : 9;
  constexpr int F0 = MU == 0 ? -2 * SIGN : MU == 1 ? -SIGN : MU == 2 ? -2 * SIGN : SIGN;
  constexpr int F1 = MU == 0 ? -2 * SIGN : MU == 1 ? SIGN : MU == 2 ? 2 * SIGN : SIGN;
  spin_mfma<F0>(w + 0, w + D0, xr, xi, gh);
  spin_mfma<F1>(w + 3, w + D1, xr, xi, gh + 6);
  reconstruct_fma<MU, SIGN>(gh, sc, acc);
}

// ---------------------------------------------------------------- subdomains
// (tables: SubTables in common.h)

// links in precision L: FP32/FP64 with the fields of that precision, FP16
// with the 16- and 8-bit formats (the paper's half-precision preconditioner
// stores its links in 16 bits too).  MW: FP16 fields with Ls a multiple of 4,
// whose SU(3) products run on MFMA blocks (term_mfma; the 8-bit format's
// integers are FP16 operands exactly).
template <typename T, typename LinkT = T, bool MW = false> struct SubGeo {
  SubTables tb;
  Lattice lat;
  int par;        // output parity (global)
  Gauge<LinkT> g;

  __device__ __forceinline__ int64_t physical(int64_t blk) const { return blk; }

  __device__ __forceinline__ SiteRef locate(int64_t blk, int sl, int ns, int Ls, int s) const {
    SiteRef r;
    r.d = (int64_t)tb.fbps.div((uint32_t)blk);   // blocks < 2^31
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
    // A neighbour outside the input region contributes nothing (the cut
    // of eq. diri).  Both terms' loads are issued without a branch (an
    // absent term reads the region's first site, a cached record, and its
    // link read falls outside the link array: zeros, no data moved) so that
    // they are in flight together; only the arithmetic is guarded.  The rim
    // of a region (two thirds of N2, one or two terms present per site) thus
    // reads no links for its absent terms.  The regions are ordered by neighbour
    // pattern, so the guard rarely diverges within a wavefront and a
    // wavefront of rim sites skips most terms.
    const int jf = nb[2 * MU], jb = nb[2 * MU + 1];
    const bool hf = jf >= 0, hb = jb >= 0;
    const int L = lat.ext(MU);
    const uint32_t st = lat.stride(MU);
    const uint32_t lb = (gco[MU] == 0) ? lx + (uint32_t)(L - 1) * st : lx - st;
    if constexpr (sizeof(T) == 8) {
      // FP64 has no registers for two terms in flight: load under the guard
      T h[12], gh[12], u[18];
      if (hf) {
        const T sc = load_project<MU, SF>(in, (base_in + (uint32_t)jf) * (uint32_t)Ls + (uint32_t)s, h);
        load_link(g, par, MU, lx >> 1, u);
        su3_mul_half<false>(u, h, gh);
        accumulate<MU, SF, S>(gh, sc, acc);
      }
      if (hb) {
        const T sc = load_project<MU, SB>(in, (base_in + (uint32_t)jb) * (uint32_t)Ls + (uint32_t)s, h);
        load_link(g, 1 - par, MU, lb >> 1, u);
        su3_mul_half<true>(u, h, gh);
        accumulate<MU, SB, S>(gh, sc, acc);
      }
      return;
    }
    const uint32_t iF = (base_in + (uint32_t)(hf ? jf : 0)) * (uint32_t)Ls + (uint32_t)s;
    const uint32_t iB = (base_in + (uint32_t)(hb ? jb : 0)) * (uint32_t)Ls + (uint32_t)s;
    if constexpr (std::is_same<S, __half>::value) {
      // FP16: the stored halves are projected under the guard too, so a rim
      // site's absent terms cost no arithmetic at all
      uint4 qF[3], qB[3];
      T uF[18], uB[18], h[12], gh[12];
      const T scF = load_site_raw16(in, iF, qF);
      load_link(g, par, MU, lx >> 1, uF, hf);
      const T scB = load_site_raw16(in, iB, qB);
      load_link(g, 1 - par, MU, lb >> 1, uB, hb);
      if (hf) {
        project_h<MU, SF>(qF, h);
        su3_mul_half<false>(uF, h, gh);
        accumulate<MU, SF, S>(gh, scF, acc);
      }
      if (hb) {
        project_h<MU, SB>(qB, h);
        su3_mul_half<true>(uB, h, gh);
        accumulate<MU, SB, S>(gh, scB, acc);
      }
      return;
    }
    T hF[12], hB[12], uF[18], uB[18], gh[12];
    // (FP32 and BF16 fields: the links of absent terms are read; cutting
    // them costs these instances registers they do not have)
    const T scF = load_project<MU, SF>(in, iF, hF);
    load_link(g, par, MU, lx >> 1, uF);
    const T scB = load_project<MU, SB>(in, iB, hB);
    load_link(g, 1 - par, MU, lb >> 1, uB);
    if (hf) {
      su3_mul_half<false>(uF, hF, gh);
      accumulate<MU, SF, S>(gh, scF, acc);
    }
    if (hb) {
      su3_mul_half<true>(uB, hB, gh);
      accumulate<MU, SB, S>(gh, scB, acc);
    }
  }

  // MFMA-term path: one direction's two terms as loaded (stored halves, the
  // lane's link words, scales, presence)
  struct Terms {
    u32x4 f0, f1, f2, b0, b1, b2;   // stored halves of the two neighbours
    u32x2 g0, g1, g2, k0, k1, k2;   // (8-bit format) stored bytes of the two neighbours
    u32x4 uF, uB;                   // the lane's link words (3 used)
    float scF, scB;
    bool hf, hb;
  };

  template <int MU, typename S>
  __device__ __forceinline__ void load_terms(const Field<S>& in, uint32_t base_in, const int* gco, uint32_t lx,
                                             const int* nb, int s, int Ls, int a, Terms& t) const {
    const int jf = nb[2 * MU], jb = nb[2 * MU + 1];
    t.hf = jf >= 0;
    t.hb = jb >= 0;
    const int L = lat.ext(MU);
    const uint32_t st = lat.stride(MU);
    const uint32_t lb = (gco[MU] == 0) ? lx + (uint32_t)(L - 1) * st : lx - st;
    const uint32_t iF = (base_in + (uint32_t)(t.hf ? jf : 0)) * (uint32_t)Ls + (uint32_t)s;
    const uint32_t iB = (base_in + (uint32_t)(t.hb ? jb : 0)) * (uint32_t)Ls + (uint32_t)s;
    if constexpr (std::is_same<S, int8_t>::value) {
      t.scF = load_site_v8(in, iF, t.g0, t.g1, t.g2);
      t.uF = link_words<false>(g, par, MU, lx >> 1, a, t.hf);
      t.scB = load_site_v8(in, iB, t.k0, t.k1, t.k2);
      t.uB = link_words<true>(g, 1 - par, MU, lb >> 1, a, t.hb);
    } else {
      t.scF = load_site_v16(in, iF, t.f0, t.f1, t.f2);
      t.uF = link_words<false>(g, par, MU, lx >> 1, a, t.hf);
      t.scB = load_site_v16(in, iB, t.b0, t.b1, t.b2);
      t.uB = link_words<true>(g, 1 - par, MU, lb >> 1, a, t.hb);
    }
  }

  template <int MU, bool DAG, typename S>
  __device__ __forceinline__ void apply_terms(const Terms& t, float* acc) const {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    if constexpr (std::is_same<S, int8_t>::value) {
      if (t.hf) term_mfma<MU, SF, false>(i8_to_h16(t.g0), i8_to_h16(t.g1), i8_to_h16(t.g2), t.uF, t.scF, acc);
      if (t.hb) term_mfma<MU, SB, true>(i8_to_h16(t.k0), i8_to_h16(t.k1), i8_to_h16(t.k2), t.uB, t.scB, acc);
    } else {
      if (t.hf) term_mfma<MU, SF, false>(t.f0, t.f1, t.f2, t.uF, t.scF, acc);
      if (t.hb) term_mfma<MU, SB, true>(t.b0, t.b1, t.b2, t.uB, t.scB, acc);
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
    if constexpr (MW) {
      static_assert((std::is_same<S, __half>::value || std::is_same<S, int8_t>::value) &&
                        std::is_same<LinkT, __half>::value, "MFMA hop terms: FP16 and 8-bit formats");
      // SU(3) products on MFMA blocks of 4 fifth-dimension slices, two
      // directions in flight: the loads of direction mu + 2 are issued
      // before the arithmetic of direction mu + 1
      const int a = min((int)(threadIdx.x & 3u), 2);
      Terms t0, t1;
      load_terms<0>(in, base_in, gco, lx, nb, s, Ls, a, t0);
      load_terms<1>(in, base_in, gco, lx, nb, s, Ls, a, t1);
      apply_terms<0, DAG, S>(t0, acc);
      pin(acc);
      load_terms<2>(in, base_in, gco, lx, nb, s, Ls, a, t0);
      apply_terms<1, DAG, S>(t1, acc);
      pin(acc);
      load_terms<3>(in, base_in, gco, lx, nb, s, Ls, a, t1);
      apply_terms<2, DAG, S>(t0, acc);
      pin(acc);
      apply_terms<3, DAG, S>(t1, acc);
      return;
    }
    dir<0, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    pin(acc);
    dir<1, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    pin(acc);
    dir<2, DAG>(in, base_in, gco, lx, nb, s, Ls, acc);
    pin(acc);
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

// ---------------------------------------------------------------- MFMA epilogue
//
// With 16 sites per block (ns = 16) and Ls <= 16 the fifth-dimension matrix
// products of a block are, per chirality chi and per component c of that
// chirality, a 16 x 16 matrix product
//     Y[s][site] = sum_t E_chi[s][t] H[t][site]      (s, t < Ls; padded to 16)
// i.e. 24 tiles of one v_mfma_f32_16x16x16_f16 (16-bit storage: operands in
// FP16, every column (site) scaled into [-1, 1] by its largest entry) or of
// four v_mfma_f32_16x16x4_f32 (FP32).  Lane l of a wavefront holds column
// l % 16 and the fifth-dimension rows 4 (l / 16) .. 4 (l / 16) + 3.

template <typename S> struct UsesMfma {
  static constexpr bool value = !std::is_same<S, double>::value;
  static constexpr bool half_ops = StoreTraits<S>::scaled;   // FP16 operands with column scales
};

// Every operand below is read at a clamped index, always inside its array,
// so that no branch guards the loads and all of them are in flight together.
// The A operands (matrix entries) are selected to zero outside the Ls x Ls
// block; the B operands need no select: rows t >= Ls meet zero A entries,
// and the clamped read returns row Ls - 1 of the same site column, a value
// that column's product reads anyway.

// A operands (the matrix) for one chirality: f16 path
__device__ __forceinline__ half4_t mfma_a16(const float* E, int chi, int Ls, int lane) {
  const int i = lane & 15, g = lane >> 4;
  const int ic = i < Ls ? i : Ls - 1;
  half4_t a;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int t = 4 * g + v;
    const float e = E[(chi * Ls + ic) * Ls + (t < Ls ? t : Ls - 1)];
    a[v] = (i < Ls && t < Ls) ? (_Float16)e : (_Float16)0.f;
  }
  return a;
}

// Per-lane LDS pointers to the B operand rows of one tile array: row
// t = 4 (lane / 16) + v of site column lane % 16, clamped to Ls - 1 (for the
// f16 path; the f32 path reads rows 4 kk + lane / 16).  Computed once, so a
// tile's reads are these pointers plus the component index.
// (element offsets into the tile: 32-bit, the tile base is uniform)
struct Rows {
  uint32_t o[4];
};
__device__ __forceinline__ Rows tile_rows(int stride, int Ls, int lane, bool f16) {
  const int col = lane & 15, g = lane >> 4;
  Rows r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int t = f16 ? 4 * g + v : 4 * v + g;
    r.o[v] = (uint32_t)(col * stride + (t < Ls ? t : Ls - 1) * 24);
  }
  return r;
}

// Tiles are taken in groups of G consecutive components (G = 4 or 2): a
// lane reads the G components of one of its rows in one LDS access (16 or 8
// bytes) and writes its G results of one row the same way.  With the site
// stride 4 x odd elements, the 8 (b128) or 16 (b64) lanes the LDS serves
// together sit in distinct site columns, on distinct banks; one component at
// a time, the 32 lanes of a half-wavefront fall on 8 banks (stride 24 rows,
// columns 8 apart on the same bank).
typedef float float2_t __attribute__((ext_vector_type(2)));
template <int G> using fgrp = typename std::conditional<G == 4, float4_t, float2_t>::type;
template <int G> using hgrp = typename std::conditional<G == 4, half4_t, half2_t>::type;

// G tiles: acc[j] += E_chi H[:, site = lane%16, component q0 + j]
template <int G>
__device__ __forceinline__ void mfma_group16(half4_t a, const float* tile, const Rows& rows, int q0, float ics,
                                             float4_t* acc) {
  half4_t b[G];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const fgrp<G> x = *reinterpret_cast<const fgrp<G>*>(tile + rows.o[v] + q0);
#pragma unroll
    for (int j = 0; j < G; ++j) b[j][v] = (_Float16)(x[j] * ics);
  }
#pragma unroll
  for (int j = 0; j < G; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b[j], acc[j], 0, 0, 0);
}

// B operand rows of an FP16 tile (the centre field of the FP16-operand
// epilogue, stored as its values over the largest one of their row)
// acc[j] += E_chi W[:, site, q0 + j] with W(t) = stored(t) x rs[t] (rs = row
// scale x column ics); rows as tile_rows(.., f16 = true) of the FP16 tile
template <int G>
__device__ __forceinline__ void mfma_group16_h(half4_t a, const _Float16* tile, const Rows& rows, int q0,
                                               const float* rs, float4_t* acc) {
  half4_t b[G];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const hgrp<G> x = *reinterpret_cast<const hgrp<G>*>(tile + rows.o[v] + q0);
#pragma unroll
    for (int j = 0; j < G; ++j) b[j][v] = (_Float16)((float)x[j] * rs[v]);
  }
#pragma unroll
  for (int j = 0; j < G; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b[j], acc[j], 0, 0, 0);
}

// A operands for one chirality: f32 path (four k-steps of 16x16x4)
struct A32 {
  float a[4];
};
__device__ __forceinline__ A32 mfma_a32(const float* E, int chi, int Ls, int lane) {
  const int col = lane & 15, g = lane >> 4;
  const int cc = col < Ls ? col : Ls - 1;
  A32 r;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int t = 4 * kk + g;
    const float e = E[(chi * Ls + cc) * Ls + (t < Ls ? t : Ls - 1)];
    r.a[kk] = (col < Ls && t < Ls) ? e : 0.f;
  }
  return r;
}

template <int G>
__device__ __forceinline__ void mfma_group32(const A32& a, const float* tile, const Rows& rows, int q0,
                                             float4_t* acc) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const fgrp<G> x = *reinterpret_cast<const fgrp<G>*>(tile + rows.o[kk] + q0);
#pragma unroll
    for (int j = 0; j < G; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.a[kk], x[j], acc[j], 0, 0, 0);
  }
}

// the G results of rows 4 (lane / 16) + v of site column lane % 16, scaled
// by the column scale cs, one G-wide store per row below Ls
template <int G>
__device__ __forceinline__ void put_group(float* dst, int stride, int Ls, int lane, int q0, const float4_t* acc,
                                          float cs) {
  const int col = lane & 15, g = lane >> 4;
  float* o = dst + col * stride + q0;
  auto row = [&](int v) {
    fgrp<G> y;
#pragma unroll
    for (int j = 0; j < G; ++j) y[j] = acc[j][v] * cs;
    *reinterpret_cast<fgrp<G>*>(o + (4 * g + v) * 24) = y;
  };
  if ((Ls & 3) == 0) {
    // Ls a multiple of 4: a lane's four rows are all valid or all beyond
    // Ls, so one branch covers every store
    if (4 * g < Ls) {
#pragma unroll
      for (int v = 0; v < 4; ++v) row(v);
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * g + v < Ls) row(v);
  }
}

// LDS layout of the site kernels:
//   red   [16] doubles            (block reduction scratch)
//   mats  [2][2][Ls][Ls] of T     (E0, E1)
//   tileA [ns][tile_stride] of T  (hop result)
//   tileB [ns][tile_stride] of T  (centre field, when E0 is dense; FP16 in the
//                                  MFMA path with FP16 operands, each row over
//                                  its largest value, kept in smaxw)
//   tileO [ns][tile_stride] of T  (MFMA path with fewer than 3 wavefronts:
//                                  epilogue result; otherwise tileA is reused)
//   smax  [ns][Ls] floats         (MFMA path with FP16 operands: column maxima)
//   smaxw [ns][Ls] floats         (same, with a centre field: row maxima of tileB)
template <typename T>
inline size_t site_lds_bytes(int ns, int Ls, bool tileB, bool mfma, bool half_ops = false) {
  size_t n = 16 * sizeof(double);
  n += sizeof(T) * (size_t)(4 * Ls * Ls);
  n += sizeof(T) * (size_t)(ns * tile_stride(Ls));
  if (tileB) n += (mfma && half_ops ? 2 : sizeof(T)) * (size_t)(ns * tile_stride(Ls));
  if (mfma) {
    const int nwave = site_block_threads(ns, Ls) / 64;
    if (nwave < 3) n += sizeof(T) * (size_t)(ns * tile_stride(Ls));
    n += sizeof(float) * (size_t)(ns * Ls);
    if (tileB && half_ops) n += sizeof(float) * (size_t)(ns * Ls);
  }
  return n;
}

// One hop with the fused epilogue
//   y = E0 w (or w if w_identity, or nothing) + E1 h (or h if E1 is null),
// and optionally one partial of Re<dotf, y> per block (the output's dot with
// a field read at the output site).  MF selects the MFMA epilogue (ns = 16).
//
// Occupancy floor: the hop is latency bound on its neighbour loads.
// (site block, RHS) work items of one hop launch, one per workgroup
struct HopWork {
  int64_t nblk;      // site blocks per RHS
  int nrhs;
  int order;         // 0: item = rhs * nblk + blk; 1: item = blk * nrhs + rhs
  int xcd;           // 1: items dealt to XCDs in contiguous ranges (xcd_block)
  const int* mask;   // RHS r skipped when mask[r] == 0 (nullable)
  FastDiv fdiv;      // division by nblk (order 0) or nrhs (order 1)
  // 32-bit arithmetic: a launch has fewer than 2^31 items
  __device__ __forceinline__ void decode(int64_t b, int64_t nb, int64_t& blk, int& rhs) const {
    const uint32_t item = (uint32_t)(xcd ? xcd_block(b, nb) : b);
    const uint32_t q = fdiv.div(item), rem = item - q * fdiv.d;
    if (order == 0) {
      rhs = (int)q;
      blk = (int64_t)rem;
    } else {
      blk = (int64_t)q;
      rhs = (int)rem;
    }
  }
};

// minimum wavefronts per SIMD the register allocation aims for
// (the FP32 full-lattice hop may take up to 168 registers for its two
// directions in flight; the compiler keeps it at four wavefronts)
template <typename G> struct IsFullF : std::false_type {};
template <> struct IsFullF<FullGeo<float>> : std::true_type {};
template <typename Geo, typename S, bool HASW> constexpr int hop_waves() {
  return sizeof(calc_t<S>) == 8 ? 2 : (IsFullF<Geo>::value && std::is_same<S, float>::value) ? 3 : 4;
}

template <typename G> struct IsSubGeo : std::false_type {};
template <typename T, typename L, bool M> struct IsSubGeo<SubGeo<T, L, M>> : std::true_type {};

template <typename Geo, typename S, bool DAG, bool HASW, bool MF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(hop_waves<Geo, S, HASW>())))
k_hop(Geo geo, Field<S> out_b, Field<S> in_b, Field<S> w_b, Field<S> dotf_b, int Ls, int ns, const calc_t<S>* E0,
      const calc_t<S>* E1, int w_identity, double* dot_partial, HopWork wk) {
  using T = calc_t<S>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* mats = reinterpret_cast<T*>(red + 16);
  T* tileA = mats + 4 * Ls * Ls;
  const bool e0_dense = HASW && !w_identity && E0 != nullptr;
  constexpr bool HOB = MF && UsesMfma<S>::half_ops;   // FP16 centre-field tile
  T* tileB = tileA + ns * tile_stride(Ls);
  _Float16* tileB16 = reinterpret_cast<_Float16*>(tileB);
  unsigned char* afterB = reinterpret_cast<unsigned char*>(tileB) +
                          (e0_dense ? (size_t)(HOB ? 2 : sizeof(T)) * ns * tile_stride(Ls) : 0);
  T* tileO = reinterpret_cast<T*>(afterB);
  float* smax = reinterpret_cast<float*>(tileO + ((blockDim.x >> 6) < 3 ? ns * tile_stride(Ls) : 0));
  float* smaxw = smax + ns * Ls;

  const int tid = threadIdx.x;
  const bool inb = tid < ns * Ls;
  const int sl = inb ? tid / Ls : 0, s = inb ? tid - sl * Ls : 0;

  const int nm = 2 * Ls * Ls;
  if constexpr (!MF) {
    for (int k = tid; k < nm; k += blockDim.x) {
      if (E0) mats[k] = E0[k];
      if (E1) mats[nm + k] = E1[k];
    }
  }
  // MFMA path (Ls <= 16, at least 16 Ls threads: at most two entries of each
  // matrix per thread): the matrices are read here, in flight with the hop's
  // loads, and written to LDS after the hop, where the epilogue reads its
  // operands with LDS latency.
  T epre[4];
  if constexpr (MF) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = min(tid + j * (int)blockDim.x, nm - 1);
      epre[j] = e0_dense ? E0[k] : (T)0;
      epre[2 + j] = E1 ? E1[k] : (T)0;
    }
  }

  int64_t blk;
  int rhs;
  wk.decode(blockIdx.x, gridDim.x, blk, rhs);
  if (wk.mask && wk.mask[rhs] == 0) return;   // uniform over the workgroup
  blk = geo.physical(blk);
  const Field<S> out = out_b.at(rhs), in = in_b.at(rhs), w = w_b.at(rhs), dotf = dotf_b.at(rhs);
  const SiteRef r = geo.locate(blk, sl, ns, Ls, s);
  const bool valid = inb && r.valid;

  T h[24], y[24];
  if (valid) geo.template hop<DAG>(in, r, s, Ls, h);
  else {
#pragma unroll
    for (int k = 0; k < 24; ++k) h[k] = 0;
  }
  T* myA = tileA + sl * tile_stride(Ls);
  T* myB = tileB + sl * tile_stride(Ls);
  if (inb) tile_put(myA, s, h);
  if constexpr (MF) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = tid + j * (int)blockDim.x;
      if (k < nm) {
        if (e0_dense) mats[k] = epre[j];
        if (E1) mats[nm + k] = epre[2 + j];
      }
    }
  }
  // centre field and the fused dot's field: on the full lattice read without
  // a branch (index 0 where there is nothing to read, then zeros selected),
  // so that their loads are in flight with the last direction of the hop and
  // with the epilogue.  FP64 keeps the branch: it has no registers to spare
  // for the overlap.  A subdomain hop's centre field covers the centre region
  // only, a small part of the output region: there a branch-free read would
  // send most lanes of the launch to one address, so only the lanes with a
  // centre site read.
  constexpr bool early = sizeof(T) == 4;
  constexpr bool early_w = early && !IsSubGeo<Geo>::value;
  T wv[24];
  bool hw = false;
  if (HASW) {
    hw = valid && r.w5 >= 0;
    if (early_w || hw) load_site(w, hw ? (uint32_t)r.w5 : 0u, wv);
#pragma unroll
    for (int k = 0; k < 24; ++k) wv[k] = hw ? wv[k] : (T)0;
    if (e0_dense && inb) {
      if constexpr (HOB) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)wv[k]));
        const float im = m > 0.f ? 1.f / m : 0.f;
        _Float16* d = tileB16 + sl * tile_stride(Ls) + s * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) d[k] = (_Float16)((float)wv[k] * im);
        smaxw[sl * Ls + s] = m;
      } else {
        tile_put(myB, s, wv);
      }
    }
  }
  T pv[24];
  // the fused dot <p, A p> belongs to the last hop of A (adjoint, with a
  // centre field): only those instances hold its field in registers
  constexpr bool DOT = DAG && HASW;
  if (DOT && early && dot_partial) load_site(dotf, valid ? (uint32_t)r.out5 : 0u, pv);

  if constexpr (MF) {
    constexpr bool HO = UsesMfma<S>::half_ops;
    if (HO && inb) {
      float m = 0.f;
#pragma unroll
      for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)h[k]));
      if (e0_dense) {
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)wv[k]));
      }
      smax[sl * Ls + s] = m;
    }
    // the centre field of a subdomain hop lives on the centre region only,
    // which the pattern order puts in the last blocks: the other blocks
    // skip its matrix product
    bool e0_live = false;
    if (e0_dense) e0_live = __syncthreads_or(hw ? 1 : 0) != 0;
    else __syncthreads();
    const int lane = tid & 63, wave = tid >> 6, nwave = (int)(blockDim.x >> 6);
    const int col = lane & 15, g = lane >> 4;
    float cs = 1.f, ics = 1.f;
    if (HO) {
      cs = 0.f;
      const float* sm = smax + col * Ls;
      if ((Ls & 3) == 0) {
        for (int t = 0; t < Ls; t += 4) cs = fmaxf(cs, fmaxf(fmaxf(sm[t], sm[t + 1]), fmaxf(sm[t + 2], sm[t + 3])));
      } else {
        for (int t = 0; t < Ls; ++t) cs = fmaxf(cs, sm[t]);
      }
      ics = cs > 0.f ? 1.f / cs : 0.f;
    }
    if (E1 || e0_dense) {
      half4_t a1[2], a0[2];
      A32 f1[2], f0[2];
#pragma unroll
      for (int chi = 0; chi < 2; ++chi) {
        if (HO) {
          if (E1) a1[chi] = mfma_a16((const float*)mats + nm, chi, Ls, lane);
          if (e0_live) a0[chi] = mfma_a16((const float*)mats, chi, Ls, lane);
        } else {
          if (E1) f1[chi] = mfma_a32((const float*)mats + nm, chi, Ls, lane);
          if (e0_live) f0[chi] = mfma_a32((const float*)mats, chi, Ls, lane);
        }
      }
      // tileA and tileB share the row layout: one set of row offsets
      const Rows rA = tile_rows(tile_stride(Ls), Ls, lane, HO);
      float rsw[4];   // centre-field rows: row maximum x column ics
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = 4 * g + v;
        rsw[v] = (HOB && e0_live) ? smaxw[col * Ls + (t < Ls ? t : Ls - 1)] * ics : 0.f;
      }
      // G tiles of one chirality starting at component q0; ra holds the
      // lane's row offsets (plus any part of q0 folded into them)
      auto group = [&](auto gc, int chi, int q0, const Rows& ra, float4_t* acc) {
        constexpr int G = decltype(gc)::value;
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
        if (HO) {
          if (E1) mfma_group16<G>(a1[chi], (const float*)tileA, ra, q0, ics, acc);
          if (e0_live) mfma_group16_h<G>(a0[chi], tileB16, ra, q0, rsw, acc);
        } else {
          if (E1) mfma_group32<G>(f1[chi], (const float*)tileA, ra, q0, acc);
          if (e0_live) mfma_group32<G>(f0[chi], (const float*)tileB, ra, q0, acc);
        }
      };
      // With three or four wavefronts each holds 8 (6) tiles in registers,
      // groups c = wave + i * NW of G = 4 (G = 2) components, then
      // overwrites the input tile once every wavefront has read it.  The
      // group sequence of a wavefront is fixed at compile time up to the
      // wavefront's own offset, so every LDS access is one base plus an
      // immediate.  Each chirality holds 12 / G groups.
      auto groups_fixed = [&](auto nwc) {
        constexpr int NW = decltype(nwc)::value;
        constexpr int G = NW == 4 ? 2 : 4;
        constexpr int NG = 24 / (G * NW);
        const int w = __builtin_amdgcn_readfirstlane(wave);
        Rows ra = rA;
#pragma unroll
        for (int v = 0; v < 4; ++v) ra.o[v] += (uint32_t)(G * w);
        float4_t accs[NG][G];
#pragma unroll
        for (int i = 0; i < NG; ++i) {
          const int q0 = G * NW * i;   // plus G * w, in ra
          const int chi = (q0 + G * w) >= 12 ? 1 : 0;
          group(std::integral_constant<int, G>(), chi, q0, ra, accs[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NG; ++i) put_group<G>(tileA, tile_stride(Ls), Ls, lane, G * (w + NW * i), accs[i], cs);
      };
      T* dst = tileA;
      if (nwave == 3) {
        groups_fixed(std::integral_constant<int, 3>());
      } else if (nwave == 4) {
        groups_fixed(std::integral_constant<int, 4>());
      } else {
        // one or two wavefronts (Ls <= 8): groups of 4 into a tile of their
        // own, one group in registers at a time
        for (int c = wave; c < 6; c += nwave) {
          float4_t acc[4];
          group(std::integral_constant<int, 4>(), c >= 3 ? 1 : 0, 4 * c, rA, acc);
          put_group<4>(tileO, tile_stride(Ls), Ls, lane, 4 * c, acc, cs);
        }
        dst = tileO;
      }
      __syncthreads();
      if (inb) {
        const T* o = dst + sl * tile_stride(Ls) + s * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) y[k] = o[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 24; ++k) y[k] = h[k];
    }
    if (HASW && w_identity) {
#pragma unroll
      for (int k = 0; k < 24; ++k) y[k] += wv[k];
    }
  } else {
    __syncthreads();
    if (inb && E1) mat5_lds(myA, mats + 2 * Ls * Ls, s, Ls, y, false);
    else {
#pragma unroll
      for (int k = 0; k < 24; ++k) y[k] = h[k];
    }
    if (HASW) {
      if (w_identity) {
#pragma unroll
        for (int k = 0; k < 24; ++k) y[k] += wv[k];
      } else if (inb && E0) {
        mat5_lds(myB, mats, s, Ls, y, true);
      }
    }
  }
  if (DOT && dot_partial) {
    T loc = 0;
    if (valid) {
      if (!early) load_site(dotf, r.out5, pv);
#pragma unroll
      for (int k = 0; k < 24; ++k) loc += pv[k] * y[k];
    }
    const double tot = block_sum((double)loc, red);
    if (tid == 0) dot_partial[(int64_t)rhs * wk.nblk + blk] = tot;
  }
  if (valid) store_site(out, r.out5, y);
}

}  // namespace mspcg
