// Device-side building blocks shared by the library's kernels: storage
// formats of single-parity 5D fields and gauge links, the spin projection of
// the Wilson hopping term in the chiral gamma basis, SU(3) products and the
// XCD-aware block remap.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace mspcg {

// --------------------------------------------------------------------------
// storage formats
//
// A single-parity 5D field holds n5 = nsites * Ls sites, s fastest
// (index = site * Ls + s).  The 24 reals of a site (spin-major, then colour,
// then re/im) are split into fixed-width chunks stored as separate arrays of
// length `stride` so that a wavefront loads each chunk fully coalesced:
//   FP64: 12 chunks of one complex (double2)
//   FP32:  6 chunks of two complex (float4)
//   FP16/BF16: 3 chunks of four complex (8 x 16-bit = 16 bytes), plus one
//   FP32 scale per 5D site: value = stored * scale, scale = max |component|.
// Chirality: spins 0,1 (components 0..11) are P+, spins 2,3 are P-.
// --------------------------------------------------------------------------

struct half8 { __half2 h[4]; };
struct bf16x8 { __hip_bfloat162 h[4]; };

template <typename S> struct StoreTraits;
template <> struct StoreTraits<double> {
  using chunk = double2; static constexpr int nchunk = 12; using calc = double; static constexpr bool scaled = false;
};
template <> struct StoreTraits<float> {
  using chunk = float4; static constexpr int nchunk = 6; using calc = float; static constexpr bool scaled = false;
};
template <> struct StoreTraits<__half> {
  using chunk = uint4; static constexpr int nchunk = 3; using calc = float; static constexpr bool scaled = true;
};
template <> struct StoreTraits<__hip_bfloat16> {
  using chunk = uint4; static constexpr int nchunk = 3; using calc = float; static constexpr bool scaled = true;
};

template <typename S> struct Field {
  using chunk = typename StoreTraits<S>::chunk;
  chunk* data;     // nchunk arrays of `stride` chunks
  float* scale;    // 16-bit formats only
  int64_t stride;
};

template <typename S> __device__ __forceinline__ void unpack8(const uint4& c, float* v);
template <> __device__ __forceinline__ void unpack8<__half>(const uint4& c, float* v) {
  const __half2* h = reinterpret_cast<const __half2*>(&c);
#pragma unroll
  for (int j = 0; j < 4; ++j) { float2 f = __half22float2(h[j]); v[2 * j] = f.x; v[2 * j + 1] = f.y; }
}
template <> __device__ __forceinline__ void unpack8<__hip_bfloat16>(const uint4& c, float* v) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(&c);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[2 * j] = __uint_as_float(w[j] << 16);
    v[2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
  }
}

// round-to-nearest-even conversion of a float already scaled into [-1, 1]
__device__ __forceinline__ uint32_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <typename S> __device__ __forceinline__ uint4 pack8(const float* v);
template <> __device__ __forceinline__ uint4 pack8<__half>(const float* v) {
  uint4 c;
  __half2* h = reinterpret_cast<__half2*>(&c);
#pragma unroll
  for (int j = 0; j < 4; ++j) h[j] = __floats2half2_rn(v[2 * j], v[2 * j + 1]);
  return c;
}
template <> __device__ __forceinline__ uint4 pack8<__hip_bfloat16>(const float* v) {
  uint4 c;
  uint32_t* w = reinterpret_cast<uint32_t*>(&c);
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = f2bf_rne(v[2 * j]) | (f2bf_rne(v[2 * j + 1]) << 16);
  return c;
}

template <typename S, typename T>
__device__ __forceinline__ void load_site(const Field<S>& f, int64_t i, T* v) {
  if constexpr (sizeof(S) == 8) {
#pragma unroll
    for (int k = 0; k < 12; ++k) { double2 c = f.data[k * f.stride + i]; v[2 * k] = c.x; v[2 * k + 1] = c.y; }
  } else if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 c = f.data[k * f.stride + i];
      v[4 * k] = c.x; v[4 * k + 1] = c.y; v[4 * k + 2] = c.z; v[4 * k + 3] = c.w;
    }
  } else {
    const float sc = f.scale[i];
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 3; ++k) unpack8<S>(f.data[k * f.stride + i], tmp + 8 * k);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = tmp[k] * sc;
  }
}

template <typename S, typename T>
__device__ __forceinline__ void store_site(const Field<S>& f, int64_t i, const T* v) {
  if constexpr (sizeof(S) == 8) {
#pragma unroll
    for (int k = 0; k < 12; ++k) f.data[k * f.stride + i] = make_double2(v[2 * k], v[2 * k + 1]);
  } else if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      f.data[k * f.stride + i] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  } else {
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) mx = fmaxf(mx, fabsf((float)v[k]));
    const float inv = mx > 0.f ? 1.0f / mx : 0.f;
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) tmp[k] = (float)v[k] * inv;
#pragma unroll
    for (int k = 0; k < 3; ++k) f.data[k * f.stride + i] = pack8<S>(tmp + 8 * k);
    f.scale[i] = mx;
  }
}

// --------------------------------------------------------------------------
// gauge links: per parity, per direction, 9 complex entries (row-major) as
// separate arrays of length vh:  U[parity][mu][entry][vh] of complex L2.
// --------------------------------------------------------------------------
template <typename L> struct Gauge {
  using c2 = typename std::conditional<sizeof(L) == 8, double2, float2>::type;
  const c2* data;
  int64_t vh;
  __device__ __forceinline__ const c2* link(int parity, int mu, int64_t site) const {
    return data + ((int64_t)(parity * 4 + mu) * 9) * vh + site;
  }
};

template <typename L, typename T>
__device__ __forceinline__ void load_link(const Gauge<L>& g, int parity, int mu, int64_t site, T* u) {
  const auto* p = g.link(parity, mu, site);
#pragma unroll
  for (int k = 0; k < 9; ++k) { auto c = p[k * g.vh]; u[2 * k] = (T)c.x; u[2 * k + 1] = (T)c.y; }
}

// --------------------------------------------------------------------------
// half-spinor projection in the chiral basis
//
// gamma_mu = [[0, G_mu], [G_mu^dag, 0]] with G_k = -i sigma_k (k = x, y, z)
// and G_t = 1.  For sign s = +-1,
//   (1 + s gamma_mu) psi = [ h ; s G_mu^dag h ],  h = psi_up + s G_mu psi_dn,
// so one hop needs the SU(3) product on the two spins of h only.
// psi index: ((spin * 3 + colour) * 2 + re/im).
// --------------------------------------------------------------------------

template <typename T> struct cplx { T re, im; };

template <int MU, int SIGN, typename T>
__device__ __forceinline__ void project(const T* p, T* h) {
  // h[(sp*3 + c)*2 + ri], sp = 0, 1
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T u0r = p[(0 * 3 + c) * 2], u0i = p[(0 * 3 + c) * 2 + 1];
    const T u1r = p[(1 * 3 + c) * 2], u1i = p[(1 * 3 + c) * 2 + 1];
    const T d2r = p[(2 * 3 + c) * 2], d2i = p[(2 * 3 + c) * 2 + 1];
    const T d3r = p[(3 * 3 + c) * 2], d3i = p[(3 * 3 + c) * 2 + 1];
    T h0r, h0i, h1r, h1i;
    if constexpr (MU == 0) {        // G psi_dn = (-i d3, -i d2)
      h0r = u0r + SIGN * d3i; h0i = u0i - SIGN * d3r;
      h1r = u1r + SIGN * d2i; h1i = u1i - SIGN * d2r;
    } else if constexpr (MU == 1) { // G psi_dn = (-d3, d2)
      h0r = u0r - SIGN * d3r; h0i = u0i - SIGN * d3i;
      h1r = u1r + SIGN * d2r; h1i = u1i + SIGN * d2i;
    } else if constexpr (MU == 2) { // G psi_dn = (-i d2, i d3)
      h0r = u0r + SIGN * d2i; h0i = u0i - SIGN * d2r;
      h1r = u1r - SIGN * d3i; h1i = u1i + SIGN * d3r;
    } else {                        // G psi_dn = (d2, d3)
      h0r = u0r + SIGN * d2r; h0i = u0i + SIGN * d2i;
      h1r = u1r + SIGN * d3r; h1i = u1i + SIGN * d3i;
    }
    h[(0 * 3 + c) * 2] = h0r; h[(0 * 3 + c) * 2 + 1] = h0i;
    h[(1 * 3 + c) * 2] = h1r; h[(1 * 3 + c) * 2 + 1] = h1i;
  }
}

// acc += [ g ; s G^dag g ] for the SU(3)-multiplied half spinor g
template <int MU, int SIGN, typename T>
__device__ __forceinline__ void reconstruct_add(const T* g, T* acc) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T g0r = g[(0 * 3 + c) * 2], g0i = g[(0 * 3 + c) * 2 + 1];
    const T g1r = g[(1 * 3 + c) * 2], g1i = g[(1 * 3 + c) * 2 + 1];
    acc[(0 * 3 + c) * 2] += g0r; acc[(0 * 3 + c) * 2 + 1] += g0i;
    acc[(1 * 3 + c) * 2] += g1r; acc[(1 * 3 + c) * 2 + 1] += g1i;
    T l0r, l0i, l1r, l1i;
    if constexpr (MU == 0) {        // G^dag g = (i g1, i g0)
      l0r = -g1i; l0i = g1r; l1r = -g0i; l1i = g0r;
    } else if constexpr (MU == 1) { // G^dag g = (g1, -g0)
      l0r = g1r; l0i = g1i; l1r = -g0r; l1i = -g0i;
    } else if constexpr (MU == 2) { // G^dag g = (i g0, -i g1)
      l0r = -g0i; l0i = g0r; l1r = g1i; l1i = -g1r;
    } else {                        // G^dag g = (g0, g1)
      l0r = g0r; l0i = g0i; l1r = g1r; l1i = g1i;
    }
    acc[(2 * 3 + c) * 2] += SIGN * l0r; acc[(2 * 3 + c) * 2 + 1] += SIGN * l0i;
    acc[(3 * 3 + c) * 2] += SIGN * l1r; acc[(3 * 3 + c) * 2 + 1] += SIGN * l1i;
  }
}

// g = U h (DAG = false) or U^dag h (DAG = true), for the two spins of h
template <bool DAG, typename T>
__device__ __forceinline__ void su3_mul_half(const T* u, const T* h, T* g) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T re = 0, im = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int k = DAG ? (b * 3 + a) : (a * 3 + b);
        const T ur = u[2 * k], ui = DAG ? -u[2 * k + 1] : u[2 * k + 1];
        const T hr = h[(sp * 3 + b) * 2], hi = h[(sp * 3 + b) * 2 + 1];
        re += ur * hr - ui * hi;
        im += ur * hi + ui * hr;
      }
      g[(sp * 3 + a) * 2] = re;
      g[(sp * 3 + a) * 2 + 1] = im;
    }
  }
}

// --------------------------------------------------------------------------
// XCD-aware block order.  Workgroups are dispatched to the 8 XCDs round
// robin (block b on XCD b % 8); each XCD has its own L2.  Remap so that XCD k
// processes one contiguous range of logical blocks and neighbouring tiles
// share an L2.
// --------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  const int64_t k = b & 7, j = b >> 3;
  return (k < r) ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j;
}

// --------------------------------------------------------------------------
// lattice geometry of one parity (single-parity index = lex / 2)
// --------------------------------------------------------------------------
struct Lattice {
  int X, Y, Z, T;
  int64_t vh;
  __device__ __forceinline__ void coords(int64_t i, int parity, int* c) const {
    const int64_t l0 = 2 * i;
    const int x0 = (int)(l0 % X);
    const int64_t r = l0 / X;
    c[1] = (int)(r % Y);
    const int64_t r2 = r / Y;
    c[2] = (int)(r2 % Z);
    c[3] = (int)(r2 / Z);
    c[0] = x0 + ((c[1] + c[2] + c[3] + parity) & 1);
  }
  __device__ __forceinline__ int64_t index(const int* c) const {
    return ((int64_t)c[0] + (int64_t)X * ((int64_t)c[1] + (int64_t)Y * ((int64_t)c[2] + (int64_t)Z * c[3]))) >> 1;
  }
  __device__ __forceinline__ int ext(int mu) const { return mu == 0 ? X : mu == 1 ? Y : mu == 2 ? Z : T; }
};

// --------------------------------------------------------------------------
// subdomain region tables
//
// Every subdomain has the same local geometry (a translate of subdomain 0),
// so one set of region tables serves all of them.  Local coordinates run over
// [-2, sub + 2) in partitioned directions and [0, L) in the others; a region
// is the set of sites of one parity within L1 distance 0, 1 or 2 of the
// subdomain (C, N1, N2).  nbr[j][2 mu + dir] is the index of the neighbour
// (dir 0: +mu, 1: -mu) in the input region of the hop, or -1 if the input
// vanishes there (outside the region: zero Dirichlet pad).
struct SubTables {
  const short4* coords;   // [n_out] local coordinates of the output sites
  const int* nbr;         // [n_out][8]
  const int* wmap;        // [n_out] index into the centre-field region, -1 = zero; null = same region
  int n_out, n_in, n_w;
  int bps;                // blocks per subdomain
  int sub[4], dims[4], nblk[4];
};

}  // namespace mspcg
