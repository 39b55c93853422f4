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

// 8-bit fixed point: a site's 24 reals as int8 in [-127, 127] (three 8-byte
// chunks) times one FP32 scale (the largest magnitude / 127)
template <> struct StoreTraits<int8_t> {
  using chunk = uint2; static constexpr int nchunk = 3; using calc = float; static constexpr bool scaled = true;
};

template <typename S> struct Field {
  using chunk = typename StoreTraits<S>::chunk;
  chunk* data;     // nchunk arrays of `stride` chunks
  float* scale;    // scaled formats (16- and 8-bit) only
  int64_t stride;
  // right-hand side r of a batch stored one whole field after another
  __device__ __forceinline__ Field at(int r) const {
    Field f = *this;
    if (data) f.data += (int64_t)r * StoreTraits<S>::nchunk * stride;
    if (scale) f.scale += (int64_t)r * stride;
    return f;
  }
};

// 16-bit values are taken from and put into 32-bit words with shifts only:
// no pointer type punning between the vector word types and __half.
__device__ __forceinline__ uint32_t word(const uint4& c, int j) {
  return j == 0 ? c.x : j == 1 ? c.y : j == 2 ? c.z : c.w;
}
__device__ __forceinline__ float half_lo(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ __forceinline__ float half_hi(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

// eight int8 values of a 64-bit chunk, sign-extended with shifts
__device__ __forceinline__ void unpack8_i8(const uint2& c, float* v) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t w = k < 4 ? c.x : c.y;
    const int sh = 8 * (k & 3);
    v[k] = (float)(((int)(w << (24 - sh))) >> 24);
  }
}
// eight values in [-127.5, 127.5] rounded to int8
__device__ __forceinline__ uint2 pack8_i8(const float* v) {
  uint32_t w[2] = {0u, 0u};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int q = __float2int_rn(v[k]);
    q = q > 127 ? 127 : (q < -127 ? -127 : q);
    w[k >> 2] |= ((uint32_t)q & 0xffu) << (8 * (k & 3));
  }
  return make_uint2(w[0], w[1]);
}

template <typename S> __device__ __forceinline__ void unpack8(const uint4& c, float* v);
template <> __device__ __forceinline__ void unpack8<__half>(const uint4& c, float* v) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t w = word(c, j);
    v[2 * j] = half_lo(w);
    v[2 * j + 1] = half_hi(w);
  }
}
template <> __device__ __forceinline__ void unpack8<__hip_bfloat16>(const uint4& c, float* v) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t w = word(c, j);
    v[2 * j] = __uint_as_float(w << 16);
    v[2 * j + 1] = __uint_as_float(w & 0xffff0000u);
  }
}

// round-to-nearest-even conversion of a float already scaled into [-1, 1]
__device__ __forceinline__ uint32_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ uint32_t f2h_bits(float f) { return (uint32_t)__half_as_ushort(__float2half_rn(f)); }

template <typename S> __device__ __forceinline__ uint4 pack8(const float* v);
template <> __device__ __forceinline__ uint4 pack8<__half>(const float* v) {
  uint4 c;
  c.x = f2h_bits(v[0]) | (f2h_bits(v[1]) << 16);
  c.y = f2h_bits(v[2]) | (f2h_bits(v[3]) << 16);
  c.z = f2h_bits(v[4]) | (f2h_bits(v[5]) << 16);
  c.w = f2h_bits(v[6]) | (f2h_bits(v[7]) << 16);
  return c;
}
template <> __device__ __forceinline__ uint4 pack8<__hip_bfloat16>(const float* v) {
  uint4 c;
  c.x = f2bf_rne(v[0]) | (f2bf_rne(v[1]) << 16);
  c.y = f2bf_rne(v[2]) | (f2bf_rne(v[3]) << 16);
  c.z = f2bf_rne(v[4]) | (f2bf_rne(v[5]) << 16);
  c.w = f2bf_rne(v[6]) | (f2bf_rne(v[7]) << 16);
  return c;
}

// Site access through raw buffer instructions: one 128-bit resource per
// field (scalar registers) and the byte offset of the site's chunk in a
// vector register.  The scalar-offset operand is always 0: with the chunk
// array's offset passed there, results of the subdomain kernels changed
// from run to run on gfx950 when other kernels ran on the device at the same
// time (vector offsets alone are reproducible).  A field must be smaller
// than 4 GiB (checked on the host).  Accesses past the resource's range read
// zero and drop stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kBufferConfig = 0x00020000;   // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(uint32_t)bytes, kBufferConfig);
}

template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const Field<S>& f) {
  using C = typename Field<S>::chunk;
  return make_rsrc(f.data, (uint64_t)StoreTraits<S>::nchunk * (uint64_t)f.stride * sizeof(C));
}

template <typename S, typename T>
__device__ __forceinline__ void load_site(const Field<S>& f, uint32_t i, T* v) {
  using C = typename Field<S>::chunk;
  const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
  const uint32_t off = i * (uint32_t)sizeof(C);
  const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
  if constexpr (sizeof(S) == 8) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * cs, 0, 0);
      v[2 * k] = __hiloint2double(c.y, c.x);
      v[2 * k + 1] = __hiloint2double(c.w, c.z);
    }
  } else if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * cs, 0, 0);
      v[4 * k] = __uint_as_float(c.x); v[4 * k + 1] = __uint_as_float(c.y);
      v[4 * k + 2] = __uint_as_float(c.z); v[4 * k + 3] = __uint_as_float(c.w);
    }
  } else if constexpr (std::is_same<S, int8_t>::value) {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    const float sc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(r, off + k * cs, 0, 0);
      unpack8_i8(make_uint2(c.x, c.y), tmp + 8 * k);
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = tmp[k] * sc;
  } else {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    const float sc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * cs, 0, 0);
      uint4 q;
      q.x = c.x; q.y = c.y; q.z = c.z; q.w = c.w;
      unpack8<S>(q, tmp + 8 * k);
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = tmp[k] * sc;
  }
}

template <typename S, typename T>
__device__ __forceinline__ void store_site(const Field<S>& f, uint32_t i, const T* v) {
  using C = typename Field<S>::chunk;
  const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
  const uint32_t off = i * (uint32_t)sizeof(C);
  const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
  if constexpr (sizeof(S) == 8) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      u32x4 c;
      const double a = (double)v[2 * k], b = (double)v[2 * k + 1];
      c.x = (uint32_t)__double2loint(a); c.y = (uint32_t)__double2hiint(a);
      c.z = (uint32_t)__double2loint(b); c.w = (uint32_t)__double2hiint(b);
      __builtin_amdgcn_raw_buffer_store_b128(c, r, off + k * cs, 0, 0);
    }
  } else if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      u32x4 c;
      c.x = __float_as_uint((float)v[4 * k]); c.y = __float_as_uint((float)v[4 * k + 1]);
      c.z = __float_as_uint((float)v[4 * k + 2]); c.w = __float_as_uint((float)v[4 * k + 3]);
      __builtin_amdgcn_raw_buffer_store_b128(c, r, off + k * cs, 0, 0);
    }
  } else if constexpr (std::is_same<S, int8_t>::value) {
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) mx = fmaxf(mx, fabsf((float)v[k]));
    const float inv = mx > 0.f ? 127.0f / mx : 0.f;
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) tmp[k] = (float)v[k] * inv;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint2 q = pack8_i8(tmp + 8 * k);
      u32x2 c;
      c.x = q.x; c.y = q.y;
      __builtin_amdgcn_raw_buffer_store_b64(c, r, off + k * cs, 0, 0);
    }
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(mx * (1.0f / 127.0f)), rs, i * 4u, 0, 0);
  } else {
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) mx = fmaxf(mx, fabsf((float)v[k]));
    const float inv = mx > 0.f ? 1.0f / mx : 0.f;
    float tmp[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) tmp[k] = (float)v[k] * inv;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint4 q = pack8<S>(tmp + 8 * k);
      u32x4 c;
      c.x = q.x; c.y = q.y; c.z = q.z; c.w = q.w;
      __builtin_amdgcn_raw_buffer_store_b128(c, r, off + k * cs, 0, 0);
    }
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(mx), rs, i * 4u, 0, 0);
  }
}

// As load_site, but the scaled formats return the stored values without their
// scale, which is returned instead (1 for FP32/FP64): a hop is linear, so
// the scale is applied once, in the final accumulate.
template <typename S, typename T>
__device__ __forceinline__ T load_site_unscaled(const Field<S>& f, uint32_t i, T* v) {
  if constexpr (!StoreTraits<S>::scaled) {
    load_site(f, i, v);
    return (T)1;
  } else if constexpr (std::is_same<S, int8_t>::value) {
    using C = typename Field<S>::chunk;
    const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
    const uint32_t off = i * (uint32_t)sizeof(C);
    const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    const float sc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(r, off + k * cs, 0, 0);
      unpack8_i8(make_uint2(c.x, c.y), v + 8 * k);
    }
    return sc;
  } else {
    using C = typename Field<S>::chunk;
    const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
    const uint32_t off = i * (uint32_t)sizeof(C);
    const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
    const float sc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * cs, 0, 0);
      uint4 q;
      q.x = c.x; q.y = c.y; q.z = c.z; q.w = c.w;
      unpack8<S>(q, v + 8 * k);
    }
    return sc;
  }
}

// --------------------------------------------------------------------------
// gauge links: per parity, per direction, per site one record of the 9
// complex entries (row-major) padded to 10, so that a link is read with
// 16-byte loads:  U[parity][mu][vh][10] of complex L2.
// --------------------------------------------------------------------------
template <typename L> struct Gauge {
  using c2 = typename std::conditional<
      sizeof(L) == 8, double2, typename std::conditional<sizeof(L) == 4, float2, __half2>::type>::type;
  const c2* data;
  int64_t vh;
};

// Byte offset of the link record (parity, mu, site); with present false, the
// end of the array: every read there is out of the buffer's range, returns
// zeros and moves no data (a hop term that is cut off loads its link without
// a branch).  The FP32 and FP16 arrays (80 vh records of 80 or 40 bytes)
// stay below 2^31 bytes under the library's size limits, so that offset plus
// a record does not wrap.
template <typename L>
__device__ __forceinline__ uint32_t link_offset(const Gauge<L>& g, int parity, int mu, uint32_t site, bool present) {
  using C2 = typename Gauge<L>::c2;
  constexpr uint32_t rec = 10u * (uint32_t)sizeof(C2);
  if (sizeof(C2) < 16 && !present) return 8u * (uint32_t)g.vh * rec;
  return ((uint32_t)(parity * 4 + mu) * (uint32_t)g.vh + site) * rec;
}

template <typename L, typename T>
__device__ __forceinline__ void load_link(const Gauge<L>& g, int parity, int mu, uint32_t site, T* u,
                                          bool present = true) {
  using C2 = typename Gauge<L>::c2;
  const __amdgpu_buffer_rsrc_t r = make_rsrc(g.data, (uint64_t)80 * (uint64_t)g.vh * sizeof(C2));
  const uint32_t off = link_offset(g, parity, mu, site, present);
  if constexpr (sizeof(C2) == 16) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * 16, 0, 0);
      u[2 * k] = (T)__hiloint2double(c.y, c.x);
      u[2 * k + 1] = (T)__hiloint2double(c.w, c.z);
    }
  } else if constexpr (sizeof(C2) == 4) {
    // FP16 record (40 bytes): entries 0-3, 4-7 and 8.  The conversions fold
    // into the consumers' v_fma_mix_f32 (the SU(3) product), so the link
    // costs no conversion instructions.
    const u32x4 c0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    const u32x4 c1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
    const uint32_t c2w = __builtin_amdgcn_raw_buffer_load_b32(r, off + 32, 0, 0);
    const uint32_t w[9] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w, c2w};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      u[2 * k] = (T)half_lo(w[k]);
      u[2 * k + 1] = (T)half_hi(w[k]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + j * 16, 0, 0);
      u[4 * j] = (T)__uint_as_float(c.x);
      u[4 * j + 1] = (T)__uint_as_float(c.y);
      if (j < 4) {
        u[4 * j + 2] = (T)__uint_as_float(c.z);
        u[4 * j + 3] = (T)__uint_as_float(c.w);
      }
    }
  }
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

// Projection straight from the 24 stored halves of a site (three 16-byte
// chunks, component index (spin * 3 + colour) * 2 + re/im): each output is
// psi_up + SIGN * (G psi_dn) in FP32.
__device__ __forceinline__ float half_at(const uint4* q, int k) {
  const uint32_t w = word(q[k >> 3], (k >> 1) & 3);
  return (k & 1) ? half_hi(w) : half_lo(w);
}

//
// Each output is one v_fma_mix_f32 on the two stored halves: the unit
// multiplier is hidden from the compiler, which would otherwise fold the
// product away and convert both halves separately before an FP32 add.  The
// result is the same FP32 number (the conversions are exact, the sum is
// rounded once either way).
template <int MU, int SIGN>
__device__ __forceinline__ void project_h(const uint4* q, float* h) {
  float S = (float)SIGN;
  asm volatile("" : "+v"(S));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float u0r = half_at(q, (0 * 3 + c) * 2), u0i = half_at(q, (0 * 3 + c) * 2 + 1);
    const float u1r = half_at(q, (1 * 3 + c) * 2), u1i = half_at(q, (1 * 3 + c) * 2 + 1);
    const float d2r = half_at(q, (2 * 3 + c) * 2), d2i = half_at(q, (2 * 3 + c) * 2 + 1);
    const float d3r = half_at(q, (3 * 3 + c) * 2), d3i = half_at(q, (3 * 3 + c) * 2 + 1);
    float h0r, h0i, h1r, h1i;
    if constexpr (MU == 0) {
      h0r = __builtin_fmaf(S, d3i, u0r); h0i = __builtin_fmaf(-S, d3r, u0i);
      h1r = __builtin_fmaf(S, d2i, u1r); h1i = __builtin_fmaf(-S, d2r, u1i);
    } else if constexpr (MU == 1) {
      h0r = __builtin_fmaf(-S, d3r, u0r); h0i = __builtin_fmaf(-S, d3i, u0i);
      h1r = __builtin_fmaf(S, d2r, u1r); h1i = __builtin_fmaf(S, d2i, u1i);
    } else if constexpr (MU == 2) {
      h0r = __builtin_fmaf(S, d2i, u0r); h0i = __builtin_fmaf(-S, d2r, u0i);
      h1r = __builtin_fmaf(-S, d3i, u1r); h1i = __builtin_fmaf(S, d3r, u1i);
    } else {
      h0r = __builtin_fmaf(S, d2r, u0r); h0i = __builtin_fmaf(S, d2i, u0i);
      h1r = __builtin_fmaf(S, d3r, u1r); h1i = __builtin_fmaf(S, d3i, u1i);
    }
    h[(0 * 3 + c) * 2] = h0r; h[(0 * 3 + c) * 2 + 1] = h0i;
    h[(1 * 3 + c) * 2] = h1r; h[(1 * 3 + c) * 2 + 1] = h1i;
  }
}

// the raw 16-bit values of a site and its scale
template <typename S>
__device__ __forceinline__ float load_site_raw16(const Field<S>& f, uint32_t i, uint4* q) {
  using C = typename Field<S>::chunk;
  const __amdgpu_buffer_rsrc_t r = field_rsrc(f);
  const uint32_t off = i * (uint32_t)sizeof(C);
  const uint32_t cs = (uint32_t)f.stride * (uint32_t)sizeof(C);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(f.scale, (uint64_t)f.stride * 4u);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, off + k * cs, 0, 0);
    q[k].x = c.x; q[k].y = c.y; q[k].z = c.z; q[k].w = c.w;
  }
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0));
}



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

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += sc [ g ; s G^dag g ]  (reconstruct_add with a scale folded into FMAs)
template <int MU, int SIGN, typename T>
__device__ __forceinline__ void reconstruct_fma(const T* g, T sc, T* acc) {
  const T ss = SIGN * sc;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T g0r = g[(0 * 3 + c) * 2], g0i = g[(0 * 3 + c) * 2 + 1];
    const T g1r = g[(1 * 3 + c) * 2], g1i = g[(1 * 3 + c) * 2 + 1];
    acc[(0 * 3 + c) * 2] = fmadd(sc, g0r, acc[(0 * 3 + c) * 2]);
    acc[(0 * 3 + c) * 2 + 1] = fmadd(sc, g0i, acc[(0 * 3 + c) * 2 + 1]);
    acc[(1 * 3 + c) * 2] = fmadd(sc, g1r, acc[(1 * 3 + c) * 2]);
    acc[(1 * 3 + c) * 2 + 1] = fmadd(sc, g1i, acc[(1 * 3 + c) * 2 + 1]);
    T l0r, l0i, l1r, l1i;
    if constexpr (MU == 0) {
      l0r = -g1i; l0i = g1r; l1r = -g0i; l1i = g0r;
    } else if constexpr (MU == 1) {
      l0r = g1r; l0i = g1i; l1r = -g0r; l1i = -g0i;
    } else if constexpr (MU == 2) {
      l0r = -g0i; l0i = g0r; l1r = g1i; l1i = -g1r;
    } else {
      l0r = g0r; l0i = g0i; l1r = g1r; l1i = g1i;
    }
    acc[(2 * 3 + c) * 2] = fmadd(ss, l0r, acc[(2 * 3 + c) * 2]);
    acc[(2 * 3 + c) * 2 + 1] = fmadd(ss, l0i, acc[(2 * 3 + c) * 2 + 1]);
    acc[(3 * 3 + c) * 2] = fmadd(ss, l1r, acc[(3 * 3 + c) * 2]);
    acc[(3 * 3 + c) * 2 + 1] = fmadd(ss, l1i, acc[(3 * 3 + c) * 2 + 1]);
  }
}

// g = U h (DAG = false) or U^dag h (DAG = true), for the two spins of h;
// every complex product-accumulate is four fused multiply-adds
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
        re = fmadd(ur, hr, re);
        re = fmadd(-ui, hi, re);
        im = fmadd(ur, hi, im);
        im = fmadd(ui, hr, im);
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
  // 32-bit arithmetic: a grid has fewer than 2^31 workgroups
  const uint32_t nb = (uint32_t)nblocks, bb = (uint32_t)b;
  const uint32_t q = nb >> 3, r = nb & 7u;
  const uint32_t k = bb & 7u, j = bb >> 3;
  return (int64_t)((k < r) ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j);
}

// --------------------------------------------------------------------------
// lattice geometry of one parity (single-parity index = lex / 2)
// --------------------------------------------------------------------------
// n / d for 0 <= n < 2^31 by multiply-high: s = ceil(log2 d),
// m = ceil(2^(32+s) / d) - 2^32, n / d = (mulhi(n, m) + n) >> s.
struct FastDiv {
  uint32_t d, m, s;
  __device__ __forceinline__ uint32_t div(uint32_t n) const { return (__umulhi(n, m) + n) >> s; }
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  if (d == 0) d = 1;   // nothing is ever divided by an empty extent; keep the constants finite
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << (32 + s)) + d - 1) / d) - (1ull << 32));
  return f;
}

struct Lattice {
  int X, Y, Z, T;
  int64_t vh;
  FastDiv fx, fy, fz;   // division by X, Y, Z

  __device__ __forceinline__ void coords(int64_t i, int parity, int* c) const {
    const uint32_t l0 = 2u * (uint32_t)i;
    const uint32_t q1 = fx.div(l0);
    const int x0 = (int)(l0 - q1 * (uint32_t)X);
    const uint32_t q2 = fy.div(q1);
    c[1] = (int)(q1 - q2 * (uint32_t)Y);
    const uint32_t q3 = fz.div(q2);
    c[2] = (int)(q2 - q3 * (uint32_t)Z);
    c[3] = (int)q3;
    c[0] = x0 + ((c[1] + c[2] + c[3] + parity) & 1);
  }
  __device__ __forceinline__ uint32_t lex(const int* c) const {
    return (uint32_t)c[0] + (uint32_t)X * ((uint32_t)c[1] + (uint32_t)Y * ((uint32_t)c[2] + (uint32_t)Z * (uint32_t)c[3]));
  }
  __device__ __forceinline__ uint32_t index(const int* c) const { return lex(c) >> 1; }
  __device__ __forceinline__ int ext(int mu) const { return mu == 0 ? X : mu == 1 ? Y : mu == 2 ? Z : T; }
  __device__ __forceinline__ uint32_t stride(int mu) const {
    return mu == 0 ? 1u : mu == 1 ? (uint32_t)X : mu == 2 ? (uint32_t)X * Y : (uint32_t)X * Y * Z;
  }
};

inline Lattice make_lattice(int X, int Y, int Z, int T) {
  Lattice l;
  l.X = X; l.Y = Y; l.Z = Z; l.T = T;
  l.vh = (int64_t)X * Y * Z * T / 2;
  l.fx = make_fastdiv(X);
  l.fy = make_fastdiv(Y);
  l.fz = make_fastdiv(Z);
  return l;
}

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
  const short4* origin;   // [nsub] global coordinates of each subdomain's corner
  const short4* coords;   // [n_out] local coordinates of the output sites
  const int* nbr;         // [n_out][8]
  const int* wmap;        // [n_out] index into the centre-field region, -1 = zero; null = same region
  int n_out, n_in, n_w;
  int bps;                // blocks per subdomain
  FastDiv fbps;           // division by bps (block -> subdomain)
  int sub[4], dims[4], nblk[4];
};

}  // namespace mspcg
