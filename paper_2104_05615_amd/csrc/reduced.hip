// Kernels of the reduced-Ls preconditioner (Sec. 3.3): the transform T,
// which mixes spin and the fifth dimension and is the identity in colour and
// on the 4D sites, its adjoint with the mu shift and the PR dots fused, and
// the site sums that form the gradient of the training loss.
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

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Sites per workgroup of the transform: the input tile [ns][Li][24] stays
// within 48 KB of LDS, at most 16 sites and 1024 threads.
int transform_sites(int Li, int Lo, Prec p) {
  const int bytes = (p == Prec::F64 ? 8 : 4) * 24 * Li;
  int ns = 49152 / bytes;
  if (ns > 16) ns = 16;
  if (ns * Lo > 1024) ns = 1024 / Lo;
  return ns < 1 ? 1 : ns;
}

int64_t transform_blocks(int64_t vh, int Li, int Lo, Prec p) {
  const int ns = transform_sites(Li, Lo, p);
  return (vh + ns - 1) / ns;
}

// out(x, so, mo, c) = sum_{si, mi} W[so][mo][si][mi] in(x, si, mi, c)
//                     (+ mu r(x, so, mo, c) when r is given),
// W complex [Lo][4][Li][4].  Workgroup: ns 4D sites x Lo output slices
// (thread = (site, so), so fastest); the sites' inputs are staged in LDS.
// With p1 set, each workgroup writes Re<out, r> (and Re<out, rold> to p2
// when rold is given) over its sites, indexed [rhs][workgroup].
template <typename S>
__global__ void __launch_bounds__(1024)
k_transform(Field<S> out_b, Field<S> in_b, const typename Cplx<calc_t<S>>::type* W, int Li, int Lo, int64_t vh, int ns,
            calc_t<S> mu, Field<S> r_b, Field<S> rold_b, bool has_r, bool has_rold, double* p1, double* p2,
            const int* mask) {
  using T = calc_t<S>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* tile = reinterpret_cast<T*>(red + 16);
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const Field<S> out = out_b.at(rhs), in = in_b.at(rhs), r = r_b.at(rhs), rold = rold_b.at(rhs);
  const int tid = threadIdx.x;
  const int64_t site0 = (int64_t)blockIdx.x * ns;
  for (int k = tid; k < ns * Li; k += blockDim.x) {
    const int sl = k / Li, si = k - sl * Li;
    const int64_t site = site0 + sl;
    T v[24];
    if (site < vh) load_site(in, (uint32_t)(site * Li + si), v);
    else {
#pragma unroll
      for (int j = 0; j < 24; ++j) v[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < 24; ++j) tile[k * 24 + j] = v[j];
  }
  __syncthreads();
  const bool inb = tid < ns * Lo;
  const int sl = inb ? tid / Lo : 0, so = inb ? tid - sl * Lo : 0;
  const int64_t site = site0 + sl;
  const bool valid = inb && site < vh;
  T acc[24];
#pragma unroll
  for (int j = 0; j < 24; ++j) acc[j] = 0;
  if (valid) {
    const T* v0 = tile + sl * Li * 24;
    for (int si = 0; si < Li; ++si) {
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) {
        const T* v = v0 + si * 24 + mi * 6;
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
          const auto w = W[((so * 4 + mo) * Li + si) * 4 + mi];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc[(mo * 3 + c) * 2] += w.x * v[2 * c] - w.y * v[2 * c + 1];
            acc[(mo * 3 + c) * 2 + 1] += w.x * v[2 * c + 1] + w.y * v[2 * c];
          }
        }
      }
    }
  }
  double d1 = 0, d2 = 0;
  if (valid && has_r) {
    T rv[24];
    load_site(r, (uint32_t)(site * Lo + so), rv);
#pragma unroll
    for (int j = 0; j < 24; ++j) {
      acc[j] += mu * rv[j];
      d1 += (double)acc[j] * (double)rv[j];
    }
    if (has_rold) {
      load_site(rold, (uint32_t)(site * Lo + so), rv);
#pragma unroll
      for (int j = 0; j < 24; ++j) d2 += (double)acc[j] * (double)rv[j];
    }
  }
  if (valid) store_site(out, (uint32_t)(site * Lo + so), acc);
  if (p1) {
    const int64_t pi = (int64_t)rhs * gridDim.x + blockIdx.x;
    const double t1 = block_sum(d1, red);
    if (tid == 0) p1[pi] = t1;
    if (has_rold) {
      const double t2 = block_sum(d2, red);
      if (tid == 0) p2[pi] = t2;
    }
  }
}

void transform(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const void* W, int Li, int Lo,
               int64_t vh, double mu, const FieldPtr* r, const FieldPtr* rold, double* p1, double* p2,
               const Batch& bt) {
  if (p != Prec::F32 && p != Prec::F64) throw std::runtime_error("transform: FP32 or FP64 fields only");
  const int ns = transform_sites(Li, Lo, p);
  const int64_t nblk = (vh + ns - 1) / ns;
  const int threads = ((ns * Lo + 63) / 64) * 64;
  const size_t lds = 16 * sizeof(double) + (size_t)ns * Li * 24 * (p == Prec::F64 ? 8 : 4);
  const FieldPtr none = in;
  const FieldPtr& rr = r ? *r : none;
  const FieldPtr& ro = rold ? *rold : none;
  dim3 grid((unsigned)nblk, (unsigned)bt.n);
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_transform<double>, grid, dim3(threads), lds, st, typed<double>(out), typed<double>(in),
                       (const double2*)W, Li, Lo, vh, ns, mu, typed<double>(rr), typed<double>(ro), r != nullptr,
                       rold != nullptr, p1, p2, bt.mask);
  else
    hipLaunchKernelGGL(k_transform<float>, grid, dim3(threads), lds, st, typed<float>(out), typed<float>(in),
                       (const float2*)W, Li, Lo, vh, ns, (float)mu, typed<float>(rr), typed<float>(ro),
                       r != nullptr, rold != nullptr, p1, p2, bt.mask);
  LAUNCH_CHECK();
}

// e = a - b over the reals of two fields of one layout; each workgroup
// writes its sum of e^2.
template <typename T>
__global__ void k_diff_norm(T* e, const T* a, const T* b, int64_t n, double* partial) {
  __shared__ double red[16];
  double l = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T d = a[i] - b[i];
    e[i] = d;
    l += (double)d * (double)d;
  }
  const double t = block_sum(l, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

void diff_norm(hipStream_t st, Prec p, void* e, const void* a, const void* b, int64_t nreal, double* partial,
               int nblocks) {
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_diff_norm<double>, dim3(nblocks), dim3(256), 0, st, (double*)e, (const double*)a,
                       (const double*)b, nreal, partial);
  else
    hipLaunchKernelGGL(k_diff_norm<float>, dim3(nblocks), dim3(256), 0, st, (float*)e, (const float*)a,
                       (const float*)b, nreal, partial);
  LAUNCH_CHECK();
}

// G[(s mf) (t mg)] = sum over sites x and colour c of f(x, s, mf, c) conj(g(x, t, mg, c)),
// f with Lf slices, g with Lg; per workgroup over a contiguous range of
// sites, entries e = entry0 + tid + j * blockDim (j < 8), written to
// partial[workgroup][e] as (re, im).
template <typename S>
__global__ void __launch_bounds__(256)
k_outer_sum(Field<S> f, Field<S> g, int Lf, int Lg, int64_t vh, int64_t per_block, int entry0, int nent,
            double2* partial) {
  using T = calc_t<S>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* fs = reinterpret_cast<T*>(lds_raw);
  T* gs = fs + Lf * 24;
  double ar[8], ai[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) ar[j] = ai[j] = 0;
  const int64_t x0 = (int64_t)blockIdx.x * per_block;
  const int64_t x1 = x0 + per_block < vh ? x0 + per_block : vh;
  const int ncol = Lg * 4;
  for (int64_t x = x0; x < x1; ++x) {
    __syncthreads();
    for (int k = threadIdx.x; k < Lf + Lg; k += blockDim.x) {
      T v[24];
      if (k < Lf) load_site(f, (uint32_t)(x * Lf + k), v);
      else load_site(g, (uint32_t)(x * Lg + (k - Lf)), v);
      T* dst = k < Lf ? fs + k * 24 : gs + (k - Lf) * 24;
#pragma unroll
      for (int j = 0; j < 24; ++j) dst[j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = entry0 + (int)threadIdx.x + j * (int)blockDim.x;
      if (e >= nent || e - entry0 >= 8 * (int)blockDim.x) continue;
      const int row = e / ncol, col = e - row * ncol;       // row = s * 4 + mf, col = t * 4 + mg
      const T* a = fs + (row >> 2) * 24 + (row & 3) * 6;
      const T* b = gs + (col >> 2) * 24 + (col & 3) * 6;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ar[j] += (double)a[2 * c] * b[2 * c] + (double)a[2 * c + 1] * b[2 * c + 1];
        ai[j] += (double)a[2 * c + 1] * b[2 * c] - (double)a[2 * c] * b[2 * c + 1];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = entry0 + (int)threadIdx.x + j * (int)blockDim.x;
    if (e < nent && e - entry0 < 8 * (int)blockDim.x) partial[(int64_t)blockIdx.x * nent + e] = make_double2(ar[j], ai[j]);
  }
}

// G[e] += sum over workgroups of partial[.][e]
__global__ void k_outer_reduce(const double2* partial, int nparts, int nent, double2* G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  double re = 0, im = 0;
  for (int b = 0; b < nparts; ++b) {
    const double2 v = partial[(int64_t)b * nent + e];
    re += v.x;
    im += v.y;
  }
  G[e].x += re;
  G[e].y += im;
}

int outer_sum_parts(int64_t vh) { return vh < 240 ? (int)vh : 240; }

void outer_sum(hipStream_t st, Prec p, const FieldPtr& f, const FieldPtr& g, int Lf, int Lg, int64_t vh,
               double2* partial, double2* G) {
  if (p != Prec::F32 && p != Prec::F64) throw std::runtime_error("outer_sum: FP32 or FP64 fields only");
  const int nparts = outer_sum_parts(vh);
  const int64_t per = (vh + nparts - 1) / nparts;
  const int nent = Lf * 4 * Lg * 4;
  const size_t lds = (size_t)(Lf + Lg) * 24 * (p == Prec::F64 ? 8 : 4);
  for (int e0 = 0; e0 < nent; e0 += 8 * 256) {
    if (p == Prec::F64)
      hipLaunchKernelGGL(k_outer_sum<double>, dim3(nparts), dim3(256), lds, st, typed<double>(f), typed<double>(g), Lf,
                         Lg, vh, per, e0, nent, partial);
    else
      hipLaunchKernelGGL(k_outer_sum<float>, dim3(nparts), dim3(256), lds, st, typed<float>(f), typed<float>(g), Lf,
                         Lg, vh, per, e0, nent, partial);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_outer_reduce, dim3((nent + 255) / 256), dim3(256), 0, st, partial, nparts, nent, G);
  LAUNCH_CHECK();
}

}  // namespace mspcg
