// Full-lattice kernels: the hop operator with its fused epilogue, the
// fifth-dimension-only operator, layout conversions, the outer solver's
// BLAS-1 and deterministic reductions.
#include <atomic>
#include <map>
#include <mutex>
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

// process-wide choice of the fifth-dimension epilogue engine for FP32 and
// 16-bit site kernels with Ls <= 16: MFMA (default) or the vector ALUs
static std::atomic<int> g_mfma_epilogue{1};
void set_mfma_epilogue(bool on) { g_mfma_epilogue.store(on ? 1 : 0); }
bool mfma_epilogue() { return g_mfma_epilogue.load() != 0; }

// ---------------------------------------------------------------- static workspace
// Device memory for the entry point that allocates nothing
// (mspcg_apply_device_noalloc): every workspace that call needs is carved
// from this array.  Each device that loads the library holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is a stand-in, not a device address):
// scratch_device_ptr resolves the address on each device once and the
// library uses only that pointer.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* scratch_device_ptr() {
  static std::mutex mu;
  static std::map<int, void*> ptr;   // device -> address of its copy
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("scratch: hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptr.find(dev);
  if (it != ptr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    throw std::runtime_error(std::string("scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
  ptr[dev] = p;
  return p;
}

bool uses_mfma(int Ls, Prec p) { return p != Prec::F64 && Ls <= 16 && mfma_epilogue(); }

int sites_per_block(int Ls, Prec p) {
  if (uses_mfma(Ls, p)) return 16;
  // blocks of <= 256 threads; FP64 tiles kept small for occupancy; the LDS
  // of the widest site kernel (two tiles and the matrices) stays <= 60 KB
  int ns = 256 / Ls;
  if (p == Prec::F64 && ns > 8) ns = 8;
  const size_t elem = p == Prec::F64 ? 8 : 4;
  while (ns > 1 && 128 + elem * (size_t)(6 * Ls * Ls + 2 * ns * tile_stride(Ls)) > 60 * 1024) --ns;
  if (ns < 1) ns = 1;
  return ns;
}

int64_t full_blocks(int64_t vh, int Ls, Prec p) {
  const int ns = sites_per_block(Ls, p);
  return (vh + ns - 1) / ns;
}

// ---------------------------------------------------------------- hop launch

// work items of a hop launch with nblk site blocks per RHS
static HopWork hop_work(int64_t nblk, const Batch& bt, const Sched& sc) {
  HopWork wk;
  wk.nblk = nblk;
  wk.nrhs = bt.n;
  wk.order = sc.order;
  wk.xcd = sc.xcd;
  wk.mask = bt.mask;
  wk.fdiv = make_fastdiv((uint32_t)(sc.order == 0 ? nblk : bt.n));
  return wk;
}

template <typename Geo, typename S, bool MF>
static void launch_hop_mf(hipStream_t st, const Geo& geo, int64_t nblocks, const FieldPtr& out, const FieldPtr& in,
                          const FieldPtr* w, int Ls, int ns, bool dagger, const Epilogue& epi, const Batch& bt,
                          const Sched& sc) {
  using T = calc_t<S>;
  if (epi.dot_partial && !(dagger && w))
    throw std::runtime_error("hop: the fused dot belongs to an adjoint hop with a centre field");
  const bool tileB = w != nullptr && !epi.w_identity && epi.E0 != nullptr;
  const size_t lds = site_lds_bytes<T>(ns, Ls, tileB, MF, UsesMfma<S>::half_ops);
  Field<S> wf = w ? typed<S>(*w) : Field<S>{};
  Field<S> df = epi.dotf ? typed<S>(*epi.dotf) : Field<S>{};
  const T* E0 = (const T*)epi.E0;
  const T* E1 = (const T*)epi.E1;
  const HopWork wk = hop_work(nblocks, bt, sc);
  dim3 grid((unsigned)(nblocks * bt.n)), block(site_block_threads(ns, Ls));
  const int wid = epi.w_identity ? 1 : 0;
  if (dagger) {
    if (w) hipLaunchKernelGGL((k_hop<Geo, S, true, true, MF>), grid, block, lds, st, geo, typed<S>(out), typed<S>(in), wf,
                              df, Ls, ns, E0, E1, wid, epi.dot_partial, wk);
    else hipLaunchKernelGGL((k_hop<Geo, S, true, false, MF>), grid, block, lds, st, geo, typed<S>(out), typed<S>(in),
                            wf, df, Ls, ns, E0, E1, wid, epi.dot_partial, wk);
  } else {
    if (w) hipLaunchKernelGGL((k_hop<Geo, S, false, true, MF>), grid, block, lds, st, geo, typed<S>(out), typed<S>(in),
                              wf, df, Ls, ns, E0, E1, wid, epi.dot_partial, wk);
    else hipLaunchKernelGGL((k_hop<Geo, S, false, false, MF>), grid, block, lds, st, geo, typed<S>(out), typed<S>(in),
                            wf, df, Ls, ns, E0, E1, wid, epi.dot_partial, wk);
  }
  LAUNCH_CHECK();
}

template <typename Geo, typename S>
static void launch_hop(hipStream_t st, const Geo& geo, int64_t nblocks, const FieldPtr& out, const FieldPtr& in,
                       const FieldPtr* w, int Ls, int ns, bool dagger, const Epilogue& epi, const Batch& bt,
                       const Sched& sc) {
  if (bt.n < 1) throw std::runtime_error("hop: batch of fewer than one RHS");
  if constexpr (std::is_same<S, double>::value) {
    launch_hop_mf<Geo, S, false>(st, geo, nblocks, out, in, w, Ls, ns, dagger, epi, bt, sc);
  } else {
    if (uses_mfma(Ls, out.prec)) launch_hop_mf<Geo, S, true>(st, geo, nblocks, out, in, w, Ls, ns, dagger, epi, bt, sc);
    else launch_hop_mf<Geo, S, false>(st, geo, nblocks, out, in, w, Ls, ns, dagger, epi, bt, sc);
  }
}

int64_t hop_full_blocks(const Lattice& lat, int Ls, Prec p) {
  const int ns = sites_per_block(Ls, p);
  return (lat.vh + ns - 1) / ns;
}

// Chunk shape of the chunked block order (BlockOrder): bzc z-planes by bb
// blocks of a plane whose input spinors take at most `budget` bytes, with the
// fewest neighbour planes and rows outside the chunk per site inside it
// (2 / bzc + 2 / rows, a dimension the chunk spans whole counting 0).
// Lexicographic order when blocks do not tile whole planes.
static BlockOrder block_order(const Lattice& lat, int ns, int Ls, int site_bytes, int64_t budget) {
  BlockOrder bo{};
  bo.chunk = 0;
  const int64_t S = lat.vh / lat.T, P = (int64_t)lat.X * lat.Y / 2, half_x = lat.X / 2;
  if (lat.vh % lat.T || S % ns || P % ns) return bo;
  const int64_t bz = P / ns, blk_bytes = (int64_t)ns * Ls * site_bytes;
  double best = 1e30;
  int64_t bbz = 0, bbb = 0;
  for (int64_t zc = 1; zc <= lat.Z; ++zc) {
    if (lat.Z % zc) continue;
    for (int64_t b = 1; b <= bz; ++b) {
      if (bz % b) continue;
      if (b < bz && (b * ns) % half_x) continue;   // a band of whole rows
      if (zc * b * blk_bytes > budget) continue;
      const double halo = (zc < lat.Z ? 2.0 / zc : 0.0) + (b < bz ? 2.0 * half_x / (b * ns) : 0.0);
      if (halo < best - 1e-12 || (halo < best + 1e-12 && zc * b > bbz * bbb)) {
        best = halo;
        bbz = zc;
        bbb = b;
      }
    }
  }
  if (bbz == 0 || (bbz == lat.Z && bbb == bz)) return bo;   // whole slices: the lexicographic order
  bo.chunk = (uint32_t)(bbz * bbb);
  bo.bzc = (uint32_t)bbz;
  bo.bb = (uint32_t)bbb;
  bo.bz = (uint32_t)bz;
  bo.bps = (uint32_t)(S / ns);
  bo.fchunk = make_fastdiv(bo.chunk);
  bo.fT = make_fastdiv((uint32_t)lat.T);
  bo.fbb = make_fastdiv(bo.bb);
  bo.fnyc = make_fastdiv((uint32_t)(bz / bbb));
  return bo;
}

template <typename S>
static void hop_full_t(hipStream_t st, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, const void* gauge,
                       const HopGeometry& geo, bool dagger, const Epilogue& epi, const Batch& bt, const Sched& sc) {
  using T = calc_t<S>;
  FullGeo<T> g;
  g.lat = geo.lat;
  g.par = geo.out_parity;
  g.g.data = reinterpret_cast<const typename Gauge<T>::c2*>(gauge);
  g.g.vh = geo.lat.vh;
  const int ns = sites_per_block(geo.Ls, out.prec);
  g.order.chunk = 0;
  if (sc.tchunk > 0 && geo.lat.vh < (int64_t)1 << 31)
    g.order = block_order(geo.lat, ns, geo.Ls, 24 * (int)sizeof(T), (int64_t)80 << (10 + sc.tchunk));
  launch_hop<FullGeo<T>, S>(st, g, (geo.lat.vh + ns - 1) / ns, out, in, w, geo.Ls, ns, dagger, epi, bt, sc);
}

void hop_full(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w,
              const void* gauge, const HopGeometry& geo, bool dagger, const Epilogue& epi, const Batch& bt,
              const Sched& sc) {
  switch (p) {
    case Prec::F64: hop_full_t<double>(st, out, in, w, gauge, geo, dagger, epi, bt, sc); break;
    case Prec::F32: hop_full_t<float>(st, out, in, w, gauge, geo, dagger, epi, bt, sc); break;
    case Prec::F16: hop_full_t<__half>(st, out, in, w, gauge, geo, dagger, epi, bt, sc); break;
    case Prec::BF16: hop_full_t<__hip_bfloat16>(st, out, in, w, gauge, geo, dagger, epi, bt, sc); break;
    case Prec::I8: hop_full_t<int8_t>(st, out, in, w, gauge, geo, dagger, epi, bt, sc); break;
  }
}

template <typename S>
static void hop_sub_t(hipStream_t st, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, const void* gauge,
                      const Lattice& lat, int out_parity, const SubTables& tb, int nsub, int Ls, bool dagger,
                      const Epilogue& epi, const Batch& bt, const Sched& sc) {
  using T = calc_t<S>;
  using L = typename std::conditional<StoreTraits<S>::scaled, __half, T>::type;
  constexpr bool half = std::is_same<S, __half>::value || std::is_same<S, int8_t>::value;
  const int ns = sites_per_block(Ls, out.prec);
  // FP16 and 8-bit storage with Ls a multiple of 4: SU(3) products on 4 x 4 x 4
  // MFMA blocks (each block's four lanes are four slices of one 4D site)
  if (half && Ls % 4 == 0) {
    SubGeo<T, L, half> g;
    g.tb = tb;
    g.lat = lat;
    g.par = out_parity;
    g.g.data = reinterpret_cast<const typename Gauge<L>::c2*>(gauge);
    g.g.vh = lat.vh;
    launch_hop<SubGeo<T, L, half>, S>(st, g, (int64_t)nsub * tb.bps, out, in, w, Ls, ns, dagger, epi, bt, sc);
    return;
  }
  SubGeo<T, L> g;
  g.tb = tb;
  g.lat = lat;
  g.par = out_parity;
  g.g.data = reinterpret_cast<const typename Gauge<L>::c2*>(gauge);
  g.g.vh = lat.vh;
  launch_hop<SubGeo<T, L>, S>(st, g, (int64_t)nsub * tb.bps, out, in, w, Ls, ns, dagger, epi, bt, sc);
}

void hop_sub(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, const void* gauge,
             const Lattice& lat, int out_parity, const SubTables& tb, int nsub, int Ls, bool dagger,
             const Epilogue& epi, const Batch& bt, const Sched& sc) {
  switch (p) {
    case Prec::F64: hop_sub_t<double>(st, out, in, w, gauge, lat, out_parity, tb, nsub, Ls, dagger, epi, bt, sc); break;
    case Prec::F32: hop_sub_t<float>(st, out, in, w, gauge, lat, out_parity, tb, nsub, Ls, dagger, epi, bt, sc); break;
    case Prec::F16: hop_sub_t<__half>(st, out, in, w, gauge, lat, out_parity, tb, nsub, Ls, dagger, epi, bt, sc); break;
    case Prec::BF16:
      hop_sub_t<__hip_bfloat16>(st, out, in, w, gauge, lat, out_parity, tb, nsub, Ls, dagger, epi, bt, sc);
      break;
    case Prec::I8: hop_sub_t<int8_t>(st, out, in, w, gauge, lat, out_parity, tb, nsub, Ls, dagger, epi, bt, sc); break;
  }
}

// ---------------------------------------------------------------- 5D-only ops

// out = E w (copy when E is null); optional |out|^2 partial per block.
// With beta_slot >= 0 the input is first updated in place,
//   w <- z + beta w  (beta = scal[beta_slot]),
// which is the search-direction update of CG fused with the M_phi that
// starts the next operator application.
template <typename S>
__global__ void __launch_bounds__(256)
k_apply5(Field<S> out, Field<S> w, Field<S> z, const double* scal, int beta_slot, int64_t nsites, int Ls, int ns,
         const calc_t<S>* E, double* norm_partial, const int* mask) {
  using T = calc_t<S>;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;   // uniform over the workgroup
  out = out.at(rhs);
  w = w.at(rhs);
  z = z.at(rhs);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* red = reinterpret_cast<double*>(lds_raw);
  T* mats = reinterpret_cast<T*>(red + 16);
  T* tileA = mats + 2 * Ls * Ls;
  const int tid = threadIdx.x;
  const bool inb = tid < ns * Ls;
  const int sl = inb ? tid / Ls : 0, s = inb ? tid - sl * Ls : 0;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t site = blk * ns + sl;
  const bool valid = inb && site < nsites;
  const int64_t i5 = site * Ls + s;
  if (E)
    for (int k = tid; k < 2 * Ls * Ls; k += blockDim.x) mats[k] = E[k];
  T v[24];
  if (valid) {
    load_site(w, i5, v);
    if (beta_slot >= 0) {
      const T beta = (T)scal[(int64_t)rhs * SLOT_COUNT + beta_slot];
      T zv[24];
      load_site(z, i5, zv);
#pragma unroll
      for (int k = 0; k < 24; ++k) v[k] = zv[k] + beta * v[k];
      store_site(w, i5, v);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0;
  }
  T* my = tileA + sl * tile_stride(Ls);
  if (inb) tile_put(my, s, v);
  __syncthreads();
  if (E && inb) mat5_lds(my, mats, s, Ls, v, false);
  if (norm_partial) {
    double loc = 0;
    if (valid) {
#pragma unroll
      for (int k = 0; k < 24; ++k) loc += (double)v[k] * (double)v[k];
    }
    const double tot = block_sum(loc, red);
    if (tid == 0) norm_partial[(int64_t)rhs * gridDim.x + blk] = tot;
  }
  if (valid) store_site(out, i5, v);
}

template <typename S>
static void apply5_t(hipStream_t st, const FieldPtr& out, const FieldPtr& w, const FieldPtr* z, const double* scal,
                     int beta_slot, const void* E, int64_t nsites, int Ls, double* norm_partial, const Batch& bt) {
  using T = calc_t<S>;
  const int ns = sites_per_block(Ls, out.prec);
  const int64_t nb = (nsites + ns - 1) / ns;
  const size_t lds = 16 * sizeof(double) + sizeof(T) * (size_t)(2 * Ls * Ls + ns * tile_stride(Ls));
  Field<S> zf = z ? typed<S>(*z) : Field<S>{};
  hipLaunchKernelGGL((k_apply5<S>), dim3((unsigned)nb, (unsigned)bt.n), dim3(site_block_threads(ns, Ls)), lds, st,
                     typed<S>(out), typed<S>(w), zf, scal, beta_slot, nsites, Ls, ns, (const T*)E, norm_partial,
                     bt.mask);
  LAUNCH_CHECK();
}

void apply5_full(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& w, const void* E, int64_t nsites,
                 int Ls, double* norm_partial, const Batch& bt) {
  switch (p) {
    case Prec::F64: apply5_t<double>(st, out, w, nullptr, nullptr, -1, E, nsites, Ls, norm_partial, bt); break;
    case Prec::F32: apply5_t<float>(st, out, w, nullptr, nullptr, -1, E, nsites, Ls, norm_partial, bt); break;
    case Prec::F16: apply5_t<__half>(st, out, w, nullptr, nullptr, -1, E, nsites, Ls, norm_partial, bt); break;
    case Prec::BF16: apply5_t<__hip_bfloat16>(st, out, w, nullptr, nullptr, -1, E, nsites, Ls, norm_partial, bt); break;
    case Prec::I8: apply5_t<int8_t>(st, out, w, nullptr, nullptr, -1, E, nsites, Ls, norm_partial, bt); break;
  }
}

void xpay_apply5(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& pvec, const FieldPtr& z,
                 const double* scal, int beta_slot, const void* E, int64_t nsites, int Ls, const Batch& bt) {
  switch (p) {
    case Prec::F64: apply5_t<double>(st, out, pvec, &z, scal, beta_slot, E, nsites, Ls, nullptr, bt); break;
    case Prec::F32: apply5_t<float>(st, out, pvec, &z, scal, beta_slot, E, nsites, Ls, nullptr, bt); break;
    default: throw std::runtime_error("xpay_apply5: outer vectors are FP64 or FP32");
  }
}

// ---------------------------------------------------------------- layout conversion

template <typename S>
__global__ void k_pack(Field<S> out, const double* canon, int64_t nsites, int Ls, const int* mask) {
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const int64_t i5 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i5 >= nsites * Ls) return;
  out = out.at(rhs);
  canon += (int64_t)rhs * nsites * Ls * 24;
  const int64_t site = i5 / Ls;
  const int s = (int)(i5 - site * Ls);
  const double* src = canon + ((int64_t)s * nsites + site) * 24;
  double v[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = src[k];
  store_site(out, i5, v);
}

template <typename S>
__global__ void k_unpack(double* canon, Field<S> in, int64_t nsites, int Ls, const int* mask) {
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const int64_t i5 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i5 >= nsites * Ls) return;
  in = in.at(rhs);
  canon += (int64_t)rhs * nsites * Ls * 24;
  const int64_t site = i5 / Ls;
  const int s = (int)(i5 - site * Ls);
  double v[24];
  load_site(in, i5, v);
  double* dst = canon + ((int64_t)s * nsites + site) * 24;
#pragma unroll
  for (int k = 0; k < 24; ++k) dst[k] = v[k];
}

void pack_field(hipStream_t st, const FieldPtr& out, const double* canon, int64_t nsites, int Ls, const Batch& bt) {
  const int64_t n = nsites * Ls;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)bt.n), block(256);
  switch (out.prec) {
    case Prec::F64:
      hipLaunchKernelGGL(k_pack<double>, grid, block, 0, st, typed<double>(out), canon, nsites, Ls, bt.mask);
      break;
    case Prec::F32:
      hipLaunchKernelGGL(k_pack<float>, grid, block, 0, st, typed<float>(out), canon, nsites, Ls, bt.mask);
      break;
    case Prec::F16:
      hipLaunchKernelGGL(k_pack<__half>, grid, block, 0, st, typed<__half>(out), canon, nsites, Ls, bt.mask);
      break;
    case Prec::BF16:
      hipLaunchKernelGGL(k_pack<__hip_bfloat16>, grid, block, 0, st, typed<__hip_bfloat16>(out), canon, nsites, Ls,
                         bt.mask);
      break;
    case Prec::I8:
      hipLaunchKernelGGL(k_pack<int8_t>, grid, block, 0, st, typed<int8_t>(out), canon, nsites, Ls, bt.mask);
      break;
  }
  LAUNCH_CHECK();
}

void unpack_field(hipStream_t st, double* canon, const FieldPtr& in, int64_t nsites, int Ls, const Batch& bt) {
  const int64_t n = nsites * Ls;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)bt.n), block(256);
  switch (in.prec) {
    case Prec::F64:
      hipLaunchKernelGGL(k_unpack<double>, grid, block, 0, st, canon, typed<double>(in), nsites, Ls, bt.mask);
      break;
    case Prec::F32:
      hipLaunchKernelGGL(k_unpack<float>, grid, block, 0, st, canon, typed<float>(in), nsites, Ls, bt.mask);
      break;
    case Prec::F16:
      hipLaunchKernelGGL(k_unpack<__half>, grid, block, 0, st, canon, typed<__half>(in), nsites, Ls, bt.mask);
      break;
    case Prec::BF16:
      hipLaunchKernelGGL(k_unpack<__hip_bfloat16>, grid, block, 0, st, canon, typed<__hip_bfloat16>(in), nsites, Ls,
                         bt.mask);
      break;
    case Prec::I8:
      hipLaunchKernelGGL(k_unpack<int8_t>, grid, block, 0, st, canon, typed<int8_t>(in), nsites, Ls, bt.mask);
      break;
  }
  LAUNCH_CHECK();
}

// zero every masked RHS of a batched buffer (a kernel, so that it may sit in
// a captured graph)
__global__ void k_zero(uint4* data, int64_t n16, const int* mask) {
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  uint4* d = data + (int64_t)rhs * n16;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill_int(hipStream_t st, int* p, int n, int v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  LAUNCH_CHECK();
}

void zero_batched(hipStream_t st, void* data, int64_t bytes_per_rhs, const Batch& bt) {
  if (bytes_per_rhs % 16) throw std::runtime_error("zero_batched: size must be a multiple of 16 bytes");
  const int64_t n16 = bytes_per_rhs / 16;
  int64_t nb = (n16 + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)nb, (unsigned)bt.n), dim3(256), 0, st, (uint4*)data, n16, bt.mask);
  LAUNCH_CHECK();
}

template <typename C2>
__global__ void k_pack_gauge(C2* out, const double* canon, Lattice lat) {
  const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t V = 2 * lat.vh;
  if (lex >= V) return;
  const int x = (int)(lex % lat.X);
  const int64_t r = lex / lat.X;
  const int y = (int)(r % lat.Y);
  const int64_t r2 = r / lat.Y;
  const int z = (int)(r2 % lat.Z);
  const int t = (int)(r2 / lat.Z);
  const int par = (x + y + z + t) & 1;
  const int64_t cb = lex >> 1;
  for (int mu = 0; mu < 4; ++mu)
    for (int k = 0; k < 9; ++k) {
      const double* src = canon + ((lex * 4 + mu) * 9 + k) * 2;
      C2 c;
      if constexpr (sizeof(C2) == 4) {
        c.x = __float2half_rn((float)src[0]);
        c.y = __float2half_rn((float)src[1]);
      } else {
        c.x = src[0];
        c.y = src[1];
      }
      out[((int64_t)(par * 4 + mu) * lat.vh + cb) * 10 + k] = c;
    }
}

void pack_gauge(hipStream_t st, void* out, int bytes_per_real, const double* canon, const Lattice& lat) {
  const int64_t V = 2 * lat.vh;
  dim3 grid((unsigned)((V + 255) / 256)), block(256);
  if (bytes_per_real == 8) hipLaunchKernelGGL(k_pack_gauge<double2>, grid, block, 0, st, (double2*)out, canon, lat);
  else if (bytes_per_real == 4) hipLaunchKernelGGL(k_pack_gauge<float2>, grid, block, 0, st, (float2*)out, canon, lat);
  else hipLaunchKernelGGL(k_pack_gauge<__half2>, grid, block, 0, st, (__half2*)out, canon, lat);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- outer BLAS-1
//
// Outer vectors (FP64 or FP32) are flat arrays of chunks; every kernel runs
// a fixed grid so its per-block partial sums land in a fixed order.

int64_t blas_blocks(int64_t nchunks) {
  int64_t nb = (nchunks + 255) / 256;
  return nb > 2048 ? 2048 : (nb < 1 ? 1 : nb);
}

template <typename C> struct ChunkOps;
template <> struct ChunkOps<float4> {
  static constexpr int n = 4;
  __device__ static float get(const float4& c, int k) { return k == 0 ? c.x : k == 1 ? c.y : k == 2 ? c.z : c.w; }
  __device__ static void set(float4& c, int k, float v) {
    if (k == 0) c.x = v; else if (k == 1) c.y = v; else if (k == 2) c.z = v; else c.w = v;
  }
};
template <> struct ChunkOps<double2> {
  static constexpr int n = 2;
  __device__ static double get(const double2& c, int k) { return k == 0 ? c.x : c.y; }
  __device__ static void set(double2& c, int k, double v) { if (k == 0) c.x = v; else c.y = v; }
};

// Batched launches put the RHS in blockIdx.y: RHS r of a vector starts r
// whole vectors after RHS 0, its scalars at scal + r * SLOT_COUNT and its
// block partials at partial + r * gridDim.x.

// x += alpha p ; rn = r - alpha q ; partial |rn|^2     (alpha = scal[alpha_slot])
template <typename C>
__global__ void __launch_bounds__(256)
k_cg_update(C* x, const C* p, const C* r, const C* q, C* rn, int64_t n, const double* scal, int alpha_slot,
            double* partial, const int* mask) {
  __shared__ double red[16];
  using O = ChunkOps<C>;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const int64_t off = (int64_t)rhs * n;
  x += off; p += off; r += off; q += off; rn += off;
  const double alpha = scal[(int64_t)rhs * SLOT_COUNT + alpha_slot];
  double loc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    C xv = x[i], pv = p[i], rv = r[i], qv = q[i], ov;
#pragma unroll
    for (int k = 0; k < O::n; ++k) {
      O::set(xv, k, O::get(xv, k) + alpha * O::get(pv, k));
      const double v = O::get(rv, k) - alpha * O::get(qv, k);
      O::set(ov, k, v);
      const double vs = O::get(ov, k);
      loc += vs * vs;
    }
    x[i] = xv;
    rn[i] = ov;
  }
  const double tot = block_sum(loc, red);
  if (threadIdx.x == 0) partial[(int64_t)rhs * gridDim.x + blockIdx.x] = tot;
}

// partial Re<a, b1>, Re<a, b2> (b2 nullable)
template <typename C>
__global__ void __launch_bounds__(256)
k_dot2(const C* a, const C* b1, const C* b2, int64_t n, double* partial1, double* partial2, const int* mask) {
  __shared__ double red[16];
  using O = ChunkOps<C>;
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  const int64_t off = (int64_t)rhs * n;
  a += off;
  b1 += off;
  if (b2) b2 += off;
  double l1 = 0, l2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const C av = a[i], bv = b1[i];
#pragma unroll
    for (int k = 0; k < O::n; ++k) l1 += (double)O::get(av, k) * (double)O::get(bv, k);
    if (b2) {
      const C cv = b2[i];
#pragma unroll
      for (int k = 0; k < O::n; ++k) l2 += (double)O::get(av, k) * (double)O::get(cv, k);
    }
  }
  const int64_t pi = (int64_t)rhs * gridDim.x + blockIdx.x;
  double t1 = block_sum(l1, red);
  if (threadIdx.x == 0) partial1[pi] = t1;
  if (b2) {
    double t2 = block_sum(l2, red);
    if (threadIdx.x == 0) partial2[pi] = t2;
  }
}

// Mixed-precision helpers.  An FP32 chunk j of 5D site i holds complex
// numbers 2j and 2j+1 of that site; in FP64 they are chunks 2j and 2j+1.
// Both layouts use stride n5 (chunks per chunk-array).

// reliable update residual: r64 = b - Ax (when given) ; partial |r64|^2 ; r_lo = (float) r64 when given
__global__ void __launch_bounds__(256)
k_residual64(const double2* b, const double2* Ax, double2* r64, float4* r_lo, int64_t n5, double* partial,
             const int* mask) {
  __shared__ double red[16];
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  b += (int64_t)rhs * 12 * n5;
  Ax += (int64_t)rhs * 12 * n5;
  if (r64) r64 += (int64_t)rhs * 12 * n5;
  if (r_lo) r_lo += (int64_t)rhs * 6 * n5;
  double loc = 0;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < 6 * n5; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = f / n5, i = f - j * n5;
    const int64_t ia = 2 * j * n5 + i, ib = ia + n5;
    const double2 b0 = b[ia], b1 = b[ib], a0 = Ax[ia], a1 = Ax[ib];
    const double2 o0 = make_double2(b0.x - a0.x, b0.y - a0.y), o1 = make_double2(b1.x - a1.x, b1.y - a1.y);
    if (r64) {
      r64[ia] = o0;
      r64[ib] = o1;
    }
    loc += o0.x * o0.x + o0.y * o0.y + o1.x * o1.x + o1.y * o1.y;
    if (r_lo) r_lo[f] = make_float4((float)o0.x, (float)o0.y, (float)o1.x, (float)o1.y);
  }
  const double tot = block_sum(loc, red);
  if (threadIdx.x == 0) partial[(int64_t)rhs * gridDim.x + blockIdx.x] = tot;
}

// x64 += x_lo ; x_lo = 0
__global__ void k_accum_lo(double2* x64, float4* xlo, int64_t n5, const int* mask) {
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  x64 += (int64_t)rhs * 12 * n5;
  xlo += (int64_t)rhs * 6 * n5;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < 6 * n5; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = f / n5, i = f - j * n5;
    const int64_t ia = 2 * j * n5 + i, ib = ia + n5;
    const float4 v = xlo[f];
    double2 a = x64[ia], c = x64[ib];
    a.x += v.x; a.y += v.y; c.x += v.z; c.y += v.w;
    x64[ia] = a;
    x64[ib] = c;
    xlo[f] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// FP64 field -> FP32 field
__global__ void k_f64_to_f32(const double2* a, float4* o, int64_t n5, const int* mask) {
  const int rhs = blockIdx.y;
  if (mask && mask[rhs] == 0) return;
  a += (int64_t)rhs * 12 * n5;
  o += (int64_t)rhs * 6 * n5;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < 6 * n5; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = f / n5, i = f - j * n5;
    const double2 u = a[2 * j * n5 + i], v = a[(2 * j + 1) * n5 + i];
    o[f] = make_float4((float)u.x, (float)u.y, (float)v.x, (float)v.y);
  }
}

void cg_update(hipStream_t st, Prec p, void* x, const void* pv, const void* r, const void* q, void* rn, int64_t nreal,
               const double* scal, int alpha_slot, double* partial, int64_t nblocks, const Batch& bt) {
  const dim3 grid((unsigned)nblocks, (unsigned)bt.n);
  if (p == Prec::F32)
    hipLaunchKernelGGL(k_cg_update<float4>, grid, dim3(256), 0, st, (float4*)x, (const float4*)pv, (const float4*)r,
                       (const float4*)q, (float4*)rn, nreal / 4, scal, alpha_slot, partial, bt.mask);
  else
    hipLaunchKernelGGL(k_cg_update<double2>, grid, dim3(256), 0, st, (double2*)x, (const double2*)pv,
                       (const double2*)r, (const double2*)q, (double2*)rn, nreal / 2, scal, alpha_slot, partial,
                       bt.mask);
  LAUNCH_CHECK();
}

void dot2(hipStream_t st, Prec p, const void* a, const void* b1, const void* b2, int64_t nreal, double* partial1,
          double* partial2, int64_t nblocks, const Batch& bt) {
  const dim3 grid((unsigned)nblocks, (unsigned)bt.n);
  if (p == Prec::F32)
    hipLaunchKernelGGL(k_dot2<float4>, grid, dim3(256), 0, st, (const float4*)a, (const float4*)b1,
                       (const float4*)b2, nreal / 4, partial1, partial2, bt.mask);
  else
    hipLaunchKernelGGL(k_dot2<double2>, grid, dim3(256), 0, st, (const double2*)a, (const double2*)b1,
                       (const double2*)b2, nreal / 2, partial1, partial2, bt.mask);
  LAUNCH_CHECK();
}

void residual64(hipStream_t st, const double* b, const double* Ax, double* r64, float* r_lo, int64_t n5,
                double* partial, int64_t nblocks, const Batch& bt) {
  hipLaunchKernelGGL(k_residual64, dim3((unsigned)nblocks, (unsigned)bt.n), dim3(256), 0, st, (const double2*)b,
                     (const double2*)Ax, (double2*)r64, (float4*)r_lo, n5, partial, bt.mask);
  LAUNCH_CHECK();
}

void accum_lo(hipStream_t st, double* x64, float* xlo, int64_t n5, const Batch& bt) {
  hipLaunchKernelGGL(k_accum_lo, dim3(2048, (unsigned)bt.n), dim3(256), 0, st, (double2*)x64, (float4*)xlo, n5,
                     bt.mask);
  LAUNCH_CHECK();
}

void f64_to_f32(hipStream_t st, const double* a, float* b, int64_t n5, const Batch& bt) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(2048, (unsigned)bt.n), dim3(256), 0, st, (const double2*)a, (float4*)b, n5,
                     bt.mask);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- scalars
//
// k_finish reduces one or two partial arrays in a fixed order and updates the
// solver scalars in `scal` (slots in kernels.h); one workgroup per RHS:
//   FIN_STORE : scal[slot] = S1
//   FIN_ALPHA : scal[PAP] = S1, alpha = rho / pAp
//   FIN_RHO   : scal[RHO] = S1
//   FIN_BETA_FR: rz = S1, beta = rz / rho, rho = rz
//   FIN_BETA_PR: rz = S1, rzold = S2, beta = (rz - rzold) / rho, rho = rz
// With p1 null, S1 = scal[slot].
__global__ void k_finish(const double* p1, const double* p2, int64_t n, double* scal, int mode, int slot,
                         const int* mask) {
  __shared__ double red[16];
  const int rhs = blockIdx.x;
  if (mask && mask[rhs] == 0) return;
  scal += (int64_t)rhs * SLOT_COUNT;
  if (p1) p1 += (int64_t)rhs * n;
  if (p2) p2 += (int64_t)rhs * n;
  double v1 = 0, v2 = 0;
  if (p1)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      v1 += p1[i];
      if (p2) v2 += p2[i];
    }
  const double r1 = block_sum(v1, red);
  const double s1 = p1 ? r1 : scal[slot];
  const double s2 = p2 ? block_sum(v2, red) : 0.0;
  if (threadIdx.x != 0) return;
  switch (mode) {
    case FIN_STORE: scal[slot] = s1; break;
    case FIN_ALPHA: scal[SLOT_PAP] = s1; scal[SLOT_ALPHA] = scal[SLOT_RHO] / s1; break;
    case FIN_RHO: scal[SLOT_RHO] = s1; break;
    case FIN_BETA_FR:
      scal[SLOT_RZ] = s1;
      scal[SLOT_BETA] = s1 / scal[SLOT_RHO];
      scal[SLOT_RHO] = s1;
      break;
    case FIN_BETA_PR:
      scal[SLOT_RZ] = s1;
      scal[SLOT_RZOLD] = s2;
      scal[SLOT_BETA] = (s1 - s2) / scal[SLOT_RHO];
      scal[SLOT_RHO] = s1;
      break;
  }
}

void finish(hipStream_t st, const double* p1, const double* p2, int64_t n, double* scal, int mode, int slot,
            const Batch& bt) {
  hipLaunchKernelGGL(k_finish, dim3((unsigned)bt.n), dim3(1024), 0, st, p1, p2, n, scal, mode, slot, bt.mask);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- per-RHS control
//
// One thread per RHS.  The decisions are those of the outer PCG with
// reliable updates (Sec. 3.2): the iterated residual triggers a reliable
// update when it falls below delta times the largest residual since the last
// one, on convergence, or at the iteration limit; convergence is decided on
// the true residual that the update recomputes.

__global__ void k_ctl_init(Ctl c, double* scal, int n, int* join) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || (join && !join[r])) return;
  double* sc = scal + (int64_t)r * SLOT_COUNT;
  const double bn2 = sc[SLOT_TMP];
  c.iters[r] = 0;
  c.rus[r] = 0;
  c.precs[r] = 0;
  c.ru[r] = 0;
  c.bzero[r] = 0;
  c.bnorm[r] = 0;
  c.rmax[r] = 0;
  c.rr[r] = 0;
  if (!isfinite(bn2)) {
    c.status[r] = RHS_BREAKDOWN;
    c.active[r] = 0;
  } else if (bn2 == 0.0) {
    c.status[r] = RHS_OK;
    c.active[r] = 0;
    c.bzero[r] = 1;
  } else {
    c.status[r] = RHS_RUNNING;
    c.active[r] = 1;
    c.bnorm[r] = sqrt(bn2);
  }
  sc[SLOT_TMP] = 0.0;   // beta of the first search direction p = z + 0 p
  if (join) join[r] = c.active[r];   // the start-up kernels that follow run on these RHS only
}

__global__ void k_ctl_start(Ctl c, const double* scal, int n, int has_x0, const int* join) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || !c.active[r] || (join && !join[r])) return;
  const double bn = c.bnorm[r];
  const double rr = has_x0 ? scal[(int64_t)r * SLOT_COUNT + SLOT_R64] : bn * bn;
  c.rr[r] = has_x0 ? rr : bn * bn;
  c.rmax[r] = has_x0 ? sqrt(rr) : bn;
  c.precs[r] = 1;   // the preconditioner application before the first iteration
}

__global__ void k_ctl_iterate(Ctl c, const double* scal, int n, CtlParams p) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || !c.active[r]) return;
  const double* sc = scal + (int64_t)r * SLOT_COUNT;
  const double pap = sc[SLOT_PAP], rr = sc[SLOT_RR];
  c.iters[r] += 1;
  c.rr[r] = rr;
  if (!(pap > 0.0) || !isfinite(pap) || !isfinite(rr)) {
    c.status[r] = RHS_BREAKDOWN;
    c.active[r] = 0;
    c.ru[r] = 0;
    return;
  }
  const double rn = sqrt(rr);
  if (rn > c.rmax[r]) c.rmax[r] = rn;
  const bool conv = rn <= p.tol * c.bnorm[r];
  const bool last = c.iters[r] >= p.maxiter;
  c.ru[r] = (conv || last || (p.delta > 0 && rn < p.delta * c.rmax[r])) ? 1 : 0;
}

__global__ void __launch_bounds__(1024) k_ctl_after_update(Ctl c, double* scal, int n, CtlParams p) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    if (!c.active[r]) continue;
    double* sc = scal + (int64_t)r * SLOT_COUNT;
    if (c.ru[r]) {
      const double rr = sc[SLOT_R64];
      c.ru[r] = 0;
      c.rus[r] += 1;
      c.rr[r] = rr;
      sc[SLOT_RR] = rr;   // the current |r|^2 is the true one
      c.rmax[r] = sqrt(rr);
      if (sqrt(rr) <= p.tol * c.bnorm[r]) {
        c.status[r] = RHS_OK;
        c.active[r] = 0;
        continue;
      }
      if (!isfinite(rr)) {
        c.status[r] = RHS_BREAKDOWN;
        c.active[r] = 0;
        continue;
      }
    }
    if (c.iters[r] >= p.maxiter) {
      c.status[r] = RHS_NOT_CONVERGED;
      c.active[r] = 0;
      continue;
    }
    c.precs[r] += 1;
    atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *c.nactive = cnt;
}

static unsigned ctl_blocks(int n) { return (unsigned)((n + 255) / 256); }

void ctl_init(hipStream_t st, const Ctl& c, double* scal, int n, int* join) {
  hipLaunchKernelGGL(k_ctl_init, dim3(ctl_blocks(n)), dim3(256), 0, st, c, scal, n, join);
  LAUNCH_CHECK();
}

void ctl_start(hipStream_t st, const Ctl& c, const double* scal, int n, bool has_x0, const int* join) {
  hipLaunchKernelGGL(k_ctl_start, dim3(ctl_blocks(n)), dim3(256), 0, st, c, scal, n, has_x0 ? 1 : 0, join);
  LAUNCH_CHECK();
}

void ctl_iterate(hipStream_t st, const Ctl& c, const double* scal, int n, const CtlParams& p) {
  hipLaunchKernelGGL(k_ctl_iterate, dim3(ctl_blocks(n)), dim3(256), 0, st, c, scal, n, p);
  LAUNCH_CHECK();
}

void ctl_after_update(hipStream_t st, const Ctl& c, double* scal, int n, const CtlParams& p) {
  hipLaunchKernelGGL(k_ctl_after_update, dim3(1), dim3(1024), 0, st, c, scal, n, p);
  LAUNCH_CHECK();
}

}  // namespace mspcg
