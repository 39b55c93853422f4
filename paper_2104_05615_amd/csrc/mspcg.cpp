// Host side of the library: the handle, the fifth-dimension matrices, the
// subdomain region tables, the operator chains, the outer solver and the
// C ABI declared in include/mspcg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "mspcg.h"

using namespace mspcg;

// ==========================================================================
// errors
// ==========================================================================
namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
  mspcg_status code;
  Error(mspcg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) {                                                                         \
      throw Error(e_ == hipErrorOutOfMemory ? MSPCG_ERR_OOM : MSPCG_ERR_HIP,                        \
                  std::string(#x) + ": " + hipGetErrorString(e_));                                  \
    }                                                                                               \
  } while (0)

// Graph capture and the runtime calls that may act on every stream of the
// device (allocation and release, stream and pinned-memory creation and
// destruction, device-wide synchronization) never overlap, also across
// threads and handles: captures hold the shared side of this lock, such
// calls the exclusive side.  A thread that is capturing allocates nothing.
std::shared_mutex g_capture_gate;
// Calls that size workspaces or launch kernels hold this shared for their
// duration; mspcg_set_mfma, which changes the epilogue engine and with it the
// sites per workgroup that every launch and partial buffer is sized for,
// takes it exclusively, so it waits until no such call is running.
std::shared_mutex g_engine_gate;
thread_local bool tl_capturing = false;

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  bool owned = true;   // false: a view into the static workspace (never freed)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void ensure(size_t bytes) {
    if (bytes <= n && p) return;
    if (!owned) throw Error(MSPCG_ERR_HIP, "workspace view cannot grow");
    if (tl_capturing) throw Error(MSPCG_ERR_HIP, "workspace growth during graph capture");
    std::unique_lock<std::shared_mutex> lk(g_capture_gate);
    free_locked();
    HIPCHK(hipMalloc(&p, bytes ? bytes : 16));
    n = bytes;
  }
  void release() {
    if (!p) return;
    if (!owned) {   // a view: nothing to free
      p = nullptr;
      n = 0;
      return;
    }
    std::unique_lock<std::shared_mutex> lk(g_capture_gate);
    free_locked();
  }
  void free_locked() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { release(); }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

Prec to_prec(mspcg_prec p) {
  switch (p) {
    case MSPCG_FP64: return Prec::F64;
    case MSPCG_FP32: return Prec::F32;
    case MSPCG_FP16: return Prec::F16;
    case MSPCG_BF16: return Prec::BF16;
    case MSPCG_INT8: return Prec::I8;
  }
  throw Error(MSPCG_ERR_INVALID_ARG, "unknown precision");
}

int64_t round16(int64_t b) { return (b + 15) / 16 * 16; }

size_t chunk_bytes(Prec p) { return p == Prec::F64 ? 192 : p == Prec::F32 ? 96 : p == Prec::I8 ? 24 : 48; }
bool scaled(Prec p) { return p == Prec::F16 || p == Prec::BF16 || p == Prec::I8; }

// --------------------------------------------------------------------------
// fifth-dimension matrices, per chirality (0: P+, 1: P-), Ls x Ls, real.
// P~ on P+ shifts s -> s+1 with psi(-1) = -mf psi(Ls-1); on P- it is the
// transpose.  M5 = a0 + a1 P~, M_phi = -(b + c P~)/2 (Sec. 2.2 with the
// Mobius construction).  M5^-1 from the geometric series of (a0 + a1 S)^-1
// with S^Ls = -mf.
// --------------------------------------------------------------------------
enum MatId {
  MAT_MPHI = 0,     // M_phi
  MAT_Q,            // M_phi M5^-1
  MAT_NEG_M5INV,    // -M5^-1
  MAT_M5INV_T,      // M5^-dag
  MAT_QT,           // (M_phi M5^-1)^dag
  MAT_M5_T,         // M5^dag
  MAT_NEG_MPHI_T,   // -M_phi^dag
  MAT_M5,
  MAT_M5INV,
  MAT_NEG_M5INVT_M5INV,   // -M5^-dag M5^-1
  MAT_COUNT
};

struct Mats {
  int Ls;
  std::vector<double> m;  // [MAT_COUNT][2][Ls][Ls]
  double* at(int id, int chi) { return m.data() + ((size_t)id * 2 + chi) * Ls * Ls; }
};

Mats build_mats(int Ls, double b, double c, double M5, double mf) {
  Mats M;
  M.Ls = Ls;
  M.m.assign((size_t)MAT_COUNT * 2 * Ls * Ls, 0.0);
  const double a0 = b * (4.0 - M5) + 1.0, a1 = c * (4.0 - M5) - 1.0;
  if (a0 == 0.0) throw Error(MSPCG_ERR_INVALID_ARG, "M5 operator singular: b(4-M5)+1 = 0");
  const double kap = -a1 / a0;
  const double den = a0 * (1.0 + mf * std::pow(kap, Ls));
  if (den == 0.0 || !std::isfinite(den)) throw Error(MSPCG_ERR_INVALID_ARG, "M5 operator singular");
  std::vector<double> S(Ls * Ls, 0.0), Minv(Ls * Ls), Mp(Ls * Ls), M5m(Ls * Ls), Q(Ls * Ls);
  for (int s = 1; s < Ls; ++s) S[s * Ls + s - 1] = 1.0;
  S[0 * Ls + Ls - 1] = -mf;
  for (int s = 0; s < Ls; ++s)
    for (int t = 0; t < Ls; ++t) {
      Minv[s * Ls + t] = s >= t ? std::pow(kap, s - t) / den : -mf * std::pow(kap, s - t + Ls) / den;
      const double id = s == t ? 1.0 : 0.0;
      Mp[s * Ls + t] = -0.5 * (b * id + c * S[s * Ls + t]);
      M5m[s * Ls + t] = a0 * id + a1 * S[s * Ls + t];
    }
  for (int s = 0; s < Ls; ++s)
    for (int t = 0; t < Ls; ++t) {
      double acc = 0;
      for (int u = 0; u < Ls; ++u) acc += Mp[s * Ls + u] * Minv[u * Ls + t];
      Q[s * Ls + t] = acc;
    }
  // chirality 0 uses the matrices as built; chirality 1 their transposes
  auto put = [&](int id, const std::vector<double>& A, double sign, bool dag) {
    for (int chi = 0; chi < 2; ++chi) {
      double* o = M.at(id, chi);
      const bool tr = (chi == 1) != dag;
      for (int s = 0; s < Ls; ++s)
        for (int t = 0; t < Ls; ++t) o[s * Ls + t] = sign * (tr ? A[t * Ls + s] : A[s * Ls + t]);
    }
  };
  put(MAT_MPHI, Mp, 1.0, false);
  put(MAT_Q, Q, 1.0, false);
  put(MAT_NEG_M5INV, Minv, -1.0, false);
  put(MAT_M5INV_T, Minv, 1.0, true);
  put(MAT_QT, Q, 1.0, true);
  put(MAT_M5_T, M5m, 1.0, true);
  put(MAT_NEG_MPHI_T, Mp, -1.0, true);
  put(MAT_M5, M5m, 1.0, false);
  put(MAT_M5INV, Minv, 1.0, false);
  for (int chi = 0; chi < 2; ++chi) {
    const double* At = M.at(MAT_M5INV_T, chi);
    const double* B = M.at(MAT_M5INV, chi);
    double* o = M.at(MAT_NEG_M5INVT_M5INV, chi);
    for (int s = 0; s < Ls; ++s)
      for (int t = 0; t < Ls; ++t) {
        double acc = 0;
        for (int u = 0; u < Ls; ++u) acc += At[s * Ls + u] * B[u * Ls + t];
        o[s * Ls + t] = -acc;
      }
  }
  return M;
}

// --------------------------------------------------------------------------
// subdomain regions (shared by all subdomains, which are translates)
// --------------------------------------------------------------------------
struct Region {
  std::vector<short4> coords;
  std::vector<int> index;   // box index -> region index or -1
};

struct HostTables {
  Region C, N1, N2;                                    // C even, N1 odd, N2 even
  std::vector<int> nbr1, nbr2, nbr3, nbr4;             // h1: N1<-C, h2: N2<-N1, h3: N1<-N2, h4: C<-N1
  std::vector<int> wmap2, wmap4;                       // N2 -> C, C -> N2
};

bool tiling_valid(const int* dims, const int* sub, std::string& why) {
  for (int m = 0; m < 4; ++m) {
    if (sub[m] <= 0 || sub[m] % 2 || dims[m] % sub[m]) {
      why = "subdomain extents must be even and divide the lattice";
      return false;
    }
    if (sub[m] < dims[m] && dims[m] - sub[m] < 4) {
      why = "a partitioned direction needs at least 4 sites outside the subdomain";
      return false;
    }
  }
  return true;
}

// 32-bit addressing limits of the kernels.  Fields and link arrays are
// read through buffer resources whose range (num_records) and per-lane byte
// offsets are 32-bit, lattice coordinates are recovered from a 32-bit
// lexicographic index by multiply-high division (exact below 2^31), and 5D
// indices of one right-hand side are 32-bit.  Every array of one RHS must
// therefore stay below 4 GiB and the 4D volume below 2^31 sites.
constexpr uint64_t kMaxArrayBytes = (1ull << 32) - 1;

// checks what is known: dims always; Ls > 0: full-lattice FP64 fields (the
// reliable updates always hold some); nN2 > 0 with Ls > 0: the largest
// subdomain region field of inner storage `inner`
void check_limits(const int* dims, int Ls, int64_t nsub, int64_t nN2, int inner) {
  const uint64_t V = (uint64_t)dims[0] * dims[1] * dims[2] * dims[3];
  if (V >= (1ull << 31)) throw Error(MSPCG_ERR_INVALID_ARG, "lattice volume must be below 2^31 sites");
  const uint64_t vh = V / 2;
  if (vh * 4 * 10 * 16 * 2 > kMaxArrayBytes)
    throw Error(MSPCG_ERR_INVALID_ARG, "FP64 gauge field of this lattice exceeds 4 GiB (32-bit buffer addressing)");
  if (Ls > 0 && vh * (uint64_t)Ls * 192 > kMaxArrayBytes)
    throw Error(MSPCG_ERR_INVALID_ARG, "an FP64 field of this lattice and Ls exceeds 4 GiB (32-bit buffer addressing)");
  if (Ls > 0 && nN2 > 0 && inner >= 0) {
    const uint64_t cb = inner == MSPCG_FP64 ? 192 : inner == MSPCG_FP32 ? 96 : inner == MSPCG_INT8 ? 24 : 48;
    if ((uint64_t)nsub * (uint64_t)nN2 * (uint64_t)Ls * cb > kMaxArrayBytes)
      throw Error(MSPCG_ERR_INVALID_ARG,
                  "a subdomain region field of this tiling, Ls and inner precision exceeds 4 GiB (32-bit buffer addressing)");
  }
}

HostTables build_tables(const int* dims, const int* sub) {
  bool part[4];
  int lo[4], ext[4];
  for (int m = 0; m < 4; ++m) {
    part[m] = sub[m] < dims[m];
    lo[m] = part[m] ? -2 : 0;
    ext[m] = part[m] ? sub[m] + 4 : dims[m];
  }
  const int64_t box = (int64_t)ext[0] * ext[1] * ext[2] * ext[3];
  auto box_index = [&](const int* l) {
    return ((int64_t)(l[3] - lo[3]) * ext[2] + (l[2] - lo[2])) * ext[1] * ext[0] + (int64_t)(l[1] - lo[1]) * ext[0] +
           (l[0] - lo[0]);
  };
  HostTables H;
  H.C.index.assign(box, -1);
  H.N1.index.assign(box, -1);
  H.N2.index.assign(box, -1);
  int l[4];
  for (l[3] = lo[3]; l[3] < lo[3] + ext[3]; ++l[3])
    for (l[2] = lo[2]; l[2] < lo[2] + ext[2]; ++l[2])
      for (l[1] = lo[1]; l[1] < lo[1] + ext[1]; ++l[1])
        for (l[0] = lo[0]; l[0] < lo[0] + ext[0]; ++l[0]) {
          int dist = 0;
          for (int m = 0; m < 4; ++m)
            if (part[m]) dist += std::max(0, std::max(-l[m], l[m] - (sub[m] - 1)));
          const int par = (l[0] + l[1] + l[2] + l[3]) & 1;
          const int64_t bi = box_index(l);
          const short4 c = make_short4((short)l[0], (short)l[1], (short)l[2], (short)l[3]);
          if (dist == 0 && par == 0) { H.C.index[bi] = (int)H.C.coords.size(); H.C.coords.push_back(c); }
          if (dist <= 1 && par == 1) { H.N1.index[bi] = (int)H.N1.coords.size(); H.N1.coords.push_back(c); }
          if (dist <= 2 && par == 0) { H.N2.index[bi] = (int)H.N2.coords.size(); H.N2.coords.push_back(c); }
        }
  // Order N1 and N2 by which neighbours their producing hop finds in its
  // input region (h1: N1 <- C, h2: N2 <- N1; stable, so box order within a
  // pattern): sites at the region's rim have one or two of the eight, and a
  // wavefront then holds sites of one pattern and skips the absent terms.
  auto wrap_or_outside = [&](int* n, int mu) {
    if (!part[mu]) n[mu] = (n[mu] + dims[mu]) % dims[mu];
    else if (n[mu] < lo[mu] || n[mu] >= lo[mu] + ext[mu]) return true;
    return false;
  };
  auto presence = [&](const short4& c, const Region& in) {
    int mask = 0;
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        int n[4] = {c.x, c.y, c.z, c.w};
        n[mu] += dir == 0 ? 1 : -1;
        if (!wrap_or_outside(n, mu) && in.index[box_index(n)] >= 0) mask |= 1 << (2 * mu + dir);
      }
    return mask;
  };
  auto reorder = [&](Region& R, const Region& in) {
    const size_t n = R.coords.size();
    std::vector<int> key(n), order(n);
    for (size_t j = 0; j < n; ++j) {
      key[j] = presence(R.coords[j], in);
      order[j] = (int)j;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<short4> coords(n);
    for (size_t j = 0; j < n; ++j) {
      coords[j] = R.coords[order[j]];
      const short4 c = coords[j];
      int l2[4] = {c.x, c.y, c.z, c.w};
      R.index[box_index(l2)] = (int)j;
    }
    R.coords.swap(coords);
  };
  reorder(H.N1, H.C);
  reorder(H.N2, H.N1);

  auto neighbours = [&](const Region& out, const Region& in) {
    std::vector<int> nb(out.coords.size() * 8, -1);
    for (size_t j = 0; j < out.coords.size(); ++j) {
      const short4 c = out.coords[j];
      for (int mu = 0; mu < 4; ++mu)
        for (int dir = 0; dir < 2; ++dir) {
          int n[4] = {c.x, c.y, c.z, c.w};
          n[mu] += dir == 0 ? 1 : -1;
          if (wrap_or_outside(n, mu)) continue;
          nb[j * 8 + 2 * mu + dir] = in.index[box_index(n)];
        }
    }
    return nb;
  };
  H.nbr1 = neighbours(H.N1, H.C);
  H.nbr2 = neighbours(H.N2, H.N1);
  H.nbr3 = neighbours(H.N1, H.N2);
  H.nbr4 = neighbours(H.C, H.N1);
  H.wmap2.resize(H.N2.coords.size());
  for (size_t j = 0; j < H.N2.coords.size(); ++j) {
    const short4 c = H.N2.coords[j];
    int l2[4] = {c.x, c.y, c.z, c.w};
    H.wmap2[j] = H.C.index[box_index(l2)];
  }
  H.wmap4.resize(H.C.coords.size());
  for (size_t j = 0; j < H.C.coords.size(); ++j) {
    const short4 c = H.C.coords[j];
    int l2[4] = {c.x, c.y, c.z, c.w};
    H.wmap4[j] = H.N2.index[box_index(l2)];
  }
  return H;
}

struct EventPair {
  hipEvent_t a, b;
};

struct CBSession;   // an open continuous-batching session (defined with the batched solver)
}  // namespace

void mspcg::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

// ==========================================================================
// the handle
// ==========================================================================
struct mspcg_ctx {
  int dims[4];
  int device;
  Lattice lat;
  bool hip_ready = false;
  hipStream_t stream = nullptr;

  // device links, FP64 and FP32 layouts; shared between handles on one field
  struct GaugeStore {
    DevBuf g64, g32, g16;
  };
  std::shared_ptr<GaugeStore> gs;
  bool have_gauge = false;

  int Ls = 0;
  double b = 0, c = 0, M5 = 0, mf = 0;
  bool have_params = false;
  DevBuf mats64, mats32;

  int sub[4] = {0, 0, 0, 0};
  bool have_tiling = false;
  int nsub = 0, nblk[4] = {1, 1, 1, 1};
  int nC = 0, nN1 = 0, nN2 = 0;
  DevBuf tb_origin, tb_cC, tb_cN1, tb_cN2, tb_nbr1, tb_nbr2, tb_nbr3, tb_nbr4, tb_w2, tb_w4;

  mspcg_solver_params sp;
  bool have_solver = false;

  std::map<std::string, std::unique_ptr<DevBuf>> ws;
  // bumped whenever a workspace is allocated or moves: a captured graph
  // holds the addresses of the generation it was captured in
  uint64_t ws_gen = 0;
  // Static-workspace mode (mspcg_apply_device_noalloc): while `arena` is set,
  // buf() hands out views of the device's static workspace, bump-allocated
  // per call, instead of growing the handle's own buffers.
  void* scratch = nullptr;   // this device's static workspace (resolved in ensure_hip)
  struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
  } arena;
  std::map<std::string, std::unique_ptr<DevBuf>> arena_ws;
  // open continuous-batching session (mspcg_cb_*), or null
  std::shared_ptr<CBSession> cb;
  // |r_k| / |b| of the last single-RHS solve, k = 0, 1, ... (iterated
  // residuals), and <p_k, A p_k> / |b|^2 of its outer iterations
  std::vector<double> history, history_pap;
  double* h_scal = nullptr;   // pinned
  int* h_flag = nullptr;      // pinned: RHS still active, one slot per graph replay in flight
  // pinned bounce buffer: every transfer between host memory the caller owns
  // (pageable) and the device goes through it, in chunks, on this handle's
  // stream -- no asynchronous copy ever reads or writes pageable memory
  char* h_bounce = nullptr;
  static constexpr size_t kBounce = 8u << 20;

  // reduced-Ls preconditioner (Sec. 3.3): z = (T^dag Mhat^-1 T + mu) r.  Lh = 0: off.
  int Lh = 0;
  double bh = 0, ch = 0, mu_red = 0;
  std::vector<double> Tm;                // host, complex interleaved [Lh][4][Ls][4]
  DevBuf T64, T32, Td64, Td32;           // T and T^dag, double2 / float2
  DevBuf D64, D32, Dd64, Dd32;           // a training search direction d and d^dag
  std::unique_ptr<mspcg_ctx> red;        // context at Lh: this handle's gauge field and tiling
  bool red_dirty = true;

  bool profiling = false;
  bool graphs = true;              // batched solves replay captured graphs
  int log_every = 0;               // progress line to stderr every this many outer iterations (0: none)
  int64_t capture_fallbacks = 0;   // batched solves whose graph capture failed (ran eagerly)
  std::vector<EventPair> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_log;   // (kind, pool index)

  mspcg_ctx(const int32_t* d, int dev) {
    for (int m = 0; m < 4; ++m) dims[m] = d[m];
    device = dev;
    lat = make_lattice(d[0], d[1], d[2], d[3]);
    sp.tol = 1e-10;
    sp.maxiter = 10000;
    sp.inner_iters = 6;
    sp.inner_prec = MSPCG_FP16;
    sp.outer_prec = MSPCG_FP32;
    sp.reliable_delta = 0.1;
    sp.beta_rule = 0;
    sp.use_precond = 1;
  }
  ~mspcg_ctx() {
    if (hip_ready) {
      (void)hipSetDevice(device);
      (void)hipStreamSynchronize(stream);
      cb.reset();
      ws.clear();
      std::unique_lock<std::shared_mutex> lk(g_capture_gate);
      for (auto& e : ev_pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
      }
      if (h_scal) (void)hipHostFree(h_scal);
      if (h_flag) (void)hipHostFree(h_flag);
      if (h_bounce) (void)hipHostFree(h_bounce);
      (void)hipStreamDestroy(stream);
    }
  }

  void ensure_hip() {
    HIPCHK(hipSetDevice(device));
    if (hip_ready) return;
    std::unique_lock<std::shared_mutex> lk(g_capture_gate);
    HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void**)&h_scal, SLOT_COUNT * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&h_flag, 4 * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&h_bounce, kBounce, hipHostMallocDefault));
    scratch = scratch_device_ptr();   // device current: its copy of the static workspace
    hip_ready = true;
  }

  // host (pageable) -> device and back through the pinned bounce buffer, in
  // order on stream st; both return when the copy is complete
  void upload(void* dev, const void* host, size_t bytes, hipStream_t st) {
    for (size_t o = 0; o < bytes; o += kBounce) {
      const size_t n = std::min(kBounce, bytes - o);
      HIPCHK(hipStreamSynchronize(st));   // the previous chunk has left the buffer
      std::memcpy(h_bounce, (const char*)host + o, n);
      HIPCHK(hipMemcpyAsync((char*)dev + o, h_bounce, n, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
  }
  void download(void* host, const void* dev, size_t bytes, hipStream_t st) {
    for (size_t o = 0; o < bytes; o += kBounce) {
      const size_t n = std::min(kBounce, bytes - o);
      HIPCHK(hipMemcpyAsync(h_bounce, (const char*)dev + o, n, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::memcpy((char*)host + o, h_bounce, n);
    }
    if (bytes == 0) HIPCHK(hipStreamSynchronize(st));
  }

  DevBuf& buf(const std::string& key, size_t bytes) {
    if (arena.base) {
      auto& v = arena_ws[key];
      if (!v) v.reset(new DevBuf());
      v->owned = false;
      if (v->p && v->n >= bytes) return *v;
      const size_t off = (arena.off + 255) & ~size_t(255);
      if (off > arena.cap || bytes > arena.cap - off)
        throw Error(MSPCG_ERR_INVALID_ARG, "workspace of this call exceeds the static workspace (" +
                                               std::to_string(arena.cap >> 20) + " MiB)");
      v->p = arena.base + off;
      v->n = bytes;
      arena.off = off + bytes;
      return *v;
    }
    auto& p = ws[key];
    if (!p) p.reset(new DevBuf());
    void* const before = p->p;
    p->ensure(bytes);
    if (p->p != before) ++ws_gen;
    return *p;
  }

  int64_t n5() const { return lat.vh * Ls; }

  // a field of nsites 4D sites (x Ls), nb right-hand sides one after another
  FieldPtr field(const std::string& key, Prec p, int64_t nsites, int nb = 1) {
    const int64_t n = nsites * Ls;
    FieldPtr f;
    f.prec = p;
    f.stride = n;
    DevBuf& d = buf(key, (size_t)nb * n * chunk_bytes(p));
    f.data = d.p;
    if (scaled(p)) f.scale = buf(key + ".scale", (size_t)round16((int64_t)nb * n * sizeof(float))).as<float>();
    return f;
  }

  const void* mat(Prec p, int id) const {
    const size_t off = (size_t)id * 2 * Ls * Ls;
    if (p == Prec::F64) return mats64.as<double>() + off;
    return mats32.as<float>() + off;
  }
  const void* gauge(Prec p) const { return p == Prec::F64 ? gs->g64.p : gs->g32.p; }
  // links of the subdomain hops: FP16 records for the 16- and 8-bit formats
  const void* gauge_sub(Prec p) const { return scaled(p) ? gs->g16.p : gauge(p); }

  // bytes of the workspaces, matrices and tables this handle holds (not the
  // gauge field)
  int64_t ws_bytes() const {
    int64_t n = (int64_t)mats64.n + (int64_t)mats32.n;
    for (const DevBuf* d : {&tb_origin, &tb_cC, &tb_cN1, &tb_cN2, &tb_nbr1, &tb_nbr2, &tb_nbr3, &tb_nbr4, &tb_w2, &tb_w4})
      n += (int64_t)d->n;
    for (auto& kv : ws) n += kv.second ? (int64_t)kv.second->n : 0;
    n += (int64_t)T64.n + (int64_t)T32.n + (int64_t)Td64.n + (int64_t)Td32.n;
    if (red) n += red->ws_bytes();
    return n;
  }

  double* partial(const std::string& key, int64_t n) { return buf("partial." + key, (size_t)n * sizeof(double)).as<double>(); }
  double* scal(int nb = 1) { return buf("scalars", (size_t)nb * SLOT_COUNT * sizeof(double)).as<double>(); }

  // ---------------------------------------------------------------- launch schedules
  // Tuned workgroup schedules of the hop kernels, per (hop kind, precision,
  // number of RHS); kinds: 0 full-lattice hops of the outer precision,
  // 1 FP64 hops, 2 subdomain hops.  Untuned: one workgroup per item, RHS of
  // one site block adjacent, XCD ranges, and for the full-lattice hops the
  // chunked t sweep with ~640 KB chunks (measured at 16^3x32 and 32^3x64,
  // Ls 12: FP32 outer hops 9 and 13 % faster than the lexicographic order).
  std::map<std::tuple<int, int, int>, Sched> tuned;
  std::map<std::tuple<int, int, int>, double> tuned_us;
  Sched sched(int kind, Prec p, int nrhs) const {
    auto it = tuned.find(std::make_tuple(kind, (int)p, nrhs));
    if (it != tuned.end()) return it->second;
    Sched sc;
    sc.order = nrhs > 1 ? 1 : 0;
    sc.xcd = 1;
    sc.tchunk = kind == 2 ? 0 : 3;
    return sc;
  }

  void invalidate_workspace() {
    if (hip_ready) HIPCHK(hipStreamSynchronize(stream));
    ws.clear();
    red_dirty = true;
  }

  // ---------------------------------------------------------------- reduced-Ls preconditioner
  // T and T^dag in both precisions on the device, from the host copy
  void upload_transform() { upload_matrix(Tm, T64, T32, Td64, Td32); }
  // a complex [Lh][4][Ls][4] matrix and its adjoint, double2 and float2
  void upload_matrix(const std::vector<double>& Tm, DevBuf& T64, DevBuf& T32, DevBuf& Td64, DevBuf& Td32) {
    const int nT = Lh * 4 * Ls * 4;
    std::vector<double> t64(2 * (size_t)nT), d64(2 * (size_t)nT);
    for (int s5 = 0; s5 < Lh; ++s5)
      for (int m = 0; m < 4; ++m)
        for (int t5 = 0; t5 < Ls; ++t5)
          for (int n = 0; n < 4; ++n) {
            const size_t i = ((size_t)(s5 * 4 + m) * Ls + t5) * 4 + n;   // T[s m][t n]
            const size_t j = ((size_t)(t5 * 4 + n) * Lh + s5) * 4 + m;   // T^dag[t n][s m]
            t64[2 * i] = Tm[2 * i];
            t64[2 * i + 1] = Tm[2 * i + 1];
            d64[2 * j] = Tm[2 * i];
            d64[2 * j + 1] = -Tm[2 * i + 1];
          }
    std::vector<float> t32(t64.begin(), t64.end()), d32(d64.begin(), d64.end());
    T64.ensure(t64.size() * sizeof(double));
    Td64.ensure(d64.size() * sizeof(double));
    T32.ensure(t32.size() * sizeof(float));
    Td32.ensure(d32.size() * sizeof(float));
    upload(T64.p, t64.data(), t64.size() * sizeof(double), stream);
    upload(Td64.p, d64.data(), d64.size() * sizeof(double), stream);
    upload(T32.p, t32.data(), t32.size() * sizeof(float), stream);
    upload(Td32.p, d32.data(), d32.size() * sizeof(float), stream);
  }
  const void* Tdev(Prec p, bool dag) const {
    if (p == Prec::F64) return dag ? Td64.p : T64.p;
    return dag ? Td32.p : T32.p;
  }
  const void* Ddev(Prec p, bool dag) const {
    if (p == Prec::F64) return dag ? Dd64.p : D64.p;
    return dag ? Dd32.p : D32.p;
  }
  // the context at Lh (built on first use and after any change of gauge
  // field, Mobius parameters or tiling); its solver parameters follow this one's
  mspcg_ctx* reduced_ctx();

  // partial sums per RHS that the preconditioner writes for the PR dots
  int64_t precond_partials(Prec O, Prec I) {
    if (Lh > 0) return transform_blocks(lat.vh, Lh, Ls, O);
    return (int64_t)nsub * tables(0, I).bps;
  }

  // ---------------------------------------------------------------- profiling
  // profiling kinds below 64 of which every prof_stride-th launch is timed
  // (the whole-preconditioner kind 2 always): the average launch time then
  // comes from a sample at a fraction of the events' cost
  int prof_stride = 1;
  int64_t prof_count[64] = {};
  size_t ev_begin(hipStream_t st, int kind) {
    if (!profiling) return (size_t)-1;
    if (prof_stride > 1 && kind != 2 && kind >= 0 && kind < 64 && prof_count[kind]++ % prof_stride != 0)
      return (size_t)-1;
    if (ev_used == ev_pool.size()) {
      EventPair e;
      HIPCHK(hipEventCreate(&e.a));
      HIPCHK(hipEventCreate(&e.b));
      ev_pool.push_back(e);
    }
    const size_t i = ev_used++;
    HIPCHK(hipEventRecord(ev_pool[i].a, st));
    ev_log.push_back({kind, i});
    return i;
  }
  void ev_end(hipStream_t st, size_t i) {
    if (i == (size_t)-1) return;
    HIPCHK(hipEventRecord(ev_pool[i].b, st));
  }

  // ---------------------------------------------------------------- tables
  SubTables tables(int which, Prec p) const {
    SubTables t;
    std::memset(&t, 0, sizeof(t));
    for (int m = 0; m < 4; ++m) {
      t.sub[m] = sub[m];
      t.dims[m] = dims[m];
      t.nblk[m] = nblk[m];
    }
    const int ns = sites_per_block(Ls, p);
    t.origin = tb_origin.as<short4>();
    switch (which) {
      case 0:   // C (restrict / update / prolong)
        t.coords = tb_cC.as<short4>(); t.nbr = nullptr; t.wmap = nullptr;
        t.n_out = nC; t.n_in = nC; t.n_w = nC; break;
      case 1:   // h1: N1 <- C
        t.coords = tb_cN1.as<short4>(); t.nbr = tb_nbr1.as<int>(); t.wmap = nullptr;
        t.n_out = nN1; t.n_in = nC; t.n_w = nN1; break;
      case 2:   // h2: N2 <- N1, centre field on C
        t.coords = tb_cN2.as<short4>(); t.nbr = tb_nbr2.as<int>(); t.wmap = tb_w2.as<int>();
        t.n_out = nN2; t.n_in = nN1; t.n_w = nC; break;
      case 3:   // h3: N1 <- N2
        t.coords = tb_cN1.as<short4>(); t.nbr = tb_nbr3.as<int>(); t.wmap = nullptr;
        t.n_out = nN1; t.n_in = nN2; t.n_w = nN1; break;
      case 4:   // h4: C <- N1, centre field on N2
        t.coords = tb_cC.as<short4>(); t.nbr = tb_nbr4.as<int>(); t.wmap = tb_w4.as<int>();
        t.n_out = nC; t.n_in = nN1; t.n_w = nN2; break;
    }
    t.bps = (t.n_out + ns - 1) / ns;
    t.fbps = make_fastdiv((uint32_t)t.bps);
    return t;
  }

  // ---------------------------------------------------------------- operators
  // stage: 1..4 for the four hops of A (0 for other uses); profiling kind
  // 20 + stage (FP32/16-bit) or 30 + stage (FP64)
  void hop(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, int out_par, bool dag,
           const Epilogue& epi, int stage = 0, const Batch& bt = Batch()) {
    HopGeometry g;
    g.lat = lat;
    g.out_parity = out_par;
    g.Ls = Ls;
    const size_t e = ev_begin(st, (p == Prec::F64 ? 30 : 20) + stage);
    hop_full(st, p, out, in, w, gauge(p), g, dag, epi, bt, sched(p == Prec::F64 ? 1 : 0, p, bt.n));
    ev_end(st, e);
  }

  Epilogue epi(Prec p, int e0, int e1, bool wid = false, double* dot = nullptr, const FieldPtr* dotf = nullptr) const {
    Epilogue E;
    E.E0 = e0 >= 0 ? mat(p, e0) : nullptr;
    E.E1 = e1 >= 0 ? mat(p, e1) : nullptr;
    E.w_identity = wid;
    E.dot_partial = dot;
    E.dotf = dotf;
    return E;
  }

  // A = D^dag D on p, given t0 = M_phi p (eq. detail, four hops):
  //   a = Q D^w t0,  c = M5^-dag p - M5^-dag M5^-1 D^w a  (= M5^-dag D p),
  //   e = Q^dag D^w^dag c,  out = M5^dag c - M_phi^dag D^w^dag e  (= D^dag D p).
  // t0 is dead after the first hop and a after the second: c is written over
  // t0 and e over a, so the chain needs one scratch field (t0 is clobbered).
  // dot_partial gets <p, A p> per block of the last hop.
  void A_from_t0(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const FieldPtr& t0,
                 const std::string& tag, double* dot_partial, const Batch& bt = Batch()) {
    FieldPtr a = field(tag + ".a", p, lat.vh, bt.n), c = t0, e = a;
    hop(st, p, a, t0, nullptr, 1, false, epi(p, -1, MAT_Q), 1, bt);
    hop(st, p, c, a, &in, 0, false, epi(p, MAT_M5INV_T, MAT_NEG_M5INVT_M5INV), 2, bt);
    hop(st, p, e, c, nullptr, 1, true, epi(p, -1, MAT_QT), 3, bt);
    hop(st, p, out, e, &c, 0, true, epi(p, MAT_M5_T, MAT_NEG_MPHI_T, false, dot_partial, &in), 4, bt);
  }

  void A_op(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const std::string& tag,
            double* norm_partial, const Batch& bt = Batch()) {
    FieldPtr t0 = field(tag + ".t0", p, lat.vh, bt.n);
    apply5_full(st, p, t0, in, mat(p, MAT_MPHI), lat.vh, Ls, nullptr, bt);
    A_from_t0(st, p, out, in, t0, tag, norm_partial, bt);
  }

  void D_op(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const std::string& tag) {
    FieldPtr t0 = field(tag + ".t0", p, lat.vh), a = field(tag + ".a", p, lat.vh);
    apply5_full(st, p, t0, in, mat(p, MAT_MPHI), lat.vh, Ls, nullptr);
    hop(st, p, a, t0, nullptr, 1, false, epi(p, -1, MAT_Q));
    hop(st, p, out, a, &in, 0, false, epi(p, -1, MAT_NEG_M5INV, true));
  }

  void Ddag_op(hipStream_t st, Prec p, const FieldPtr& out, const FieldPtr& in, const std::string& tag) {
    FieldPtr t0 = field(tag + ".t0", p, lat.vh), e = field(tag + ".e", p, lat.vh);
    apply5_full(st, p, t0, in, mat(p, MAT_M5INV_T), lat.vh, Ls, nullptr);
    hop(st, p, e, t0, nullptr, 1, true, epi(p, -1, MAT_QT));
    hop(st, p, out, e, &in, 0, true, epi(p, -1, MAT_NEG_MPHI_T, true));
  }

  // A_s p_s for every subdomain (inner storage I), given t0 = M_phi p_s on C.
  // <p_s, A_s p_s> partials [d][bps of C] when dot != null.
  void Asub(hipStream_t st, Prec I, const FieldPtr& q, const FieldPtr& ps, const FieldPtr& t0, double* dot,
            const Batch& bt = Batch()) {
    // e (on N1) is written over a (on N1), which the second hop has consumed
    FieldPtr a = field("in.a", I, (int64_t)nsub * nN1, bt.n), c = field("in.c", I, (int64_t)nsub * nN2, bt.n),
             e = a;
    const Sched sc = sched(2, I, bt.n);
    auto run = [&](int which, const FieldPtr& out, const FieldPtr& in, const FieldPtr* w, int par, bool dag,
                   const Epilogue& E) {
      const size_t ev = ev_begin(st, 10 + which);
      hop_sub(st, I, out, in, w, gauge_sub(I), lat, par, tables(which, I), nsub, Ls, dag, E, bt, sc);
      ev_end(st, ev);
    };
    run(1, a, t0, nullptr, 1, false, epi(I, -1, MAT_Q));
    run(2, c, a, &ps, 0, false, epi(I, MAT_M5INV_T, MAT_NEG_M5INVT_M5INV));
    run(3, e, c, nullptr, 1, true, epi(I, -1, MAT_QT));
    run(4, q, e, &c, 0, true, epi(I, MAT_M5_T, MAT_NEG_MPHI_T, false, dot, &ps));
  }

  // z = (+)_s CG_k(A_s, R_s r).  Outer precision O for r, z, r_old.
  // dots: partials of <z, r> and <z, r_old> into pz1/pz2 (nsub * bpsC entries).
  int precondition(hipStream_t st, Prec O, Prec I, const FieldPtr& z, const FieldPtr& r, const FieldPtr* rold,
                   int k, double* pz1, double* pz2, const Batch& bt = Batch()) {
    if (Lh > 0) return precondition_reduced(st, O, I, z, r, rold, k, pz1, pz2, bt);
    const size_t ev = ev_begin(st, 2);
    const int64_t nc = (int64_t)nsub * nC;
    const int nb = bt.n;
    FieldPtr rs = field("in.r", I, nc, nb), ps = field("in.p", I, nc, nb), zs = field("in.z", I, nc, nb),
             qs = field("in.q", I, nc, nb), t0 = field("in.t0", I, nc, nb);
    SubScalars sc;
    sc.rho = buf("in.rho", (size_t)nb * nsub * sizeof(double)).as<double>();
    sc.rho_next = buf("in.rho2", (size_t)nb * nsub * sizeof(double)).as<double>();
    sc.alpha = buf("in.alpha", (size_t)nb * nsub * sizeof(double)).as<double>();
    sc.beta = buf("in.beta", (size_t)nb * nsub * sizeof(double)).as<double>();
    sc.active = buf("in.active", (size_t)nb * nsub * sizeof(int)).as<int>();
    const SubTables tc = tables(0, I);
    double* prr = partial("in.rr", (int64_t)nb * nsub * tc.bps);
    double* ppap = partial("in.pap", (int64_t)nb * nsub * tc.bps);
    sub_restrict(st, O, I, r, rs, ps, t0, mat(I, MAT_MPHI), lat, tc, nsub, Ls, prr, bt);
    sub_finish(st, prr, tc.bps, nsub, sc, SUB_INIT, bt);
    // the per-subdomain alpha and beta are formed inside the kernels that
    // use them (sub_update, sub_xpay5) from the partials of the kernel
    // before; rho alternates between two arrays so that no block of
    // sub_xpay5 overwrites the rho another block still reads
    for (int it = 0; it < k; ++it) {
      if (it > 0) {
        sub_xpay5(st, I, ps, rs, t0, sc, prr, mat(I, MAT_MPHI), tc, nsub, Ls, bt);
        std::swap(sc.rho, sc.rho_next);
      }
      Asub(st, I, qs, ps, t0, ppap, bt);
      sub_update(st, I, zs, ps, rs, qs, sc, it == 0, it == k - 1, tc, nsub, Ls, ppap, prr, bt);
    }
    sub_prolong(st, O, I, z, zs, r, rold, lat, tc, nsub, Ls, pz1, pz2, bt);
    ev_end(st, ev);
    return k;
  }

  // z = (T^dag Mhat^-1 T + mu) r with Mhat^-1 the same k-step inner CG at Lh;
  // the PR dots of z with r and r_old fused into the back transform
  int precondition_reduced(hipStream_t st, Prec O, Prec I, const FieldPtr& z, const FieldPtr& r,
                           const FieldPtr* rold, int k, double* pz1, double* pz2, const Batch& bt) {
    const size_t ev = ev_begin(st, 2);
    mspcg_ctx* c = reduced_ctx();
    c->sp = sp;
    const int nb = bt.n;
    FieldPtr rh = c->field("red.r", O, lat.vh, nb), zh = c->field("red.z", O, lat.vh, nb);
    const int64_t nzc = c->precond_partials(O, I);
    double* q1 = c->partial("red.z1", nzc * nb);
    double* q2 = c->partial("red.z2", nzc * nb);
    transform(st, O, rh, r, Tdev(O, false), Ls, Lh, lat.vh, 0.0, nullptr, nullptr, nullptr, nullptr, bt);
    c->precondition(st, O, I, zh, rh, nullptr, k, q1, q2, bt);
    transform(st, O, z, zh, Tdev(O, true), Lh, Ls, lat.vh, mu_red, &r, rold, pz1, pz2, bt);
    ev_end(st, ev);
    return k;
  }

  // out = (+)_s A_s in: every subdomain's part through its local operator
  // (storage P), the results put back in place
  void local_op(hipStream_t st, Prec O, Prec P, const FieldPtr& fo, const FieldPtr& fi) {
    const SubTables tc = tables(0, P);
    const int64_t nz = (int64_t)nsub * tc.bps;
    double* p1 = partial("ap.z1", nz);
    double* p2 = partial("ap.z2", nz);
    const int64_t nc = (int64_t)nsub * nC;
    FieldPtr rs = field("in.r", P, nc), ps = field("in.p", P, nc), t0 = field("in.t0", P, nc), qs = field("in.q", P, nc);
    sub_restrict(st, O, P, fi, rs, ps, t0, mat(P, MAT_MPHI), lat, tc, nsub, Ls, p1);
    Asub(st, P, qs, ps, t0, nullptr);
    sub_prolong(st, O, P, fo, qs, fi, nullptr, lat, tc, nsub, Ls, p1, p2);
  }
};

// ==========================================================================
// solver
// ==========================================================================
namespace {

void check_status(mspcg_status s) {
  if (s != MSPCG_OK) throw Error(s, g_last_error);
}

}  // namespace

mspcg_ctx* mspcg_ctx::reduced_ctx() {
  if (red && !red_dirty) return red.get();
  if (!have_gauge) throw Error(MSPCG_ERR_NO_GAUGE, "no gauge field loaded");
  if (!have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "the reduced-Ls preconditioner needs mspcg_set_subdomains");
  if (red && hip_ready) HIPCHK(hipStreamSynchronize(stream));
  std::unique_ptr<mspcg_ctx> c(new mspcg_ctx(dims, device));
  check_status(mspcg_share_gauge(c.get(), this));
  check_status(mspcg_set_mobius(c.get(), Lh, bh, ch, M5, mf));
  check_status(mspcg_set_subdomains(c.get(), sub));
  c->sp = sp;
  red = std::move(c);
  red_dirty = false;
  return red.get();
}

namespace {

// chi^2 = sum_i |M (T^dag Mhat^-1 T + mu) v_i - v_i|^2, M = (+)_s A_s, over nvec
// device FP64 fields; with grad set, d chi^2/d Re T + i d chi^2/d Im T with
// Mhat^-1 taken as linear: 2 sum_i [ G(b_i, m_i) + G(a_i, v_i) ], b = Mhat^-1 T v,
// m = M e, a = Mhat^-1 T m, G(f, g) = sum over sites and colour of f conj(g).
double reduced_loss_impl(mspcg_ctx* h, int nvec, const double* v, std::vector<double>* grad, hipStream_t st) {
  const Prec O = to_prec(h->sp.outer_prec), I = to_prec(h->sp.inner_prec);
  mspcg_ctx* c = h->reduced_ctx();
  c->sp = h->sp;
  const int64_t vh = h->lat.vh, nreal = h->n5() * 24;
  const int Ls = h->Ls, Lh = h->Lh, k = h->sp.inner_iters;
  FieldPtr vf = h->field("tr.v", O, vh), zf = h->field("tr.z", O, vh), ef = h->field("tr.e", O, vh),
           mfield = h->field("tr.m", O, vh);
  FieldPtr rh = c->field("tr.rh", O, vh), bfield = c->field("tr.bh", O, vh), afield = c->field("tr.ah", O, vh);
  const int64_t nzc = c->precond_partials(O, I);
  double* q1 = c->partial("tr.q1", nzc);
  double* q2 = c->partial("tr.q2", nzc);
  const int nbn = 240;
  double* pn = h->partial("tr.norm", nbn);
  const int nent = Lh * 4 * Ls * 4;
  double2* G = nullptr;
  double2* part = nullptr;
  if (grad) {
    G = h->buf("tr.G", (size_t)nent * sizeof(double2)).as<double2>();
    part = h->buf("tr.Gpart", (size_t)outer_sum_parts(vh) * nent * sizeof(double2)).as<double2>();
    zero_batched(st, G, (int64_t)nent * sizeof(double2), Batch());
  }
  std::vector<double> hp(nbn);
  double total = 0;
  for (int i = 0; i < nvec; ++i) {
    pack_field(st, vf, v + (int64_t)i * nreal, vh, Ls);
    transform(st, O, rh, vf, h->Tdev(O, false), Ls, Lh, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
    c->precondition(st, O, I, bfield, rh, nullptr, k, q1, q2);
    transform(st, O, zf, bfield, h->Tdev(O, true), Lh, Ls, vh, h->mu_red, &vf, nullptr, nullptr, nullptr);
    h->local_op(st, O, I, ef, zf);
    diff_norm(st, O, ef.data, ef.data, vf.data, nreal, pn, nbn);
    HIPCHK(hipMemcpyAsync(h->h_bounce, pn, nbn * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(hp.data(), h->h_bounce, nbn * sizeof(double));
    for (int j = 0; j < nbn; ++j) total += hp[j];
    if (grad) {
      h->local_op(st, O, I, mfield, ef);
      transform(st, O, rh, mfield, h->Tdev(O, false), Ls, Lh, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
      c->precondition(st, O, I, afield, rh, nullptr, k, q1, q2);
      outer_sum(st, O, bfield, mfield, Lh, Ls, vh, part, G);
      outer_sum(st, O, afield, vf, Lh, Ls, vh, part, G);
    }
  }
  if (grad) {
    grad->assign(2 * (size_t)nent, 0.0);
    HIPCHK(hipMemcpyAsync(h->h_bounce, G, (size_t)nent * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(grad->data(), h->h_bounce, (size_t)nent * sizeof(double2));
    for (double& g : *grad) g *= 2.0;
  }
  return total;
}

// coefficients c_0..c_4 of chi^2(T + eta d) with Mhat^-1 taken as linear:
// per vector, Ha = Mhat^-1 T v, Hb = Mhat^-1 d v, e(eta) = e0 + eta e1 + eta^2 e2
// with e0 = M (T^dag Ha + mu v) - v, e1 = M (T^dag Hb + d^dag Ha), e2 = M d^dag Hb
void line_quartic_impl(mspcg_ctx* h, int nvec, const double* v, const std::vector<double>& d, double* cf,
                       hipStream_t st) {
  const Prec O = to_prec(h->sp.outer_prec), I = to_prec(h->sp.inner_prec);
  mspcg_ctx* c = h->reduced_ctx();
  c->sp = h->sp;
  h->upload_matrix(d, h->D64, h->D32, h->Dd64, h->Dd32);
  const int64_t vh = h->lat.vh, nreal = h->n5() * 24;
  const int Ls = h->Ls, Lh = h->Lh, k = h->sp.inner_iters;
  FieldPtr vf = h->field("tr.v", O, vh), z0 = h->field("tr.z", O, vh), z1 = h->field("tr.m", O, vh),
           e0 = h->field("tr.e", O, vh), e1 = h->field("tr.e1", O, vh), e2 = h->field("tr.e2", O, vh);
  FieldPtr rh = c->field("tr.rh", O, vh), ha = c->field("tr.bh", O, vh), hb = c->field("tr.ah", O, vh);
  const int64_t nzc = c->precond_partials(O, I);
  double* q1 = c->partial("tr.q1", nzc);
  double* q2 = c->partial("tr.q2", nzc);
  const int64_t nbl = blas_blocks(nreal / (O == Prec::F64 ? 2 : 4));
  double* pa = h->partial("tr.da", nbl);
  double* pb = h->partial("tr.db", nbl);
  double* pn = h->partial("tr.norm", 240);
  std::vector<double> ha_(nbl), hb_(nbl);
  auto sums = [&](double& x, double& y) {
    HIPCHK(hipMemcpyAsync(h->h_bounce, pa, nbl * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h->h_bounce + nbl * sizeof(double), pb, nbl * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(ha_.data(), h->h_bounce, nbl * sizeof(double));
    std::memcpy(hb_.data(), h->h_bounce + nbl * sizeof(double), nbl * sizeof(double));
    x = y = 0;
    for (int64_t j = 0; j < nbl; ++j) {
      x += ha_[j];
      y += hb_[j];
    }
  };
  for (int j = 0; j < 5; ++j) cf[j] = 0;
  for (int i = 0; i < nvec; ++i) {
    pack_field(st, vf, v + (int64_t)i * nreal, vh, Ls);
    transform(st, O, rh, vf, h->Tdev(O, false), Ls, Lh, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
    c->precondition(st, O, I, ha, rh, nullptr, k, q1, q2);
    transform(st, O, rh, vf, h->Ddev(O, false), Ls, Lh, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
    c->precondition(st, O, I, hb, rh, nullptr, k, q1, q2);
    transform(st, O, z0, ha, h->Tdev(O, true), Lh, Ls, vh, h->mu_red, &vf, nullptr, nullptr, nullptr);
    h->local_op(st, O, I, e0, z0);
    diff_norm(st, O, e0.data, e0.data, vf.data, nreal, pn, 240);
    transform(st, O, z1, hb, h->Tdev(O, true), Lh, Ls, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
    transform(st, O, z0, ha, h->Ddev(O, true), Lh, Ls, vh, 1.0, &z1, nullptr, nullptr, nullptr);
    h->local_op(st, O, I, e1, z0);
    transform(st, O, z1, hb, h->Ddev(O, true), Lh, Ls, vh, 0.0, nullptr, nullptr, nullptr, nullptr);
    h->local_op(st, O, I, e2, z1);
    double n00, n01, n02, n11, n12, n22, unused;
    dot2(st, O, e0.data, e0.data, e1.data, nreal, pa, pb, nbl);
    sums(n00, n01);
    dot2(st, O, e2.data, e0.data, e1.data, nreal, pa, pb, nbl);
    sums(n02, n12);
    dot2(st, O, e1.data, e1.data, e2.data, nreal, pa, pb, nbl);
    sums(n11, unused);
    dot2(st, O, e2.data, e2.data, nullptr, nreal, pa, nullptr, nbl);
    HIPCHK(hipMemcpyAsync(h->h_bounce, pa, nbl * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(ha_.data(), h->h_bounce, nbl * sizeof(double));
    n22 = 0;
    for (int64_t j = 0; j < nbl; ++j) n22 += ha_[j];
    cf[0] += n00;
    cf[1] += 2 * n01;
    cf[2] += n11 + 2 * n02;
    cf[3] += 2 * n12;
    cf[4] += n22;
  }
}

// minimiser over eta >= 0 of sum c_j eta^j: the best of 0 and the positive
// real roots of the derivative (a cubic: bracketed between the roots of its
// derivative and a bound on its roots, then bisected)
double quartic_min(const double* cf) {
  auto p = [&](double u) { return (((cf[4] * u + cf[3]) * u + cf[2]) * u + cf[1]) * u + cf[0]; };
  auto dp = [&](double u) { return ((4 * cf[4] * u + 3 * cf[3]) * u + 2 * cf[2]) * u + cf[1]; };
  const double d3 = 4 * cf[4], d2 = 3 * cf[3], d1 = 2 * cf[2], d0 = cf[1];
  // Cauchy bound on the roots of p' (1 + max |lower coefficient / leading|)
  double bound = 1;
  if (d3 != 0) bound = 1 + std::max({std::fabs(d2 / d3), std::fabs(d1 / d3), std::fabs(d0 / d3)});
  else if (d2 != 0) bound = 1 + std::max(std::fabs(d1 / d2), std::fabs(d0 / d2));
  else if (d1 != 0) bound = 1 + std::fabs(d0 / d1);
  std::vector<double> pts = {0.0, bound};
  const double a = 3 * d3, b = 2 * d2, cc = d1;   // derivative of p'
  if (a != 0) {
    const double disc = b * b - 4 * a * cc;
    if (disc >= 0) {
      const double sq = std::sqrt(disc);
      for (double r : {(-b - sq) / (2 * a), (-b + sq) / (2 * a)})
        if (r > 0 && r < bound) pts.push_back(r);
    }
  } else if (b != 0) {
    const double r = -cc / b;
    if (r > 0 && r < bound) pts.push_back(r);
  }
  std::sort(pts.begin(), pts.end());
  double best = 0, bestv = p(0);
  for (size_t j = 0; j + 1 < pts.size(); ++j) {
    double lo = pts[j], hi = pts[j + 1];
    double flo = dp(lo);
    const double fhi = dp(hi);
    if (!(flo == 0 || fhi == 0 || (flo < 0) != (fhi < 0))) continue;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, hi); ++it) {
      const double mid = 0.5 * (lo + hi);
      const double fm = dp(mid);
      if ((fm < 0) == (flo < 0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    const double u = 0.5 * (lo + hi);
    if (p(u) < bestv) {
      bestv = p(u);
      best = u;
    }
  }
  return best;
}

void set_transform(mspcg_ctx* h, const std::vector<double>& T) {
  h->Tm = T;
  h->upload_transform();
}

// line search along d = -grad + momentum d_prev (Sec. 3.3; readings as the oracle's)
void train_reduced_impl(mspcg_ctx* h, int nvec, const double* v, int iters, double momentum, double* hist,
                        hipStream_t st) {
  std::vector<double> T = h->Tm, g, d_prev(T.size(), 0.0), d(T.size());
  const double f0 = reduced_loss_impl(h, nvec, v, nullptr, st);
  if (hist) hist[0] = f0;
  double last = f0;
  for (int it = 0; it < iters; ++it) {
    reduced_loss_impl(h, nvec, v, &g, st);
    bool any = false;
    for (size_t i = 0; i < T.size(); ++i) {
      d[i] = -g[i] + momentum * d_prev[i];
      any = any || d[i] != 0;
    }
    if (!any) {
      for (int j = it + 1; j <= iters; ++j)
        if (hist) hist[j] = last;
      break;
    }
    double cf[5];
    line_quartic_impl(h, nvec, v, d, cf, st);
    const double eta = quartic_min(cf);
    for (size_t i = 0; i < T.size(); ++i) T[i] += eta * d[i];
    set_transform(h, T);
    d_prev = d;
    last = reduced_loss_impl(h, nvec, v, nullptr, st);
    if (hist) hist[it + 1] = last;
  }
}

void read_scalars(mspcg_ctx* h, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(h->h_scal, h->scal(), SLOT_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

mspcg_status solve_impl(mspcg_ctx* h, const double* b_dev, double* x_dev, const double* x0_dev, hipStream_t st,
                        mspcg_stats* stats) {
  const mspcg_solver_params& sp = h->sp;
  const Prec O = to_prec(sp.outer_prec);
  const Prec I = to_prec(sp.inner_prec);
  const bool pre = sp.use_precond != 0;
  const bool pr = sp.beta_rule == 0;
  const int64_t vh = h->lat.vh, n5 = h->n5(), nreal = n5 * 24;
  const int Ls = h->Ls;
  if (pre && !h->have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "MSPCG needs mspcg_set_subdomains");
  if (pre && sp.inner_iters < 1) throw Error(MSPCG_ERR_INVALID_ARG, "MSPCG needs inner_iters >= 1");

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));

  double* scal = h->scal();
  const int64_t nbl = blas_blocks(nreal / (O == Prec::F64 ? 2 : 4));
  const int64_t nbl64 = blas_blocks(nreal / 2);
  double* p_upd = h->partial("upd", nbl);
  double* p_ru = h->partial("ru", nbl64);
  double* p_b = h->partial("b", nbl64);
  const int64_t bps_hop = full_blocks(vh, Ls, O);
  double* p_pap = h->partial("pap", bps_hop);
  int64_t nz = 0;
  double *p_z1 = nullptr, *p_z2 = nullptr;
  if (pre) {
    nz = h->precond_partials(O, I);
    p_z1 = h->partial("z1", nz);
    p_z2 = h->partial("z2", nz);
  } else {
    p_z1 = h->partial("z1", nbl);
  }

  // FP64 copies: b, x_hi, r64, A64 workspace output
  FieldPtr b64 = h->field("s.b64", Prec::F64, vh), x64 = h->field("s.x64", Prec::F64, vh);
  FieldPtr r64 = h->field("s.r64", Prec::F64, vh), q64 = h->field("s.q64", Prec::F64, vh);
  pack_field(st, b64, b_dev, vh, Ls);
  if (x0_dev) pack_field(st, x64, x0_dev, vh, Ls);
  else HIPCHK(hipMemsetAsync(x64.data, 0, (size_t)n5 * 192, st));

  // outer vectors
  FieldPtr x = O == Prec::F64 ? x64 : h->field("s.x", O, vh);
  FieldPtr rA = h->field("s.rA", O, vh);
  FieldPtr rB = h->field("s.rB", O, vh);
  FieldPtr z = pre ? h->field("s.z", O, vh) : rA;
  FieldPtr p = h->field("s.p", O, vh), q = h->field("s.q", O, vh), t0 = h->field("s.t0", O, vh);
  if (O == Prec::F32) HIPCHK(hipMemsetAsync(x.data, 0, (size_t)n5 * 96, st));
  HIPCHK(hipMemsetAsync(p.data, 0, (size_t)n5 * chunk_bytes(O), st));

  // |b|^2
  dot2(st, Prec::F64, b64.data, b64.data, nullptr, nreal, p_b, nullptr, nbl64);
  finish(st, p_b, nullptr, nbl64, scal, FIN_STORE, SLOT_TMP);
  read_scalars(h, st);
  const double bnorm2 = h->h_scal[SLOT_TMP];
  if (!std::isfinite(bnorm2)) throw Error(MSPCG_ERR_BREAKDOWN, "source is not finite");
  const double bnorm = std::sqrt(bnorm2);

  FieldPtr* r = &rA;
  FieldPtr* rold = &rB;

  // true residual r = b - A x (FP64), lower precision copy into r
  auto true_residual = [&]() -> double {
    h->A_op(st, Prec::F64, q64, x64, "A64", nullptr);
    residual64(st, b64.data ? (const double*)b64.data : nullptr, (const double*)q64.data, (double*)r64.data,
               O == Prec::F32 ? (float*)r->data : nullptr, n5, p_ru, nbl64);
    if (O == Prec::F64 && r->data != r64.data)
      HIPCHK(hipMemcpyAsync(r->data, r64.data, (size_t)n5 * 192, hipMemcpyDeviceToDevice, st));
    finish(st, p_ru, nullptr, nbl64, scal, FIN_STORE, SLOT_R64);
    read_scalars(h, st);
    return h->h_scal[SLOT_R64];
  };

  mspcg_stats S;
  std::memset(&S, 0, sizeof(S));
  mspcg_status status = MSPCG_NOT_CONVERGED;
  h->history.clear();
  h->history_pap.clear();
  if (bnorm2 == 0.0) {
    HIPCHK(hipMemsetAsync(x64.data, 0, (size_t)n5 * 192, st));
    status = MSPCG_OK;
  } else {
    double rr = x0_dev ? true_residual() : bnorm2;
    if (!x0_dev) {
      // r = b
      if (O == Prec::F64) HIPCHK(hipMemcpyAsync(r->data, b64.data, (size_t)n5 * 192, hipMemcpyDeviceToDevice, st));
      else f64_to_f32(st, (const double*)b64.data, (float*)r->data, n5);
      HIPCHK(hipMemcpyAsync(r64.data, b64.data, (size_t)n5 * 192, hipMemcpyDeviceToDevice, st));
    }
    double rmax = std::sqrt(rr);
    const double delta = sp.reliable_delta > 0 ? sp.reliable_delta : 0.0;
    const double* rr_partial = nullptr;
    h->history.push_back(std::sqrt(rr) / bnorm);

    // z = M r ; rho = <r, z>
    auto apply_precond = [&](bool with_rold) {
      if (pre) {
        h->precondition(st, O, I, z, *r, with_rold ? rold : nullptr, sp.inner_iters, p_z1, p_z2);
        S.inner_iters_total += sp.inner_iters;
      }
    };
    apply_precond(false);
    if (pre) finish(st, p_z1, nullptr, nz, scal, FIN_RHO, 0);
    else {
      dot2(st, O, r->data, r->data, nullptr, nreal, p_z1, nullptr, nbl);
      finish(st, p_z1, nullptr, nbl, scal, FIN_RHO, 0);
    }
    // p = z ; t0 = M_phi p   (p is zero, beta slot holds 0)
    HIPCHK(hipMemsetAsync(scal + SLOT_TMP, 0, sizeof(double), st));
    xpay_apply5(st, O, t0, p, z, scal, SLOT_TMP, h->mat(O, MAT_MPHI), vh, Ls);

    int it = 0;
    while (true) {
      // q = A p, <p, A p> = |D p|^2
      h->A_from_t0(st, O, q, p, t0, "Aout", p_pap);
      finish(st, p_pap, nullptr, bps_hop, scal, FIN_ALPHA, 0);
      // x += alpha p ; r_new = r - alpha q
      cg_update(st, O, x.data, p.data, r->data, q.data, rold->data, nreal, scal, SLOT_ALPHA, p_upd, nbl);
      std::swap(r, rold);   // r: new residual, rold: previous
      finish(st, p_upd, nullptr, nbl, scal, FIN_STORE, SLOT_RR);
      rr_partial = p_upd;
      read_scalars(h, st);
      ++it;
      const double pap = h->h_scal[SLOT_PAP];
      rr = h->h_scal[SLOT_RR];
      if (!(pap > 0.0) || !std::isfinite(pap) || !std::isfinite(rr)) {
        // x is returned as the last iterate whose values are finite, with its
        // true residual: the breaking step is kept when its alpha and residual
        // are finite (FP32: the low-order part is folded into x_hi), else
        // (FP32) x_hi holds the solution of the last reliable update
        status = MSPCG_ERR_BREAKDOWN;
        S.iter_rel_resid = std::sqrt(std::fabs(rr)) / bnorm;
        const double alpha = h->h_scal[SLOT_ALPHA];
        if (O == Prec::F32 && std::isfinite(alpha) && std::isfinite(rr))
          accum_lo(st, (double*)x64.data, (float*)x.data, n5);
        rr = true_residual();
        break;
      }
      const double rn = std::sqrt(rr);
      S.iter_rel_resid = rn / bnorm;
      h->history.push_back(rn / bnorm);
      h->history_pap.push_back(pap / bnorm2);
      rmax = std::max(rmax, rn);
      if (h->log_every > 0 && it % h->log_every == 0)
        std::fprintf(stderr, "[mspcg] iteration %d  |r|/|b| = %.3e  reliable updates %d\n", it, rn / bnorm,
                     S.reliable_updates);
      const bool conv = rn <= sp.tol * bnorm;
      const bool last = it >= sp.maxiter;
      const bool ru = conv || last || (delta > 0 && rn < delta * rmax);
      if (ru) {
        if (O == Prec::F32) accum_lo(st, (double*)x64.data, (float*)x.data, n5);
        // keep the previous residual's copy: with FP32 the new residual
        // overwrites *r in place, r_old is untouched
        rr = true_residual();
        rr_partial = p_ru;
        ++S.reliable_updates;
        rmax = std::sqrt(rr);
        S.iter_rel_resid = std::sqrt(rr) / bnorm;
        if (std::sqrt(rr) <= sp.tol * bnorm) { status = MSPCG_OK; break; }
        if (!std::isfinite(rr)) { status = MSPCG_ERR_BREAKDOWN; break; }
      }
      if (last) { status = MSPCG_NOT_CONVERGED; break; }
      // z = M r ; beta
      if (pre) {
        apply_precond(pr);
        finish(st, p_z1, pr ? p_z2 : nullptr, nz, scal, pr ? FIN_BETA_PR : FIN_BETA_FR, 0);
      } else {
        if (pr) {
          dot2(st, O, r->data, r->data, rold->data, nreal, p_z1, p_z2 ? p_z2 : h->partial("z2", nbl), nbl);
          finish(st, p_z1, h->partial("z2", nbl), nbl, scal, FIN_BETA_PR, 0);
        } else {
          finish(st, rr_partial, nullptr, rr_partial == p_ru ? nbl64 : nbl, scal, FIN_BETA_FR, 0);
        }
      }
      // p = z + beta p ; t0 = M_phi p
      xpay_apply5(st, O, t0, p, pre ? z : *r, scal, SLOT_BETA, h->mat(O, MAT_MPHI), vh, Ls);
    }
    S.outer_iters = it;
    S.true_rel_resid = std::sqrt(std::fabs(rr)) / bnorm;
  }
  S.status = status;
  unpack_field(st, x_dev, x64, vh, Ls);
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  S.ms_total = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (h->profiling) {
    double tot = 0;
    for (auto& kv : h->ev_log)
      if (kv.first == 2) {
        float m = 0;
        if (hipEventElapsedTime(&m, h->ev_pool[kv.second].a, h->ev_pool[kv.second].b) == hipSuccess) tot += m;
      }
    S.ms_precond = tot;
  }
  if (stats) *stats = S;
  return status;
}

// --------------------------------------------------------------------------
// The full 5D system M psi = phi on both parities (the block form of Sec.
// 2.2, [[M5, M4_eo], [M4_oe, M5]] with M4 = D^w M_phi) through the even-odd
// Schur complement (eq. dirac_equation):
//   phi^_e = M5^-1 phi_e - M5^-1 M4_eo M5^-1 phi_o
//   D^dag D psi_e = D^dag phi^_e        (the configured solver)
//   psi_o = M5^-1 (phi_o - M4_oe psi_e)
// Every step outside the solve is FP64; M4_eo M5^-1 phi_o is one hop of
// Q phi_o (Q = M_phi M5^-1) with the M5^-1 epilogues fused.  full_resid
// (nullable) gets || phi - M psi || / || phi || in FP64.
// --------------------------------------------------------------------------
mspcg_status solve_full_impl(mspcg_ctx* h, const double* phi, double* psi, hipStream_t st, mspcg_stats* stats,
                             double* full_resid) {
  const int64_t vh = h->lat.vh, n5 = h->n5(), half = n5 * 24;
  const int Ls = h->Ls;
  const Prec P = Prec::F64;
  FieldPtr pe = h->field("f.pe", P, vh), po = h->field("f.po", P, vh), t = h->field("f.t", P, vh);
  FieldPtr he = h->field("f.he", P, vh), bq = h->field("f.b", P, vh);
  FieldPtr xe = h->field("f.xe", P, vh), xo = h->field("f.xo", P, vh);
  double* bcan = h->buf("f.bcan", (size_t)half * sizeof(double)).as<double>();
  pack_field(st, pe, phi, vh, Ls);
  pack_field(st, po, phi + half, vh, Ls);
  // phi^_e = M5^-1 phi_e - M5^-1 D^w_eo (Q phi_o) ; b = D^dag phi^_e
  apply5_full(st, P, t, po, h->mat(P, MAT_Q), vh, Ls, nullptr);
  h->hop(st, P, he, t, &pe, 0, false, h->epi(P, MAT_M5INV, MAT_NEG_M5INV));
  h->Ddag_op(st, P, bq, he, "f");
  unpack_field(st, bcan, bq, vh, Ls);
  const mspcg_status status = solve_impl(h, bcan, psi, nullptr, st, stats);
  if (status != MSPCG_OK && status != MSPCG_NOT_CONVERGED) return status;
  // psi_o = M5^-1 phi_o - M5^-1 D^w_oe (M_phi psi_e)
  pack_field(st, xe, psi, vh, Ls);
  apply5_full(st, P, t, xe, h->mat(P, MAT_MPHI), vh, Ls, nullptr);
  h->hop(st, P, xo, t, &po, 1, false, h->epi(P, MAT_M5INV, MAT_NEG_M5INV));
  unpack_field(st, psi + half, xo, vh, Ls);
  if (full_resid) {
    // (M psi)_e = M5 psi_e + D^w_eo M_phi psi_o ; (M psi)_o = M5 psi_o + D^w_oe M_phi psi_e
    FieldPtr me = h->field("f.me", P, vh), mo = h->field("f.mo", P, vh);
    apply5_full(st, P, t, xo, h->mat(P, MAT_MPHI), vh, Ls, nullptr);
    h->hop(st, P, me, t, &xe, 0, false, h->epi(P, MAT_M5, -1));
    apply5_full(st, P, t, xe, h->mat(P, MAT_MPHI), vh, Ls, nullptr);
    h->hop(st, P, mo, t, &xo, 1, false, h->epi(P, MAT_M5, -1));
    const int64_t nbl64 = blas_blocks(half / 2);
    double* part = h->partial("f.r", nbl64);
    double* scal = h->scal();
    double v[4];
    const FieldPtr* a[4] = {&pe, &po, &pe, &po};
    const FieldPtr* m[4] = {&me, &mo, nullptr, nullptr};
    for (int k = 0; k < 4; ++k) {
      if (m[k]) residual64(st, (const double*)a[k]->data, (const double*)m[k]->data, nullptr, nullptr, n5, part, nbl64);
      else dot2(st, P, a[k]->data, a[k]->data, nullptr, half, part, nullptr, nbl64);
      finish(st, part, nullptr, nbl64, scal, FIN_STORE, SLOT_TMP);
      read_scalars(h, st);
      v[k] = h->h_scal[SLOT_TMP];
    }
    const double pn = v[2] + v[3];
    *full_resid = pn > 0 ? std::sqrt((v[0] + v[1]) / pn) : 0.0;
  }
  HIPCHK(hipStreamSynchronize(st));
  return status;
}

// --------------------------------------------------------------------------
// Batched solve: nrhs right-hand sides on one gauge field, every kernel of
// an iteration launched once for all of them.  The iteration's decisions are
// taken on the device (ctl_*), masks drop finished RHS from every launch, and
// two iterations (one period of the r / r_old ping-pong) are captured in a
// graph that is replayed until no RHS is active.  The arithmetic of every RHS
// is that of the single-RHS solve: the same kernels, block partitions and
// reduction orders, with the same decisions taken in the same order.
// --------------------------------------------------------------------------
struct GraphGuard {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  ~GraphGuard() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
  }
};

// ---------------------------------------------------------------- batched solver engine
// The batched solver over n RHS slots: every kernel of an iteration runs once
// for all slots, masked by the per-slot control state on the device
// (k_ctl_*).  Slots start between iteration pairs through the start-up
// sequence masked to them (join), so right-hand sides can enter while others
// iterate (continuous batching); the one-shot batched solve starts every slot
// at once and runs pairs until none is active.  Each slot's arithmetic never
// depends on the other slots, so a slot's solution is the same whichever
// slots run beside it and whenever it starts.
struct BatchEngine {
  mspcg_ctx* h;
  const int n;
  const hipStream_t st;
  const std::string tag;   // workspace names ("s" for the one-shot solve, "cb" for an open session)
  mspcg_solver_params sp;
  Prec O, I;
  bool pre, pr, use_graph;
  int64_t vh, n5, nreal, nbl, nbl64, bps_hop, nz, bytes64, bytesO;
  int Ls;
  double *scal, *p_upd, *p_ru, *p_b, *p_pap, *p_z1, *p_z2;
  int* ci = nullptr;
  double* cd = nullptr;
  int* join = nullptr;
  Ctl c;
  CtlParams cp;
  Batch all, act, rum, bz, jn;
  FieldPtr b64, x64, q64, x, rA, rB, z, p, q, t0;
  FieldPtr* r = &rA;
  FieldPtr* rold = &rB;
  // Launch width: the kernels of an iteration cover slots [0, w) (a
  // continuous-batching session keeps w at one past its highest running
  // slot, so idle slots above it launch no workgroups).  One captured pair
  // per width, replayed while no workspace has moved since its capture.
  int w;
  struct PairGraph {
    GraphGuard gg;
    bool tried = false, ok = false, first_done = false;
    uint64_t gen = 0;
  };
  std::map<int, std::unique_ptr<PairGraph>> graphs;

  BatchEngine(mspcg_ctx* hh, int nn, hipStream_t s, const std::string& t) : h(hh), n(nn), st(s), tag(t) {
    sp = h->sp;
    O = to_prec(sp.outer_prec);
    I = to_prec(sp.inner_prec);
    pre = sp.use_precond != 0;
    pr = sp.beta_rule == 0;
    vh = h->lat.vh;
    n5 = h->n5();
    nreal = n5 * 24;
    Ls = h->Ls;
    if (pre && !h->have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "MSPCG needs mspcg_set_subdomains");
    if (pre && sp.inner_iters < 1) throw Error(MSPCG_ERR_INVALID_ARG, "MSPCG needs inner_iters >= 1");
    use_graph = h->graphs && !h->profiling;
    scal = h->scal(n);
    nbl = blas_blocks(nreal / (O == Prec::F64 ? 2 : 4));
    nbl64 = blas_blocks(nreal / 2);
    p_upd = h->partial("upd", nbl * n);
    p_ru = h->partial("ru", nbl64 * n);
    p_b = h->partial("b", nbl64 * n);
    bps_hop = full_blocks(vh, Ls, O);
    p_pap = h->partial("pap", bps_hop * n);
    nz = pre ? h->precond_partials(O, I) : nbl;
    p_z1 = h->partial("z1", nz * n);
    p_z2 = h->partial("z2", nz * n);
    ci = h->buf(tag + ".ctl.i", (size_t)round16((int64_t)(8 * n + 1) * sizeof(int))).as<int>();
    cd = h->buf(tag + ".ctl.d", (size_t)3 * n * sizeof(double)).as<double>();
    join = h->buf(tag + ".ctl.join", (size_t)n * sizeof(int)).as<int>();
    c.active = ci;
    c.ru = ci + n;
    c.bzero = ci + 2 * n;
    c.status = ci + 3 * n;
    c.iters = ci + 4 * n;
    c.rus = ci + 5 * n;
    c.precs = ci + 6 * n;
    c.nactive = ci + 8 * n;
    c.bnorm = cd;
    c.rmax = cd + n;
    c.rr = cd + 2 * n;
    cp.tol = sp.tol;
    cp.delta = sp.reliable_delta > 0 ? sp.reliable_delta : 0.0;
    cp.maxiter = sp.maxiter;
    set_width(n);
    act.mask = c.active;
    rum.mask = c.ru;
    bz.mask = c.bzero;
    jn.mask = join;
    b64 = h->field(tag + ".b64", Prec::F64, vh, n);
    x64 = h->field(tag + ".x64", Prec::F64, vh, n);
    q64 = h->field(tag + ".q64", Prec::F64, vh, n);
    x = O == Prec::F64 ? x64 : h->field(tag + ".x", O, vh, n);
    rA = h->field(tag + ".rA", O, vh, n);
    rB = h->field(tag + ".rB", O, vh, n);
    z = pre ? h->field(tag + ".z", O, vh, n) : rA;
    p = h->field(tag + ".p", O, vh, n);
    q = h->field(tag + ".q", O, vh, n);
    t0 = h->field(tag + ".t0", O, vh, n);
    bytes64 = n5 * 192;
    bytesO = n5 * (int64_t)chunk_bytes(O);
    // every slot idle: no kernel of an iteration touches it
    zero_batched(st, ci, round16((int64_t)(8 * n + 1) * sizeof(int)), Batch());
  }

  void set_width(int nw) {
    w = nw;
    all.n = act.n = rum.n = bz.n = jn.n = nw;
  }

  // One start-up (no slot joining) and one iteration pair with no slot
  // taking part, at the full width: every workspace of the engine reaches
  // its final size here, so no later pair, at any width, moves one.
  void size_workspaces() {
    set_width(n);
    fill_int(st, join, n, 0);
    start(false);
    iteration();
    iteration();
  }

  // slot i of a batched field
  FieldPtr slot(const FieldPtr& f, int i) const {
    FieldPtr v = f;
    v.data = (char*)f.data + (size_t)i * (size_t)f.stride * chunk_bytes(f.prec);
    if (f.scale) v.scale = f.scale + (size_t)i * (size_t)f.stride;
    return v;
  }

  // r = b - A x (FP64) for the masked RHS; lower-precision copy into *r
  void true_residual(const Batch& m) {
    h->A_op(st, Prec::F64, q64, x64, "A64", nullptr, m);
    residual64(st, (const double*)b64.data, (const double*)q64.data, O == Prec::F64 ? (double*)r->data : nullptr,
               O == Prec::F32 ? (float*)r->data : nullptr, n5, p_ru, nbl64, m);
    finish(st, p_ru, nullptr, nbl64, scal, FIN_STORE, SLOT_R64, m);
  }

  // The start-up sequence of Alg. 1 for the slots whose join flag the host
  // has set (the sources already packed into b64 by the caller): x = x0 or
  // 0, |b|, r = b - A x, z = M r, rho = <r, z>, p = z, t0 = M_phi p.
  void start(bool has_x0) {
    zero_batched(st, p.data, bytesO, jn);
    if (!has_x0) zero_batched(st, x64.data, bytes64, jn);
    if (O == Prec::F32) zero_batched(st, x.data, bytesO, jn);
    dot2(st, Prec::F64, b64.data, b64.data, nullptr, nreal, p_b, nullptr, nbl64, jn);
    finish(st, p_b, nullptr, nbl64, scal, FIN_STORE, SLOT_TMP, jn);
    ctl_init(st, c, scal, n, join);            // join becomes "joining and active"
    zero_batched(st, x64.data, bytes64, bz);
    if (has_x0) true_residual(jn);
    else if (O == Prec::F32) f64_to_f32(st, (const double*)b64.data, (float*)r->data, n5, jn);
    else apply5_full(st, Prec::F64, *r, b64, nullptr, vh, Ls, nullptr, jn);
    ctl_start(st, c, scal, n, has_x0, join);
    if (pre) {
      h->precondition(st, O, I, z, *r, nullptr, sp.inner_iters, p_z1, p_z2, jn);
      finish(st, p_z1, nullptr, nz, scal, FIN_RHO, 0, jn);
    } else {
      dot2(st, O, r->data, r->data, nullptr, nreal, p_z1, nullptr, nbl, jn);
      finish(st, p_z1, nullptr, nbl, scal, FIN_RHO, 0, jn);
    }
    xpay_apply5(st, O, t0, p, pre ? z : *r, scal, SLOT_TMP, h->mat(O, MAT_MPHI), vh, Ls, jn);
  }

  void iteration() {
    h->A_from_t0(st, O, q, p, t0, "Aout", p_pap, act);
    finish(st, p_pap, nullptr, bps_hop, scal, FIN_ALPHA, 0, act);
    cg_update(st, O, x.data, p.data, r->data, q.data, rold->data, nreal, scal, SLOT_ALPHA, p_upd, nbl, act);
    std::swap(r, rold);
    finish(st, p_upd, nullptr, nbl, scal, FIN_STORE, SLOT_RR, act);
    ctl_iterate(st, c, scal, n, cp);
    if (O == Prec::F32) accum_lo(st, (double*)x64.data, (float*)x.data, n5, rum);
    true_residual(rum);
    ctl_after_update(st, c, scal, n, cp);
    if (pre) {
      h->precondition(st, O, I, z, *r, pr ? rold : nullptr, sp.inner_iters, p_z1, p_z2, act);
      finish(st, p_z1, pr ? p_z2 : nullptr, nz, scal, pr ? FIN_BETA_PR : FIN_BETA_FR, 0, act);
    } else if (pr) {
      dot2(st, O, r->data, r->data, rold->data, nreal, p_z1, p_z2, nbl, act);
      finish(st, p_z1, p_z2, nbl, scal, FIN_BETA_PR, 0, act);
    } else {
      finish(st, nullptr, nullptr, 0, scal, FIN_BETA_FR, SLOT_RR, act);
    }
    xpay_apply5(st, O, t0, p, pre ? z : *r, scal, SLOT_BETA, h->mat(O, MAT_MPHI), vh, Ls, act);
  }

  // Two iterations (the r / r_old swap returns to its start), then the count
  // of active slots into the handle's pinned flag `slot`.  The first pair runs
  // eagerly (it sizes every workspace); the second is captured and every
  // later one replays the graph (eager if the capture failed: same kernels).
  void run_pair(int flag_slot) {
    std::unique_ptr<PairGraph>& slotp = graphs[w];
    if (slotp && slotp->ok && slotp->gen != h->ws_gen) {
      HIPCHK(hipStreamSynchronize(st));   // no replay of the old graph still in flight
      slotp.reset();
    }
    if (!slotp) slotp.reset(new PairGraph());
    PairGraph& G = *slotp;
    if (G.tried || !use_graph) {
      if (G.ok) HIPCHK(hipGraphLaunch(G.gg.e, st));
      else {
        iteration();
        iteration();
      }
    } else if (!G.first_done) {
      iteration();
      iteration();
      G.first_done = true;
    } else {
      G.tried = true;
      std::shared_lock<std::shared_mutex> lk(g_capture_gate);
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        FieldPtr* const r_at = r;   // a capture cut short leaves the swap half done
        FieldPtr* const ro_at = rold;
        tl_capturing = true;
        try {
          iteration();
          iteration();
        } catch (...) {
          ok = false;
        }
        tl_capturing = false;
        r = r_at;
        rold = ro_at;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        ok = ok && ec == hipSuccess && g != nullptr;
        if (ok) G.gg.g = g;
        else if (g) (void)hipGraphDestroy(g);
      }
      lk.unlock();
      if (ok) ok = hipGraphInstantiate(&G.gg.e, G.gg.g, nullptr, nullptr, 0) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        ++h->capture_fallbacks;
      }
      G.ok = ok;
      G.gen = h->ws_gen;
      if (G.ok) HIPCHK(hipGraphLaunch(G.gg.e, st));   // nothing ran during the capture
      else {
        iteration();
        iteration();
      }
    }
    HIPCHK(hipMemcpyAsync(h->h_flag + flag_slot, c.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
  }

  // statistics of slot i from the control arrays copied to the host
  void stats_of(int i, const std::vector<int>& hi, const std::vector<double>& hd, float ms, double ms_pre,
                mspcg_stats& S) const {
    std::memset(&S, 0, sizeof(S));
    const int status = hi[3 * n + i];
    S.outer_iters = hi[4 * n + i];
    S.reliable_updates = hi[5 * n + i];
    S.inner_iters_total = pre ? hi[6 * n + i] * sp.inner_iters : 0;
    const double bn = hd[i], rr = hd[2 * n + i];
    const double rel = (hi[2 * n + i] || !(bn > 0)) ? 0.0 : std::sqrt(std::fabs(rr)) / bn;
    S.true_rel_resid = rel;
    S.iter_rel_resid = rel;
    S.ms_total = ms;
    S.ms_precond = ms_pre;
    S.status = status == RHS_OK ? MSPCG_OK : status == RHS_BREAKDOWN ? MSPCG_ERR_BREAKDOWN : MSPCG_NOT_CONVERGED;
  }
  void download_ctl(std::vector<int>& hi, std::vector<double>& hd) {
    hi.resize((size_t)8 * n + 1);
    hd.resize((size_t)3 * n);
    h->download(hi.data(), ci, hi.size() * sizeof(int), st);
    h->download(hd.data(), cd, hd.size() * sizeof(double), st);
  }
};

mspcg_status solve_batch_impl(mspcg_ctx* h, int nrhs, const double* b_dev, double* x_dev, const double* x0_dev,
                              hipStream_t st, mspcg_stats* stats) {
  const int n = nrhs;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));
  hipEvent_t fev[2] = {nullptr, nullptr};
  std::unique_ptr<BatchEngine> E;
  try {
    E.reset(new BatchEngine(h, n, st, "s"));
    BatchEngine& B = *E;
    pack_field(st, B.b64, b_dev, B.vh, B.Ls, B.all);
    if (x0_dev) pack_field(st, B.x64, x0_dev, B.vh, B.Ls, B.all);
    fill_int(st, B.join, n, 1);
    B.start(x0_dev != nullptr);
    HIPCHK(hipEventCreateWithFlags(&fev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&fev[1], hipEventDisableTiming));
    // the host reads the active count of pair k while pair k + 1 runs
    const int64_t limit = (int64_t)B.sp.maxiter + 8;
    int64_t launched = 0;
    B.run_pair(0);
    launched += 2;
    HIPCHK(hipStreamSynchronize(st));
    if (h->h_flag[0] > 0) {
      for (int64_t k = 0;; ++k) {
        B.run_pair((int)(k & 1));
        launched += 2;
        HIPCHK(hipEventRecord(fev[k & 1], st));
        if (k > 0) {
          HIPCHK(hipEventSynchronize(fev[(k - 1) & 1]));
          if (h->h_flag[(k - 1) & 1] == 0) break;
          if (h->log_every > 0 && (launched - 2) % h->log_every < 2)
            std::fprintf(stderr, "[mspcg] batch: %lld iterations launched, %d of %d RHS active\n",
                         (long long)(launched - 2), h->h_flag[(k - 1) & 1], n);
        }
        if (launched > limit) {
          HIPCHK(hipEventSynchronize(fev[k & 1]));
          if (h->h_flag[k & 1] == 0) break;
          throw Error(MSPCG_ERR_HIP, "batched solve did not stop at the iteration limit");
        }
      }
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);
    for (hipEvent_t e : fev)
      if (e) (void)hipEventDestroy(e);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  for (hipEvent_t e : fev) (void)hipEventDestroy(e);
  BatchEngine& B = *E;
  unpack_field(st, x_dev, B.x64, B.vh, B.Ls, B.all);
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::vector<int> hi;
  std::vector<double> hd;
  B.download_ctl(hi, hd);
  double ms_pre = 0;
  if (h->profiling) {
    for (auto& kv : h->ev_log)
      if (kv.first == 2) {
        float m = 0;
        if (hipEventElapsedTime(&m, h->ev_pool[kv.second].a, h->ev_pool[kv.second].b) == hipSuccess) ms_pre += m;
      }
  }
  bool any_nc = false, any_bd = false;
  for (int i = 0; i < n; ++i) {
    const int status = hi[3 * n + i];
    any_bd |= status == RHS_BREAKDOWN;
    any_nc |= status == RHS_NOT_CONVERGED || status == RHS_RUNNING;
    if (stats) B.stats_of(i, hi, hd, ms, ms_pre, stats[i]);
  }
  if (any_bd) return MSPCG_ERR_BREAKDOWN;
  return any_nc ? MSPCG_NOT_CONVERGED : MSPCG_OK;
}

// ---------------------------------------------------------------- continuous batching
std::atomic<int> g_cb_sessions{0};   // open sessions of the process (mspcg_set_mfma waits for none)

enum SlotState { SLOT_FREE = 0, SLOT_PENDING, SLOT_RUNNING, SLOT_DONE };

struct CBSession {
  mspcg_ctx* h;
  hipStream_t st;
  std::unique_ptr<BatchEngine> E;
  struct Slot {
    int state = SLOT_FREE;
    const double* b = nullptr;
    double* x = nullptr;
    std::chrono::steady_clock::time_point t0;
    mspcg_stats stats;
  };
  std::vector<Slot> slots;
  int* h_status = nullptr;   // pinned copy of the per-slot RhsStatus
  CBSession(mspcg_ctx* hh, int n, hipStream_t s) : h(hh), st(s), slots((size_t)n) {
    E.reset(new BatchEngine(h, n, st, "cb"));
    E->size_workspaces();
    std::unique_lock<std::shared_mutex> lk(g_capture_gate);
    HIPCHK(hipHostMalloc((void**)&h_status, (size_t)n * sizeof(int), hipHostMallocDefault));
    ++g_cb_sessions;
  }
  ~CBSession() {
    (void)hipStreamSynchronize(st);
    {
      std::unique_lock<std::shared_mutex> lk(g_capture_gate);
      if (h_status) (void)hipHostFree(h_status);
    }
    --g_cb_sessions;
  }

  // pending slots start, one iteration pair runs, finished slots deliver x
  void step(int* running, int* pending) {
    BatchEngine& B = *E;
    const int n = B.n;
    std::vector<int> joining;
    int width = 0;   // one past the highest slot that runs or joins now
    for (int i = 0; i < n; ++i) {
      if (slots[i].state == SLOT_PENDING) joining.push_back(i);
      if (slots[i].state == SLOT_PENDING || slots[i].state == SLOT_RUNNING) width = i + 1;
    }
    if (width > 0) B.set_width(width);
    if (!joining.empty()) {
      fill_int(st, B.join, n, 0);
      for (int i : joining) {
        pack_field(st, B.slot(B.b64, i), slots[i].b, B.vh, B.Ls, Batch());
        fill_int(st, B.join + i, 1, 1);
        slots[i].state = SLOT_RUNNING;
        slots[i].t0 = std::chrono::steady_clock::now();
      }
      B.start(false);
    }
    bool any_running = false;
    for (const Slot& sl : slots) any_running |= sl.state == SLOT_RUNNING;
    if (any_running) B.run_pair(0);
    HIPCHK(hipMemcpyAsync(h_status, B.c.status, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> fin;
    for (int i = 0; i < n; ++i)
      if (slots[i].state == SLOT_RUNNING && h_status[i] != RHS_RUNNING) fin.push_back(i);
    if (!fin.empty()) {
      for (int i : fin) unpack_field(st, slots[i].x, B.slot(B.x64, i), B.vh, B.Ls, Batch());
      std::vector<int> hi;
      std::vector<double> hd;
      B.download_ctl(hi, hd);   // synchronizes: the x of every finished slot is written
      const auto now = std::chrono::steady_clock::now();
      for (int i : fin) {
        const float ms = (float)std::chrono::duration<double, std::milli>(now - slots[i].t0).count();
        B.stats_of(i, hi, hd, ms, 0.0, slots[i].stats);
        slots[i].state = SLOT_DONE;
        slots[i].b = nullptr;
        slots[i].x = nullptr;
      }
    }
    int nr = 0, np = 0;
    for (const Slot& sl : slots) {
      nr += sl.state == SLOT_RUNNING;
      np += sl.state == SLOT_PENDING;
    }
    if (running) *running = nr;
    if (pending) *pending = np;
  }
};

void no_session(const mspcg_ctx* h) {
  if (h->cb) throw Error(MSPCG_ERR_INVALID_ARG, "a continuous-batching session is open on this handle");
}

// --------------------------------------------------------------------------
// Autotuner of the hop schedules: time the four hops of one A application
// (outer precision, FP64) and of one A_s application (inner precision) for
// nrhs right-hand sides under every candidate schedule; keep the fastest.
// --------------------------------------------------------------------------
void autotune_impl(mspcg_ctx* h, int nrhs, hipStream_t st) {
  // block orders of the full-lattice hops: lexicographic or chunked t
  // sweeps of four chunk sizes (the subdomain hops take the first only)
  std::vector<Sched> cand;
  for (int tchunk = 0; tchunk < 5; ++tchunk)
    for (int order = 0; order < (nrhs > 1 ? 2 : 1); ++order)
      for (int xcd = 0; xcd < 2; ++xcd) {
        Sched sc;
        sc.order = order;
        sc.xcd = xcd;
        sc.tchunk = tchunk;
        cand.push_back(sc);
      }
  const Prec O = to_prec(h->sp.outer_prec), I = to_prec(h->sp.inner_prec);
  const int64_t vh = h->lat.vh;
  Batch bt;
  bt.n = nrhs;
  hipEvent_t ea, eb;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  const bool prof = h->profiling;
  h->profiling = false;
  struct Kind {
    int kind;
    Prec p;
  };
  std::vector<Kind> kinds;
  kinds.push_back({O == Prec::F64 ? 1 : 0, O});
  if (O != Prec::F64) kinds.push_back({1, Prec::F64});
  if (h->have_tiling) kinds.push_back({2, I});
  try {
    for (const Kind& k : kinds) {
      std::function<void()> run;
      FieldPtr in, out, t0;
      if (k.kind == 2) {
        const int64_t nc = (int64_t)h->nsub * h->nC;
        in = h->field("tune.in", k.p, nc, nrhs);
        out = h->field("tune.out", k.p, nc, nrhs);
        t0 = h->field("tune.t0", k.p, nc, nrhs);
        run = [&]() { h->Asub(st, k.p, out, in, t0, nullptr, bt); };
      } else {
        in = h->field("tune.in", k.p, vh, nrhs);
        out = h->field("tune.out", k.p, vh, nrhs);
        t0 = h->field("tune.t0", k.p, vh, nrhs);
        run = [&]() { h->A_from_t0(st, k.p, out, in, t0, "tune", nullptr, bt); };
      }
      const int64_t bytes = in.stride * (int64_t)chunk_bytes(k.p);
      zero_batched(st, in.data, bytes, bt);
      zero_batched(st, t0.data, bytes, bt);
      if (in.scale) {
        zero_batched(st, in.scale, round16((int64_t)nrhs * in.stride * 4), Batch());
        zero_batched(st, t0.scale, round16((int64_t)nrhs * t0.stride * 4), Batch());
      }
      const auto key = std::make_tuple(k.kind, (int)k.p, nrhs);
      double best = 1e30;
      Sched bsc;
      for (const Sched& sc : cand) {
        if (k.kind == 2 && sc.tchunk != 0) continue;
        h->tuned[key] = sc;
        run();   // warm
        HIPCHK(hipEventRecord(ea, st));
        const int reps = 3;
        for (int r = 0; r < reps; ++r) run();
        HIPCHK(hipEventRecord(eb, st));
        HIPCHK(hipEventSynchronize(eb));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ea, eb));
        const double us = 1e3 * ms / reps;
        if (h->log_every > 0)
          std::fprintf(stderr, "[mspcg] autotune kind %d nrhs %d: order %d xcd %d tchunk %d  %.1f us\n", k.kind, nrhs,
                       sc.order, sc.xcd, sc.tchunk, us);
        if (us < best) {
          best = us;
          bsc = sc;
        }
      }
      h->tuned[key] = bsc;
      h->tuned_us[key] = best;
    }
  } catch (...) {
    h->profiling = prof;
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    throw;
  }
  h->profiling = prof;
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  for (auto it = h->ws.begin(); it != h->ws.end();) {
    if (it->first.compare(0, 5, "tune.") == 0) it = h->ws.erase(it);
    else ++it;
  }
}

// Device bytes of the workspaces a batched solve of nrhs right-hand sides
// allocates (the fields and partial arrays of solve_batch_impl, the operator
// chains and the preconditioner), plus the matrices and tables.
int64_t estimate_solve_bytes(const mspcg_ctx* h, int nrhs) {
  const mspcg_solver_params& sp = h->sp;
  const Prec O = to_prec(sp.outer_prec), I = to_prec(sp.inner_prec);
  const bool pre = sp.use_precond != 0;
  const int64_t vh = h->lat.vh, n5 = h->n5(), nreal = n5 * 24;
  const int Ls = h->Ls;
  auto fbytes = [&](Prec p, int64_t sites5) {
    int64_t b = sites5 * (int64_t)chunk_bytes(p);
    if (scaled(p)) b += round16(sites5 * 4);
    return b;
  };
  int64_t n = 0;
  // FP64: b, x, A x and the A64 chain (t0, a)
  n += 5 * fbytes(Prec::F64, n5);
  // outer vectors: x (FP32), r, r_old, z, p, q, t0 and the A chain's a
  const int nO = (O == Prec::F32 ? 1 : 0) + 2 + (pre ? 1 : 0) + 3 + 1;
  n += nO * fbytes(O, n5);
  const int64_t nbl = blas_blocks(nreal / (O == Prec::F64 ? 2 : 4)), nbl64 = blas_blocks(nreal / 2);
  int64_t parts = nbl + 2 * nbl64 + full_blocks(vh, Ls, O);
  if (pre && h->have_tiling) {
    const int64_t bps = (h->nC + sites_per_block(Ls, I) - 1) / sites_per_block(Ls, I);
    const int64_t nc5 = (int64_t)h->nsub * h->nC * Ls;
    n += 5 * fbytes(I, nc5);
    n += fbytes(I, (int64_t)h->nsub * h->nN1 * Ls) + fbytes(I, (int64_t)h->nsub * h->nN2 * Ls);
    parts += 4 * (int64_t)h->nsub * bps;
    n += (int64_t)h->nsub * (4 * 8 + 4);   // rho (two arrays), alpha, beta, active
  } else {
    parts += 2 * nbl;
  }
  n += parts * 8;
  n *= nrhs;
  n += round16((int64_t)(8 * nrhs + 1) * 4) + (int64_t)3 * nrhs * 8 + (int64_t)nrhs * 4 + (int64_t)nrhs * SLOT_COUNT * 8;
  // matrices and tables
  n += (int64_t)h->mats64.n + (int64_t)h->mats32.n;
  for (const DevBuf* d : {&h->tb_origin, &h->tb_cC, &h->tb_cN1, &h->tb_cN2, &h->tb_nbr1, &h->tb_nbr2, &h->tb_nbr3,
                          &h->tb_nbr4, &h->tb_w2, &h->tb_w4})
    n += (int64_t)d->n;
  return n;
}

void apply_impl(mspcg_ctx* h, int op, Prec P, const double* in_dev, double* out_dev, hipStream_t st) {
  const int64_t vh = h->lat.vh;
  const int Ls = h->Ls;
  if (op == MSPCG_OP_A_SUB || op == MSPCG_OP_PRECOND) {
    if (!h->have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "operator needs mspcg_set_subdomains");
    const Prec O = (P == Prec::F64) ? Prec::F64 : Prec::F32;
    FieldPtr fi = h->field("ap.in", O, vh), fo = h->field("ap.out", O, vh);
    pack_field(st, fi, in_dev, vh, Ls);
    if (op == MSPCG_OP_PRECOND) {
      const int64_t nz = h->precond_partials(O, P);
      double* p1 = h->partial("ap.z1", nz);
      double* p2 = h->partial("ap.z2", nz);
      h->precondition(st, O, P, fo, fi, nullptr, h->sp.inner_iters, p1, p2);
    } else {
      h->local_op(st, O, P, fo, fi);
    }
    unpack_field(st, out_dev, fo, vh, Ls);
    return;
  }
  FieldPtr fi = h->field("ap.in", P, vh), fo = h->field("ap.out", P, vh);
  pack_field(st, fi, in_dev, vh, Ls);
  switch (op) {
    case MSPCG_OP_DSLASH_EO: h->hop(st, P, fo, fi, nullptr, 0, false, Epilogue()); break;
    case MSPCG_OP_DSLASH_OE: h->hop(st, P, fo, fi, nullptr, 1, false, Epilogue()); break;
    case MSPCG_OP_DSLASH_DAG_EO: h->hop(st, P, fo, fi, nullptr, 0, true, Epilogue()); break;
    case MSPCG_OP_DSLASH_DAG_OE: h->hop(st, P, fo, fi, nullptr, 1, true, Epilogue()); break;
    case MSPCG_OP_M5: apply5_full(st, P, fo, fi, h->mat(P, MAT_M5), vh, Ls, nullptr); break;
    case MSPCG_OP_M5INV: apply5_full(st, P, fo, fi, h->mat(P, MAT_M5INV), vh, Ls, nullptr); break;
    case MSPCG_OP_MPHI: apply5_full(st, P, fo, fi, h->mat(P, MAT_MPHI), vh, Ls, nullptr); break;
    case MSPCG_OP_D: h->D_op(st, P, fo, fi, "ap"); break;
    case MSPCG_OP_DDAG: h->Ddag_op(st, P, fo, fi, "ap"); break;
    case MSPCG_OP_A: h->A_op(st, P, fo, fi, "ap", nullptr); break;
    case MSPCG_OP_STORE: fo = fi; break;
    default: throw Error(MSPCG_ERR_INVALID_ARG, "unknown operator");
  }
  unpack_field(st, out_dev, fo, vh, Ls);
}

void need_state(mspcg_ctx* h) {
  if (!h->have_gauge) throw Error(MSPCG_ERR_NO_GAUGE, "no gauge field loaded");
  if (!h->have_params) throw Error(MSPCG_ERR_NO_PARAMS, "Mobius parameters not set");
  check_limits(h->dims, h->Ls, h->have_tiling ? h->nsub : 0, h->have_tiling ? h->nN2 : 0, (int)h->sp.inner_prec);
}

template <typename F> mspcg_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MSPCG_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MSPCG_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return MSPCG_ERR_HIP;
  }
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

mspcg_status mspcg_create(mspcg_t* out, const int32_t dims[4], int32_t device) {
  return guarded([&]() -> mspcg_status {
    if (!out || !dims) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    for (int m = 0; m < 4; ++m)
      if (dims[m] < 2 || dims[m] % 2 || dims[m] > 32000) throw Error(MSPCG_ERR_INVALID_ARG, "lattice extents must be even and >= 2");
    if (device < 0) throw Error(MSPCG_ERR_INVALID_ARG, "device must be >= 0");
    check_limits(dims, 0, 0, 0, -1);
    *out = new mspcg_ctx(dims, device);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_destroy(mspcg_t h) {
  return guarded([&]() -> mspcg_status {
    delete h;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_load_gauge(mspcg_t h, const double* U) {
  return guarded([&]() -> mspcg_status {
    if (!h || !U) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    h->ensure_hip();
    hipStream_t st = h->stream;
    const int64_t V = 2 * h->lat.vh;
    const size_t canon = (size_t)V * 4 * 9 * 2 * sizeof(double);
    DevBuf stage;
    stage.ensure(canon);
    h->upload(stage.p, U, canon, st);
    auto g = std::make_shared<mspcg_ctx::GaugeStore>();
    g->g64.ensure((size_t)V * 4 * 10 * sizeof(double2));
    g->g32.ensure((size_t)V * 4 * 10 * sizeof(float2));
    g->g16.ensure((size_t)V * 4 * 10 * 2 * sizeof(uint16_t));
    pack_gauge(st, g->g64.p, 8, stage.as<double>(), h->lat);
    pack_gauge(st, g->g32.p, 4, stage.as<double>(), h->lat);
    pack_gauge(st, g->g16.p, 2, stage.as<double>(), h->lat);
    h->gs = g;
    h->red_dirty = true;
    HIPCHK(hipStreamSynchronize(st));
    h->have_gauge = true;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_mobius(mspcg_t h, int32_t Ls, double b, double c, double M5, double mf) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    if (Ls < 2 || Ls > 32) throw Error(MSPCG_ERR_INVALID_ARG, "Ls must be in [2, 32]");
    if (!std::isfinite(b) || !std::isfinite(c) || !std::isfinite(M5) || !std::isfinite(mf))
      throw Error(MSPCG_ERR_INVALID_ARG, "non-finite Mobius parameter");
    check_limits(h->dims, Ls, h->have_tiling ? h->nsub : 0, h->have_tiling ? h->nN2 : 0,
                 h->have_solver ? (int)h->sp.inner_prec : -1);
    Mats M = build_mats(Ls, b, c, M5, mf);
    h->ensure_hip();
    h->invalidate_workspace();
    std::vector<float> m32(M.m.begin(), M.m.end());
    h->mats64.ensure(M.m.size() * sizeof(double));
    h->mats32.ensure(m32.size() * sizeof(float));
    h->upload(h->mats64.p, M.m.data(), M.m.size() * sizeof(double), h->stream);
    h->upload(h->mats32.p, m32.data(), m32.size() * sizeof(float), h->stream);
    h->tuned.clear();
    h->tuned_us.clear();
    if (Ls != h->Ls) {   // T has the old shape
      h->Lh = 0;
      h->red.reset();
    }
    h->Ls = Ls;
    h->b = b;
    h->c = c;
    h->M5 = M5;
    h->mf = mf;
    h->have_params = true;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_subdomains(mspcg_t h, const int32_t sub[4]) {
  return guarded([&]() -> mspcg_status {
    if (!h || !sub) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    int s[4] = {sub[0], sub[1], sub[2], sub[3]};
    std::string why;
    if (!tiling_valid(h->dims, s, why)) throw Error(MSPCG_ERR_BAD_TILING, why);
    HostTables H = build_tables(h->dims, s);
    {
      int64_t ns = 1;
      for (int m = 0; m < 4; ++m) ns *= h->dims[m] / s[m];
      check_limits(h->dims, h->have_params ? h->Ls : 0, ns, (int64_t)H.N2.coords.size(),
                   h->have_solver ? (int)h->sp.inner_prec : -1);
    }
    h->ensure_hip();
    h->invalidate_workspace();
    auto up = [&](DevBuf& d, const void* src, size_t bytes) {
      d.ensure(bytes);
      if (bytes) h->upload(d.p, src, bytes, h->stream);
    };
    up(h->tb_cC, H.C.coords.data(), H.C.coords.size() * sizeof(short4));
    up(h->tb_cN1, H.N1.coords.data(), H.N1.coords.size() * sizeof(short4));
    up(h->tb_cN2, H.N2.coords.data(), H.N2.coords.size() * sizeof(short4));
    up(h->tb_nbr1, H.nbr1.data(), H.nbr1.size() * sizeof(int));
    up(h->tb_nbr2, H.nbr2.data(), H.nbr2.size() * sizeof(int));
    up(h->tb_nbr3, H.nbr3.data(), H.nbr3.size() * sizeof(int));
    up(h->tb_nbr4, H.nbr4.data(), H.nbr4.size() * sizeof(int));
    up(h->tb_w2, H.wmap2.data(), H.wmap2.size() * sizeof(int));
    up(h->tb_w4, H.wmap4.data(), H.wmap4.size() * sizeof(int));
    std::vector<short4> origin;
    int nb[4];
    for (int m = 0; m < 4; ++m) nb[m] = h->dims[m] / s[m];
    for (int d3 = 0; d3 < nb[3]; ++d3)
      for (int d2 = 0; d2 < nb[2]; ++d2)
        for (int d1 = 0; d1 < nb[1]; ++d1)
          for (int d0 = 0; d0 < nb[0]; ++d0)
            origin.push_back(make_short4((short)(d0 * s[0]), (short)(d1 * s[1]), (short)(d2 * s[2]), (short)(d3 * s[3])));
    up(h->tb_origin, origin.data(), origin.size() * sizeof(short4));
    h->nC = (int)H.C.coords.size();
    h->nN1 = (int)H.N1.coords.size();
    h->nN2 = (int)H.N2.coords.size();
    h->nsub = 1;
    for (int m = 0; m < 4; ++m) {
      h->sub[m] = s[m];
      h->nblk[m] = h->dims[m] / s[m];
      h->nsub *= h->nblk[m];
    }
    h->have_tiling = true;
    h->tuned.clear();
    h->tuned_us.clear();
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_solver(mspcg_t h, const mspcg_solver_params* p) {
  return guarded([&]() -> mspcg_status {
    if (!h || !p) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (!(p->tol > 0) || p->maxiter < 1 || p->inner_iters < 0 || p->inner_iters > 1000)
      throw Error(MSPCG_ERR_INVALID_ARG, "tol > 0, maxiter >= 1, 0 <= inner_iters <= 1000 required");
    if (p->outer_prec != MSPCG_FP64 && p->outer_prec != MSPCG_FP32)
      throw Error(MSPCG_ERR_INVALID_ARG, "outer precision must be FP64 or FP32");
    (void)to_prec(p->inner_prec);
    if (p->beta_rule != 0 && p->beta_rule != 1) throw Error(MSPCG_ERR_INVALID_ARG, "beta_rule must be 0 or 1");
    if (!(p->reliable_delta >= 0) || p->reliable_delta >= 1) throw Error(MSPCG_ERR_INVALID_ARG, "reliable_delta in [0, 1)");
    check_limits(h->dims, h->have_params ? h->Ls : 0, h->have_tiling ? h->nsub : 0, h->have_tiling ? h->nN2 : 0,
                 (int)p->inner_prec);
    h->sp = *p;
    h->have_solver = true;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_solve_device(mspcg_t h, const double* b, double* x, const double* x0, void* hip_stream,
                                mspcg_stats* st) {
  return guarded([&]() -> mspcg_status {
    if (!h || !b || !x) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->stream;
    return solve_impl(h, b, x, x0, s, st);
  });
}

mspcg_status mspcg_solve(mspcg_t h, const double* b, double* x, const double* x0, mspcg_stats* st) {
  return guarded([&]() -> mspcg_status {
    if (!h || !b || !x) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    const size_t bytes = (size_t)h->n5() * 24 * sizeof(double);
    DevBuf db, dx, dx0;
    db.ensure(bytes);
    dx.ensure(bytes);
    h->upload(db.p, b, bytes, h->stream);
    if (x0) {
      dx0.ensure(bytes);
      h->upload(dx0.p, x0, bytes, h->stream);
    }
    mspcg_status r = solve_impl(h, db.as<double>(), dx.as<double>(), x0 ? dx0.as<double>() : nullptr, h->stream, st);
    h->download(x, dx.p, bytes, h->stream);
    return r;
  });
}

mspcg_status mspcg_solve_full_device(mspcg_t h, const double* phi, double* psi, void* hip_stream, mspcg_stats* st,
                                     double* full_rel_resid) {
  return guarded([&]() -> mspcg_status {
    if (!h || !phi || !psi) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->stream;
    return solve_full_impl(h, phi, psi, s, st, full_rel_resid);
  });
}

mspcg_status mspcg_solve_batch_device(mspcg_t h, int32_t nrhs, const double* b, double* x, const double* x0,
                                      void* hip_stream, mspcg_stats* st) {
  return guarded([&]() -> mspcg_status {
    if (!h || !b || !x) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (nrhs < 1 || nrhs > 1024) throw Error(MSPCG_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->stream;
    return solve_batch_impl(h, nrhs, b, x, x0, s, st);
  });
}

mspcg_status mspcg_share_gauge(mspcg_t h, mspcg_t src) {
  return guarded([&]() -> mspcg_status {
    if (!h || !src) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    if (!src->have_gauge) throw Error(MSPCG_ERR_NO_GAUGE, "source handle has no gauge field");
    for (int m = 0; m < 4; ++m)
      if (h->dims[m] != src->dims[m]) throw Error(MSPCG_ERR_INVALID_ARG, "lattice extents differ");
    if (h->device != src->device) throw Error(MSPCG_ERR_INVALID_ARG, "handles are on different devices");
    h->ensure_hip();
    h->gs = src->gs;
    h->red_dirty = true;
    h->have_gauge = true;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_reduced(mspcg_t h, int32_t Lhat, double b_hat, double c_hat, double mu, const double* T) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    if (Lhat == 0) {
      if (h->hip_ready) HIPCHK(hipStreamSynchronize(h->stream));
      h->Lh = 0;
      h->red.reset();
      return MSPCG_OK;
    }
    if (!h->have_params) throw Error(MSPCG_ERR_NO_PARAMS, "Mobius parameters not set");
    if (Lhat < 1 || Lhat > h->Ls) throw Error(MSPCG_ERR_INVALID_ARG, "Lhat must be in [1, Ls]");
    if (!T) throw Error(MSPCG_ERR_INVALID_ARG, "null transform");
    if (!std::isfinite(b_hat) || !std::isfinite(c_hat) || !std::isfinite(mu))
      throw Error(MSPCG_ERR_INVALID_ARG, "non-finite parameter");
    const size_t n = 2 * (size_t)Lhat * 4 * h->Ls * 4;
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(T[i])) throw Error(MSPCG_ERR_INVALID_ARG, "non-finite transform entry");
    // the reduced operator must be invertible: b (4 - M5) + 1 != 0 (checked by set_mobius on the context)
    h->ensure_hip();
    HIPCHK(hipStreamSynchronize(h->stream));
    h->Lh = Lhat;
    h->bh = b_hat;
    h->ch = c_hat;
    h->mu_red = mu;
    h->Tm.assign(T, T + n);
    h->upload_transform();
    h->red.reset();
    h->red_dirty = true;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_get_reduced(mspcg_t h, int32_t* Lhat, double* T) {
  return guarded([&]() -> mspcg_status {
    if (!h || !Lhat) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    *Lhat = h->Lh;
    if (T && h->Lh > 0) std::memcpy(T, h->Tm.data(), h->Tm.size() * sizeof(double));
    return MSPCG_OK;
  });
}

mspcg_status mspcg_reduced_loss(mspcg_t h, int32_t nvec, const double* v, double* chi2, double* grad) {
  return guarded([&]() -> mspcg_status {
    if (!h || !v || !chi2) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (nvec < 1) throw Error(MSPCG_ERR_INVALID_ARG, "nvec must be >= 1");
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    if (h->Lh == 0) throw Error(MSPCG_ERR_INVALID_ARG, "no reduced-Ls preconditioner set");
    if (!h->have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "needs mspcg_set_subdomains");
    h->ensure_hip();
    std::vector<double> g;
    *chi2 = reduced_loss_impl(h, nvec, v, grad ? &g : nullptr, h->stream);
    if (grad) std::memcpy(grad, g.data(), g.size() * sizeof(double));
    return MSPCG_OK;
  });
}

mspcg_status mspcg_train_reduced(mspcg_t h, int32_t nvec, const double* v, int32_t iters, double momentum,
                                 double* history) {
  return guarded([&]() -> mspcg_status {
    if (!h || !v) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (nvec < 1 || iters < 0) throw Error(MSPCG_ERR_INVALID_ARG, "nvec must be >= 1 and iters >= 0");
    if (!std::isfinite(momentum)) throw Error(MSPCG_ERR_INVALID_ARG, "non-finite momentum");
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    if (h->Lh == 0) throw Error(MSPCG_ERR_INVALID_ARG, "no reduced-Ls preconditioner set");
    if (!h->have_tiling) throw Error(MSPCG_ERR_BAD_TILING, "needs mspcg_set_subdomains");
    h->ensure_hip();
    train_reduced_impl(h, nvec, v, iters, momentum, history, h->stream);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_mfma(int32_t on) {
  return guarded([&]() -> mspcg_status {
    std::unique_lock<std::shared_mutex> lk(g_engine_gate);
    if (g_cb_sessions.load() > 0)
      throw Error(MSPCG_ERR_INVALID_ARG, "continuous-batching sessions are open (their launches are sized for "
                                         "the current epilogue engine)");
    set_mfma_epilogue(on != 0);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_log(mspcg_t h, int32_t every) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    if (every < 0) throw Error(MSPCG_ERR_INVALID_ARG, "every must be >= 0");
    h->log_every = every;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_graphs(mspcg_t h, int32_t on) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    h->graphs = on != 0;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_footprint(mspcg_t h, int32_t nrhs, int64_t* estimate, int64_t* allocated) {
  return guarded([&]() -> mspcg_status {
    if (!h || !estimate || !allocated) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    if (nrhs < 1 || nrhs > 1024) throw Error(MSPCG_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    if (!h->have_params) throw Error(MSPCG_ERR_NO_PARAMS, "Mobius parameters not set");
    *estimate = estimate_solve_bytes(h, nrhs);
    *allocated = h->ws_bytes();
    return MSPCG_OK;
  });
}

mspcg_status mspcg_autotune(mspcg_t h, int32_t nrhs) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    if (nrhs < 1 || nrhs > 1024) throw Error(MSPCG_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    autotune_impl(h, nrhs, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return MSPCG_OK;
  });
}

static std::tuple<int, int, int> sched_key(const mspcg_t h, int32_t kind, int32_t nrhs) {
  if (kind < 0 || kind > 2) throw Error(MSPCG_ERR_INVALID_ARG, "kind must be 0, 1 or 2");
  if (nrhs < 1 || nrhs > 1024) throw Error(MSPCG_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
  const Prec p = kind == 1 ? Prec::F64 : to_prec(kind == 0 ? h->sp.outer_prec : h->sp.inner_prec);
  const int k = (kind == 0 && p == Prec::F64) ? 1 : kind;
  return std::make_tuple(k, (int)p, (int)nrhs);
}

mspcg_status mspcg_set_schedule(mspcg_t h, int32_t kind, int32_t nrhs, int32_t order, int32_t xcd, int32_t tchunk) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    no_session(h);
    if (order < 0 || order > 1 || xcd < 0 || xcd > 1 || tchunk < 0 || tchunk > 4)
      throw Error(MSPCG_ERR_INVALID_ARG, "order and xcd must be 0 or 1, tchunk in [0, 4]");
    const auto key = sched_key(h, kind, nrhs);
    Sched sc;
    sc.order = order;
    sc.xcd = xcd;
    sc.tchunk = std::get<0>(key) == 2 ? 0 : tchunk;
    h->tuned[key] = sc;
    h->tuned_us.erase(key);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_get_tchunk(mspcg_t h, int32_t kind, int32_t nrhs, int32_t* tchunk) {
  return guarded([&]() -> mspcg_status {
    if (!h || !tchunk) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    const auto key = sched_key(h, kind, nrhs);
    *tchunk = h->sched(std::get<0>(key), (Prec)std::get<1>(key), nrhs).tchunk;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_get_schedule(mspcg_t h, int32_t kind, int32_t nrhs, int32_t* order, int32_t* xcd, double* us) {
  return guarded([&]() -> mspcg_status {
    if (!h || !order || !xcd || !us) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    if (kind < 0 || kind > 2) throw Error(MSPCG_ERR_INVALID_ARG, "kind must be 0, 1 or 2");
    const Prec p = kind == 1 ? Prec::F64 : to_prec(kind == 0 ? h->sp.outer_prec : h->sp.inner_prec);
    const int k = (kind == 0 && p == Prec::F64) ? 1 : kind;
    const Sched sc = h->sched(k, p, nrhs);
    *order = sc.order;
    *xcd = sc.xcd;
    auto it = h->tuned_us.find(std::make_tuple(k, (int)p, nrhs));
    *us = it == h->tuned_us.end() ? 0.0 : it->second;
    return MSPCG_OK;
  });
}

// the size limits an operator application depends on: region fields in the
// requested precision only for the operators that use them (A_s and the
// preconditioner)
static void check_op_limits(const mspcg_ctx* h, int32_t op, mspcg_prec prec) {
  const bool regions = h->have_tiling && (op == MSPCG_OP_A_SUB || op == MSPCG_OP_PRECOND);
  check_limits(h->dims, h->Ls, regions ? h->nsub : 0, regions ? h->nN2 : 0, (int)prec);
}

mspcg_status mspcg_apply_device(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out,
                                void* hip_stream) {
  return guarded([&]() -> mspcg_status {
    if (!h || !in || !out) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (op < MSPCG_OP_DSLASH_EO || op > MSPCG_OP_STORE) throw Error(MSPCG_ERR_INVALID_ARG, "unknown operator");
    const Prec P = to_prec(prec);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    check_op_limits(h, op, prec);
    h->ensure_hip();
    apply_impl(h, op, P, in, out, hip_stream ? (hipStream_t)hip_stream : h->stream);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_apply_device_noalloc(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out,
                                        void* hip_stream) {
  return guarded([&]() -> mspcg_status {
    if (!h || !in || !out) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (op < MSPCG_OP_DSLASH_EO || op > MSPCG_OP_STORE) throw Error(MSPCG_ERR_INVALID_ARG, "unknown operator");
    const Prec P = to_prec(prec);
    need_state(h);
    if (!h->hip_ready || !h->scratch) throw Error(MSPCG_ERR_NO_GAUGE, "handle not initialised on its device");
    if (op == MSPCG_OP_PRECOND && h->Lh > 0)
      throw Error(MSPCG_ERR_INVALID_ARG, "the reduced-Ls preconditioner is not available without allocation");
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    check_op_limits(h, op, prec);
    HIPCHK(hipSetDevice(h->device));
    struct Restore {   // leave the handle as it was, also on an error
      mspcg_ctx* h;
      bool prof;
      ~Restore() {
        h->arena = mspcg_ctx::Arena();
        h->arena_ws.clear();
        h->profiling = prof;
      }
    } restore{h, h->profiling};
    h->profiling = false;   // no event creation inside this call
    h->arena_ws.clear();
    h->arena.base = static_cast<char*>(h->scratch);
    h->arena.cap = kScratchBytes;
    h->arena.off = 0;
    apply_impl(h, op, P, in, out, hip_stream ? (hipStream_t)hip_stream : h->stream);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_apply(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out) {
  return guarded([&]() -> mspcg_status {
    if (!h || !in || !out) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    no_session(h);
    if (op < MSPCG_OP_DSLASH_EO || op > MSPCG_OP_STORE) throw Error(MSPCG_ERR_INVALID_ARG, "unknown operator");
    const Prec P = to_prec(prec);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    check_op_limits(h, op, prec);
    h->ensure_hip();
    const size_t bytes = (size_t)h->n5() * 24 * sizeof(double);
    DevBuf di, dout;
    di.ensure(bytes);
    dout.ensure(bytes);
    h->upload(di.p, in, bytes, h->stream);
    apply_impl(h, op, P, di.as<double>(), dout.as<double>(), h->stream);
    h->download(out, dout.p, bytes, h->stream);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_get_history(mspcg_t h, double* out, double* pap, int32_t max, int32_t* count) {
  return guarded([&]() -> mspcg_status {
    if (!h || !count || (max > 0 && !out)) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    if (max < 0) throw Error(MSPCG_ERR_INVALID_ARG, "max must be >= 0");
    const int n = (int)std::min<size_t>((size_t)max, h->history.size());
    for (int i = 0; i < n; ++i) out[i] = h->history[(size_t)i];
    if (pap)
      for (int i = 0; i < n; ++i) pap[i] = (size_t)i < h->history_pap.size() ? h->history_pap[(size_t)i] : 0.0;
    *count = (int32_t)h->history.size();
    return MSPCG_OK;
  });
}

mspcg_status mspcg_cb_open(mspcg_t h, int32_t slots, void* hip_stream) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    if (slots < 1 || slots > 1024) throw Error(MSPCG_ERR_INVALID_ARG, "slots must be in [1, 1024]");
    no_session(h);
    need_state(h);
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    h->ensure_hip();
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->stream;
    h->cb = std::make_shared<CBSession>(h, slots, s);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_cb_submit(mspcg_t h, const double* b, double* x, int32_t* slot) {
  return guarded([&]() -> mspcg_status {
    if (!h || !b || !x || !slot) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    if (!h->cb) throw Error(MSPCG_ERR_INVALID_ARG, "no continuous-batching session is open");
    *slot = -1;
    auto& sl = h->cb->slots;
    for (size_t i = 0; i < sl.size(); ++i)
      if (sl[i].state == SLOT_FREE) {
        sl[i].state = SLOT_PENDING;
        sl[i].b = b;
        sl[i].x = x;
        *slot = (int32_t)i;
        return MSPCG_OK;
      }
    g_last_error = "every slot is taken";
    return MSPCG_BUSY;
  });
}

mspcg_status mspcg_cb_step(mspcg_t h, int32_t* running, int32_t* pending) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    if (!h->cb) throw Error(MSPCG_ERR_INVALID_ARG, "no continuous-batching session is open");
    std::shared_lock<std::shared_mutex> engine_lock(g_engine_gate);
    HIPCHK(hipSetDevice(h->device));
    int r = 0, p = 0;
    h->cb->step(&r, &p);
    if (running) *running = r;
    if (pending) *pending = p;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_cb_poll(mspcg_t h, int32_t slot, int32_t* done, mspcg_stats* st) {
  return guarded([&]() -> mspcg_status {
    if (!h || !done) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    if (!h->cb) throw Error(MSPCG_ERR_INVALID_ARG, "no continuous-batching session is open");
    auto& sl = h->cb->slots;
    if (slot < 0 || (size_t)slot >= sl.size()) throw Error(MSPCG_ERR_INVALID_ARG, "slot out of range");
    *done = sl[slot].state == SLOT_DONE ? 1 : 0;
    if (*done) {
      if (st) *st = sl[slot].stats;
      sl[slot].state = SLOT_FREE;
    }
    return MSPCG_OK;
  });
}

mspcg_status mspcg_cb_close(mspcg_t h) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    if (h->cb) {
      HIPCHK(hipSetDevice(h->device));
      h->cb.reset();
    }
    return MSPCG_OK;
  });
}

mspcg_status mspcg_set_profiling(mspcg_t h, int32_t on) {
  return guarded([&]() -> mspcg_status {
    if (!h) throw Error(MSPCG_ERR_INVALID_ARG, "null handle");
    if (h->hip_ready) HIPCHK(hipStreamSynchronize(h->stream));
    if (on < 0) throw Error(MSPCG_ERR_INVALID_ARG, "on must be >= 0");
    h->profiling = on != 0;
    h->prof_stride = on > 1 ? on : 1;
    for (int64_t& c : h->prof_count) c = 0;
    h->ev_used = 0;
    h->ev_log.clear();
    return MSPCG_OK;
  });
}

mspcg_status mspcg_get_kernel_time(mspcg_t h, int32_t kind, int64_t* launches, double* ms) {
  return guarded([&]() -> mspcg_status {
    if (!h || !launches || !ms) throw Error(MSPCG_ERR_INVALID_ARG, "null argument");
    *launches = 0;
    *ms = 0;
    if (!h->hip_ready) return MSPCG_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    auto match = [kind](int k) {
      switch (kind) {
        case 0: return k >= 20 && k < 30;
        case 1: return k >= 10 && k < 20;
        case 3: return k >= 30 && k < 40;
        default: return k == kind;
      }
    };
    for (auto& kv : h->ev_log) {
      if (!match(kv.first)) continue;
      float m = 0;
      HIPCHK(hipEventElapsedTime(&m, h->ev_pool[kv.second].a, h->ev_pool[kv.second].b));
      *ms += m;
      ++*launches;
    }
    return MSPCG_OK;
  });
}

const char* mspcg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
