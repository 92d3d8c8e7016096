// librve C ABI: context, workspace, transform tables and the PCG driver.
//
// The driver enqueues every step of the corrector path as HIP kernels on the
// context's stream. The PCG iterations run in chunks of RVE_DIRECTION_RING
// iterations whose launches do not depend on the chunk's position (the
// iteration counter lives on the device), so a chunk is captured once as a
// HIP graph and replayed; the host only polls a pinned all-converged counter
// once per chunk, keeping one chunk queued ahead so the GPU does not drain
// while it waits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rve.h"
#include "launch.h"

using namespace rve;

static_assert(kRing == RVE_DIRECTION_RING, "direction ring length must match the header");

namespace {

constexpr int kMinN = 64, kMaxN = 4096;
constexpr int kMaxN3 = 256;   // three dimensions: n^3 nodes per system

// Scratch of rve_grad_noalloc: a fixed device array, one per GPU, held until
// the process ends. Host code never passes this name to a kernel (on the
// host it is only a stand-in for the symbol): rve_create looks up its device
// address with hipGetSymbolAddress and keeps it in the context.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

struct Tables {
  double* q64 = nullptr;
  float* q32 = nullptr;
  __bf16* q16 = nullptr;
  double* einv64 = nullptr;
  float* einv32 = nullptr;
  double* einv64_fd = nullptr;   // 1/E of the finite-difference Laplacian (five-point scheme)
  float* einv32_fd = nullptr;
  __bf16* ch16 = nullptr;   // [n/2][n/2] cos(2 pi k t / n)/sqrt(n), row k (n % 256 == 0 only)
  __bf16* sh16 = nullptr;   // [n/2][n/2] sin(2 pi k t / n)/sqrt(n)
  double* einv3_64 = nullptr;   // [n][n][n] 1/E of the 3D operator, built on first use
  float* einv3_32 = nullptr;
  // FP16 transforms: Q in FP16 and E_min / E (entries <= 1) per scheme
  _Float16* qh = nullptr;
  float* einvh = nullptr;
  float* einvh_fd = nullptr;
  float* einv3h = nullptr;
  double emin = 1.0, emin_fd = 1.0, emin3 = 1.0;
  float* sin2 = nullptr;   // [n] sin^2(pi k / n) (the 16-bit transforms form 1/E from it)
  int cus = 0;             // compute units of the device
};

// Timed kernels: 0 fused direction step + operator apply, 1..4 the four
// transform GEMMs of the preconditioner, 5 residual update, 6 iterate update
// from the direction ring.
constexpr int kTimedClasses = 7;

struct EventTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> pairs;   // (class, first event index)
  size_t used = 0;
  double ms[kTimedClasses] = {0, 0, 0, 0, 0, 0, 0};
  long long count[kTimedClasses] = {0, 0, 0, 0, 0, 0, 0};
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

}  // namespace

// Autotuner key: (kind, n, precision, floor(log2 B)); kind 0 = shape of the
// FP64 operator apply, 1 = transform-GEMM tile variant, 2 = shape of the FP32
// operator apply.
using TuneKey = std::tuple<int, int, int, int>;

struct rve_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;   // private stream the iteration chunks are captured on
  int graphs = 1;                     // replay captured chunks (1) or launch them one by one (0)
  int force_stencil = -1;             // operator-apply shape to use instead of the tuner's (-1: none)
  int force_update = -1;              // shape of the recomputing residual update (-1: the tuner's, or
                                      // force_stencil when that is set)
  int force_gemm = -1;                // transform-GEMM variant to use instead of the tuner's (-1: none)
  int small_solver = 1;               // single-workgroup PCG where it fits (n = 64, FP64)
  int direction_update = 1;           // the last transform forms the next direction where it can
  int direction_bf16 = 1;             // ... in BF16 (16-bit transforms; n, contrast: kDir16Max*)
  std::map<std::vector<long long>, hipGraphExec_t> graph_cache;
  int autotune = 1;
  std::map<TuneKey, int> tune;
  std::string tune_path;     // JSON-lines cache of tuned choices, or empty
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::map<int, Tables> tables;
  int* h_count = nullptr;   // pinned: 2 convergence-poll slots, then the not-two-valued flag
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  bool timing = false;
  EventTimer timer;
  double* one_out = nullptr;   // device staging of rve_solve's and rve_dos_plan's host outputs (16 doubles)
  char* noalloc_scratch = nullptr;   // device address of this device's `scratch` array
};

namespace {

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) {                             \
      fprintf(stderr, "librve: %s failed: %s\n", #expr, hipGetErrorString(e_)); \
      return RVE_EHIP;                                  \
    }                                                   \
  } while (0)

inline void ignore(hipError_t) {}

bool n_supported(int n) { return n >= kMinN && n <= kMaxN && n % 64 == 0; }
bool n_supported3(int n) { return n >= kMinN && n <= kMaxN3 && n % 64 == 0; }

// Errors (negative codes) dominate warnings; among equals the larger magnitude.
int worse(int x, int y) { return (x < 0 || y < 0) ? std::min(x, y) : std::max(x, y); }

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Host tables for the Hartley transform of size n, in FP64: exact integer
// reduction of k*j mod n before the angle, host libm cos/sin.
int build_tables(rve_ctx* ctx, int n, Tables** out) {
  auto it = ctx->tables.find(n);
  if (it != ctx->tables.end()) {
    *out = &it->second;
    return RVE_OK;
  }
  const size_t N2 = (size_t)n * n;
  std::vector<double> q(N2), einv(N2), einvf(N2);
  std::vector<float> q32(N2), einv32(N2), einvf32(N2);
  std::vector<__bf16> q16(N2);
  const double two_pi = 6.283185307179586476925286766559;
  const double inv_sqrt = 1.0 / std::sqrt((double)n);
  std::vector<double> cas(n), c(n);
  for (int m = 0; m < n; ++m) {
    const double ang = two_pi * (double)m / (double)n;
    cas[m] = (std::cos(ang) + std::sin(ang)) * inv_sqrt;
    c[m] = std::cos(ang);
  }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) {
      const double v = cas[(size_t)((long long)k * j % n)];
      q[(size_t)k * n + j] = v;
      q32[(size_t)k * n + j] = (float)v;
      q16[(size_t)k * n + j] = (__bf16)(float)v;
    }
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < n; ++l) {
      const double E = (8.0 - 2.0 * c[k] - 2.0 * c[l] - 4.0 * c[k] * c[l]) / 3.0;
      const double inv = (k == 0 && l == 0) ? 0.0 : 1.0 / E;
      einv[(size_t)k * n + l] = inv;
      einv32[(size_t)k * n + l] = (float)inv;
      // five-point: (2 - 2 c_k) + (2 - 2 c_l)
      const double Ef = 4.0 - 2.0 * c[k] - 2.0 * c[l];
      const double invf = (k == 0 && l == 0) ? 0.0 : 1.0 / Ef;
      einvf[(size_t)k * n + l] = invf;
      einvf32[(size_t)k * n + l] = (float)invf;
    }
  // half-size cosine and sine parts of Q for the even/odd-folded transform
  const int h = n / 2;
  const size_t H2 = (size_t)h * h;
  std::vector<__bf16> ch(H2), sh(H2);
  for (int k = 0; k < h; ++k)
    for (int j = 0; j < h; ++j) {
      const double ang = two_pi * (double)((long long)k * j % n) / (double)n;
      ch[(size_t)k * h + j] = (__bf16)(float)(std::cos(ang) * inv_sqrt);
      sh[(size_t)k * h + j] = (__bf16)(float)(std::sin(ang) * inv_sqrt);
    }
  // FP16: Q rounded to FP16, and 1/E scaled by the smallest nonzero E
  std::vector<_Float16> qh(N2);
  for (size_t i = 0; i < N2; ++i) qh[i] = (_Float16)(float)q[i];
  double emin = 1e300, emin_fd = 1e300;
  for (size_t i = 1; i < N2; ++i) {
    emin = std::min(emin, 1.0 / einv[i]);
    emin_fd = std::min(emin_fd, 1.0 / einvf[i]);
  }
  std::vector<float> einvh(N2), einvh_fd(N2);
  for (size_t i = 0; i < N2; ++i) {
    einvh[i] = (float)(einv[i] * emin);
    einvh_fd[i] = (float)(einvf[i] * emin_fd);
  }
  std::vector<float> sin2(n);
  for (int k = 0; k < n; ++k) {
    const double sk = std::sin(0.5 * two_pi * (double)k / (double)n);
    sin2[k] = (float)(sk * sk);
  }
  Tables t;
  t.emin = emin;
  t.emin_fd = emin_fd;
  HIP_TRY(hipDeviceGetAttribute(&t.cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  if (hipMalloc(&t.sin2, (size_t)n * 4) != hipSuccess) return RVE_ENOMEM;
  HIP_TRY(hipMemcpy(t.sin2, sin2.data(), (size_t)n * 4, hipMemcpyHostToDevice));
  if (hipMalloc(&t.qh, N2 * 2) != hipSuccess || hipMalloc(&t.einvh, N2 * 4) != hipSuccess ||
      hipMalloc(&t.einvh_fd, N2 * 4) != hipSuccess) {
    ignore(hipFree(t.qh)); ignore(hipFree(t.einvh)); ignore(hipFree(t.einvh_fd));
    return RVE_ENOMEM;
  }
  HIP_TRY(hipMemcpy(t.qh, qh.data(), N2 * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einvh, einvh.data(), N2 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einvh_fd, einvh_fd.data(), N2 * 4, hipMemcpyHostToDevice));
  if (hipMalloc(&t.q64, N2 * 8) != hipSuccess || hipMalloc(&t.q32, N2 * 4) != hipSuccess ||
      hipMalloc(&t.q16, N2 * 2) != hipSuccess || hipMalloc(&t.einv64, N2 * 8) != hipSuccess ||
      hipMalloc(&t.einv32, N2 * 4) != hipSuccess || hipMalloc(&t.ch16, H2 * 2) != hipSuccess ||
      hipMalloc(&t.sh16, H2 * 2) != hipSuccess || hipMalloc(&t.einv64_fd, N2 * 8) != hipSuccess ||
      hipMalloc(&t.einv32_fd, N2 * 4) != hipSuccess) {
    ignore(hipFree(t.q64)); ignore(hipFree(t.q32)); ignore(hipFree(t.q16));
    ignore(hipFree(t.einv64)); ignore(hipFree(t.einv32)); ignore(hipFree(t.ch16)); ignore(hipFree(t.sh16));
    ignore(hipFree(t.einv64_fd)); ignore(hipFree(t.einv32_fd));
    return RVE_ENOMEM;
  }
  HIP_TRY(hipMemcpy(t.q64, q.data(), N2 * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.q32, q32.data(), N2 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.q16, q16.data(), N2 * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einv64, einv.data(), N2 * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einv32, einv32.data(), N2 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.ch16, ch.data(), H2 * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einv64_fd, einvf.data(), N2 * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.einv32_fd, einvf32.data(), N2 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t.sh16, sh.data(), H2 * 2, hipMemcpyHostToDevice));
  ctx->tables[n] = t;
  *out = &ctx->tables[n];
  return RVE_OK;
}

// The 3D symbol's reciprocal (kappa = 2 - 2c, mu = (4 + 2c)/6, c = cos(2 pi k / n)):
// E = kappa_k mu_l mu_m + mu_k kappa_l mu_m + mu_k mu_l kappa_m, (0,0,0) -> 0.
int build_tables3(rve_ctx* ctx, int n, Tables** out) {
  int rc = build_tables(ctx, n, out);
  if (rc) return rc;
  Tables* t = *out;
  if (t->einv3_64) return RVE_OK;
  const size_t N3 = (size_t)n * n * n;
  std::vector<double> e64(N3);
  std::vector<float> e32(N3);
  std::vector<double> kap(n), mu(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < n; ++k) {
    const double c = std::cos(two_pi * (double)k / (double)n);
    kap[k] = 2.0 - 2.0 * c;
    mu[k] = (4.0 + 2.0 * c) / 6.0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double E = kap[i] * mu[j] * mu[k] + mu[i] * kap[j] * mu[k] + mu[i] * mu[j] * kap[k];
        const double inv = (i == 0 && j == 0 && k == 0) ? 0.0 : 1.0 / E;
        const size_t o = ((size_t)i * n + j) * n + k;
        e64[o] = inv;
        e32[o] = (float)inv;
      }
  double emin3 = 1e300;
  for (size_t i = 1; i < N3; ++i) emin3 = std::min(emin3, 1.0 / e64[i]);
  std::vector<float> eh(N3);
  for (size_t i = 0; i < N3; ++i) eh[i] = (float)(e64[i] * emin3);
  double* d64 = nullptr;
  float* d32 = nullptr;
  float* dh = nullptr;
  if (hipMalloc(&d64, N3 * 8) != hipSuccess || hipMalloc(&d32, N3 * 4) != hipSuccess ||
      hipMalloc(&dh, N3 * 4) != hipSuccess) {
    ignore(hipFree(d64));
    ignore(hipFree(d32));
    ignore(hipFree(dh));
    (void)hipGetLastError();
    return RVE_ENOMEM;
  }
  HIP_TRY(hipMemcpy(d64, e64.data(), N3 * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d32, e32.data(), N3 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dh, eh.data(), N3 * 4, hipMemcpyHostToDevice));
  t->einv3_64 = d64;
  t->einv3_32 = d32;
  t->einv3h = dh;
  t->emin3 = emin3;
  return RVE_OK;
}

// The transform-GEMM type of an rve_precision.
int gemm_prec(int prec) {
  return prec == RVE_FP64 ? kGemmF64 : prec == RVE_MIX_FP32 ? kGemmF32 : prec == RVE_MIX_FP16 ? kGemmF16 : kGemmBF16;
}

// The tables one precision, scheme and dimension use.
GemmTables gemm_tables(const Tables* tb, int prec, int scheme) {
  GemmTables g;
  const bool fd = scheme == RVE_SCHEME_FD5;
  g.einv64 = fd ? tb->einv64_fd : tb->einv64;
  g.einv3_64 = tb->einv3_64;
  g.ch16 = tb->ch16;
  g.sh16 = tb->sh16;
  g.sin2 = tb->sin2;
  g.fd = fd ? 1 : 0;
  g.cus = tb->cus;
  if (prec == RVE_MIX_FP16) {
    g.q = tb->qh;
    g.einv32 = fd ? tb->einvh_fd : tb->einvh;
    g.einv3_32 = tb->einv3h;
    g.emin = fd ? tb->emin_fd : tb->emin;
  } else {
    g.q = prec == RVE_FP64 ? (const void*)tb->q64 : prec == RVE_MIX_FP32 ? (const void*)tb->q32
                                                                         : (const void*)tb->q16;
    g.einv32 = fd ? tb->einv32_fd : tb->einv32;
    g.einv3_32 = tb->einv3_32;
  }
  return g;
}

// Workspace: a control block shared by every batch of a solve (iteration
// counter, per-iteration counts of systems still iterating), then one region
// per equal-n batch, carved by plan() with offsets from the region start.
struct Layout {
  size_t off_a, off_a8, off_a32, off_f, off_x, off_r, off_ring, off_ahist, off_q, off_z, off_rlo, off_u1, off_u2, off_sys,
      off_real;
  size_t off_pq, off_rr, off_rzo, off_rz, off_misc, off_status, total;
};

Layout plan(int B, int n, int prec, int sprec, int scheme, int dim, Work* w) {
  Layout L{};
  const long long S = (long long)dim * B, N2 = dim == 3 ? (long long)n * n * n : (long long)n * n;
  // RHS / A_hom / gradient tiles per realization
  const int P_tile = dim == 3 ? tiles3(n) : (n / kTile) * (n / kTile);
  const int sc = stencil_choice_default(n);
  const int P_st = dim == 3 ? tiles3(n) : stencil_tiles_per_realization(n, sc);
  long long vb = N2 / 1024;
  if (vb > 256) vb = 256;
  if (vb < 1) vb = 1;
  const int P_vec = (int)vb;
  const int gp = gemm_prec(prec);
  const int gv = dim == 2 && gemm_variant_valid(n, gp, 1) ? 1 : 0;
  const int P_gemm = dim == 3 ? gemm_tiles_per_system3(n) : gemm_tiles_per_system(n, gp, gv);
  const int misc_nv = dim == 3 ? kMiscNV3 : kMiscNV;
  const size_t vec = align_up((size_t)(S * N2) * 8);
  const size_t pzvec = align_up((size_t)(S * N2) * (prec == RVE_FP64 ? 8 : 4));
  const size_t uvec = align_up((size_t)(S * N2) * gemm_elem_size(gp));
  size_t o = 0;
  // the batch's coefficients, copied in at the start of a solve: the
  // captured chunks then reference workspace memory only
  L.off_a = o; o += align_up((size_t)(B * N2) * 8);
  // one byte per cell for two-valued fields (FP64 operator apply, 2D)
  L.off_a8 = o; o += (dim == 2 && !sprec) ? align_up((size_t)(B * N2)) : 0;
  // FP32 operator apply: FP32 coefficients and the right-hand sides
  L.off_a32 = o; o += sprec ? align_up((size_t)(B * N2) * 4) : 0;
  L.off_f = o; o += sprec ? vec : 0;
  L.off_x = o; o += vec;
  L.off_r = o; o += vec;
  // direction ring: one slot more in 2D, for the last transform writing the
  // next direction before the chunk's fold (Work::pdirect)
  const int ring_slots = dim == 2 ? kRing + 1 : kRing;
  L.off_ring = o; o += (size_t)ring_slots * pzvec;
  L.off_ahist = o; o += align_up((size_t)S * ring_slots * 8);
  L.off_q = o; o += vec;
  L.off_z = o; o += pzvec;
  L.off_rlo = o; o += prec == RVE_FP64 ? 0 : uvec;
  L.off_u1 = o; o += uvec;
  L.off_u2 = o; o += uvec;
  L.off_sys = o; o += align_up(S * sizeof(SysState));
  L.off_real = o; o += align_up(B * sizeof(RealState));
  L.off_pq = o; o += align_up(S * std::max(P_tile, P_st) * 8);
  // r.r / r.z_old partials: per vector workgroup, or per apply tile of the
  // recomputing residual update (at most (n/64)^2 tiles per realization)
  const long long P_rr_max = dim == 3 ? P_vec : std::max<long long>(P_vec, (long long)(n / kWave) * (n / kWave));
  L.off_rr = o; o += align_up(S * P_rr_max * 8);
  L.off_rzo = o; o += align_up(S * P_rr_max * 8);
  L.off_rz = o; o += align_up(S * (dim == 3 ? gemm_tiles_per_system3(n) : gemm_tiles_per_system_max(n)) * 8);
  L.off_misc = o; o += align_up((size_t)B * P_tile * misc_nv * 8);
  L.off_status = o; o += align_up((size_t)B * sizeof(int));
  L.total = o;
  w->B = B;
  w->n = n;
  w->dim = dim;
  w->S = (int)S;
  w->N2 = N2;
  w->P_tile = P_tile;
  w->P_st = P_st;
  w->P_vec = P_vec;
  w->P_rr = P_vec;
  w->qfree = 0;
  w->P_gemm = P_gemm;
  w->mixed = gp;   // GemmPrec: 0 FP64, 1 FP32, 2 BF16, 3 FP16
  w->stencil = sc;
  w->ustencil = sc;
  w->m_ring = kRing;
  w->sprec = sprec;
  w->scheme = scheme;
  w->gemm_variant = gv;
  return L;
}

// Control block: kiter at the start, the not-two-valued flag at byte
// kTwoValuedFlagOffset, count[count_len] after the first 256 bytes.
constexpr size_t kTwoValuedFlagOffset = 64;
size_t ctl_bytes(int count_len) { return align_up(256) + align_up((size_t)count_len * sizeof(int)); }

void clear_graphs(rve_ctx* ctx) {
  for (auto& kv : ctx->graph_cache) ignore(hipGraphExecDestroy(kv.second));
  ctx->graph_cache.clear();
}

int ensure_ws(rve_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return RVE_OK;
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    clear_graphs(ctx);   // captured chunks point into the old arena
    ignore(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return RVE_ENOMEM;
  }
  ctx->ws_bytes = bytes;
  return RVE_OK;
}

void bind(char* base, const Layout& L, Work* w) {
  w->x = reinterpret_cast<double*>(base + L.off_x);
  w->r = reinterpret_cast<double*>(base + L.off_r);
  w->pring = base + L.off_ring;
  w->alpha_hist = reinterpret_cast<double*>(base + L.off_ahist);
  w->q = reinterpret_cast<double*>(base + L.off_q);
  w->z = base + L.off_z;
  w->rlo = w->mixed ? base + L.off_rlo : nullptr;
  w->u1 = base + L.off_u1;
  w->u2 = base + L.off_u2;
  w->sys = reinterpret_cast<SysState*>(base + L.off_sys);
  w->real = reinterpret_cast<RealState*>(base + L.off_real);
  w->part_pq = reinterpret_cast<double*>(base + L.off_pq);
  w->part_rr = reinterpret_cast<double*>(base + L.off_rr);
  w->part_rzo = reinterpret_cast<double*>(base + L.off_rzo);
  w->part_rz = reinterpret_cast<double*>(base + L.off_rz);
  w->part_misc = reinterpret_cast<double*>(base + L.off_misc);
  w->a32 = w->sprec ? reinterpret_cast<const float*>(base + L.off_a32) : nullptr;
  w->f = w->sprec ? reinterpret_cast<double*>(base + L.off_f) : nullptr;
}

// The context's small device buffer for results that go to the host.
int ensure_one_out(rve_ctx* ctx) {
  if (ctx->one_out) return RVE_OK;
  if (hipMalloc(reinterpret_cast<void**>(&ctx->one_out), 16 * sizeof(double)) != hipSuccess) {
    ctx->one_out = nullptr;
    (void)hipGetLastError();
    return RVE_ENOMEM;
  }
  return RVE_OK;
}

int check_opts(const rve_opts* o) {
  if (!o) return RVE_EINVAL;
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return RVE_EINVAL;
  if (o->maxit < 1 || o->maxit > 1000000) return RVE_EINVAL;
  if (o->prec < RVE_FP64 || o->prec > RVE_MIX_FP16) return RVE_EINVAL;
  if (o->stencil_prec != RVE_STENCIL_FP64 && o->stencil_prec != RVE_STENCIL_FP32) return RVE_EINVAL;
  if (o->scheme != RVE_SCHEME_Q1 && o->scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  if (o->scheme == RVE_SCHEME_FD5 && o->stencil_prec != RVE_STENCIL_FP64) return RVE_EINVAL;
  return RVE_OK;
}

// Kernel-class timing with event pairs on the context stream (never used
// while a chunk is being captured: timing runs launch eagerly).
struct Timed {
  rve_ctx* ctx;
  int cls;
  Timed(rve_ctx* c, int k) : ctx(c), cls(k) {
    if (ctx->timing) {
      hipEvent_t e = ctx->timer.next();
      if (e) {
        ctx->timer.pairs.push_back({cls, (int)ctx->timer.used - 1});
        ignore(hipEventRecord(e, ctx->stream));
      }
    }
  }
  ~Timed() {
    if (ctx->timing) {
      hipEvent_t e = ctx->timer.next();
      if (e) ignore(hipEventRecord(e, ctx->stream));
    }
  }
};

int harvest_timing(rve_ctx* ctx) {
  if (!ctx->timing) return RVE_OK;
  EventTimer& T = ctx->timer;
  for (auto& pr : T.pairs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, T.pool[pr.second], T.pool[pr.second + 1]) == hipSuccess) {
      T.ms[pr.first] += ms;
      T.count[pr.first] += 1;
    }
  }
  T.pairs.clear();
  T.used = 0;
  return RVE_OK;
}

int batch_bucket(int B) {
  int b = 0;
  while ((2 << b) <= B) ++b;
  return b;
}

void load_tune_cache(rve_ctx* ctx) {
  if (ctx->tune_path.empty()) return;
  FILE* f = fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    int kind, n, prec, bb, choice;
    if (sscanf(line, " {\"kind\": %d, \"n\": %d, \"prec\": %d, \"batch_log2\": %d, \"choice\": %d",
               &kind, &n, &prec, &bb, &choice) == 5)
      ctx->tune[TuneKey(kind, n, prec, bb)] = choice;
  }
  fclose(f);
}

void save_tune_entry(rve_ctx* ctx, const TuneKey& k, int choice, const std::vector<std::pair<int, float>>& ms) {
  if (ctx->tune_path.empty()) return;
  FILE* f = fopen(ctx->tune_path.c_str(), "a");
  if (!f) return;
  fprintf(f, "{\"kind\": %d, \"n\": %d, \"prec\": %d, \"batch_log2\": %d, \"choice\": %d, \"ms\": {",
          std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), choice);
  for (size_t i = 0; i < ms.size(); ++i) fprintf(f, "%s\"%d\": %.4f", i ? ", " : "", ms[i].first, ms[i].second);
  fprintf(f, "}}\n");
  fclose(f);
}

// Best of three event-timed runs of `launch` for each candidate; the
// launches must be idempotent (they are: the first PCG direction step and a
// preconditioner apply to a fixed residual). `pre` runs before each of them,
// outside the timed region.
struct NoPre {
  void operator()() const {}
};
template <class F, class P = NoPre>
int tune_pick(rve_ctx* ctx, const TuneKey& key, const std::vector<int>& cands, F launch, P pre = P()) {
  auto it = ctx->tune.find(key);
  // a cached choice is used only if it is a candidate for this shape
  if (it != ctx->tune.end() && std::find(cands.begin(), cands.end(), it->second) != cands.end())
    return it->second;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return cands[0];
  if (hipEventCreate(&e1) != hipSuccess) {
    ignore(hipEventDestroy(e0));
    return cands[0];
  }
  std::vector<std::pair<int, float>> times;
  int best = cands[0];
  float best_ms = 1e30f;
  for (int c : cands) {
    pre();
    launch(c);   // warm-up (code load, caches)
    float cbest = 1e30f;
    for (int r = 0; r < 3; ++r) {
      pre();
      ignore(hipEventRecord(e0, ctx->stream));
      launch(c);
      ignore(hipEventRecord(e1, ctx->stream));
      ignore(hipEventSynchronize(e1));
      float ms = 1e30f;
      if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < cbest) cbest = ms;
    }
    times.push_back({c, cbest});
    if (cbest < best_ms) {
      best_ms = cbest;
      best = c;
    }
  }
  ignore(hipEventDestroy(e0));
  ignore(hipEventDestroy(e1));
  ctx->tune[key] = best;
  save_tune_entry(ctx, key, best, times);
  return best;
}

// Number of systems that start iterating (read back once, for the tuner).
int count_active(rve_ctx* ctx, const Work& w) {
  std::vector<SysState> h(w.S);
  if (hipMemcpyAsync(h.data(), w.sys, w.S * sizeof(SysState), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return 0;
  int c = 0;
  for (const auto& s : h) c += s.active;
  return c;
}

// The four transform GEMMs, each bracketed by the timer when it is on.
void precond_timed(rve_ctx* ctx, const Work& w, int prec, const GemmTables& gt, hipStream_t st) {
  if (!ctx->timing) {
    launch_precond(w, prec, gt, st);
    return;
  }
  // classes 1..4: the first transform, the scaling one, the plain ones, the
  // last (2D: phases 0..3; 3D: 0, 2, {1, 3, 4}, 5)
  const int np = precond_phases(w);
  for (int ph = 0; ph < np; ++ph) {
    const int cls = np == 4 ? 1 + ph : ph == 0 ? 1 : ph == 2 ? 2 : ph == 5 ? 4 : 3;
    Timed t(ctx, cls);
    launch_precond(w, prec, gt, st, ph);
  }
}

// The preconditioner apply of one batch followed by beta (and, for the last
// batch of an iteration, the counter advance). With pdirect the four
// transforms are split around beta: the scaling transform's r.z partials
// give beta, and the last transform then writes p = z + beta p_old.
void precond_beta(rve_ctx* ctx, const Work& w, int prec, const GemmTables& gt, int flexible, int first,
                  hipStream_t st, int* advance) {
  if (!w.pdirect) {
    precond_timed(ctx, w, prec, gt, st);
    launch_scalar_beta(w, flexible, first, st, advance);
    return;
  }
  Work v = w;
  v.pdir_first = first;
  for (int ph = 0; ph < 4; ++ph) {
    if (ph == 2) launch_scalar_beta(v, flexible, first, st, nullptr);
    Timed t(ctx, 1 + ph);
    launch_precond(v, prec, gt, st, ph);
  }
  if (advance) launch_advance(advance, st);
}

// One equal-n batch of a solve: its inputs and outputs (device) and its
// workspace region.
struct Batch {
  int B = 0, n = 0;
  int dim = 2;
  const double* a = nullptr;                 // [B][n^dim], or the items below
  std::vector<const double*> a_items;        // item k's n x n cells (when not contiguous)
  double *phi = nullptr, *ahom = nullptr, *flux = nullptr, *relres = nullptr;
  int *iters = nullptr, *status = nullptr;
  Work w;
  Layout L;
  size_t base = 0;
  GemmTables gt;
  int prec = kGemmF64;
};

// One chunk of kRing PCG iterations for every batch: the fold of the previous
// chunk's directions into x, then per iteration and batch: operator apply
// with the direction step, alpha, residual update, stopping test, the four
// transforms z = B^+ r, beta; then the shared iteration counter advances.
// Nothing in it depends on the chunk's position, so it can be captured once
// and replayed.
void run_chunk(rve_ctx* ctx, std::vector<Batch>& bs, const rve_opts* o, int flexible, hipStream_t st) {
  for (auto& b : bs) {
    {
      Timed t(ctx, 6);
      launch_fold_x(b.w, 0, st);
    }
    // FP32 operator apply: the residual restarts from r = f - A x (FP64)
    if (b.w.sprec) launch_replace_r(b.w, st);
  }
  for (int it = 0; it < kRing; ++it) {
    for (auto& b : bs) {
      {
        Timed t(ctx, 0);
        launch_stencil_fused(b.w, st);
      }
      launch_scalar_alpha(b.w, st);
      {
        Timed t(ctx, 5);
        launch_update_r(b.w, flexible, st);
      }
      launch_scalar_conv(b.w, o->tol, o->maxit, st);
      // the last batch also advances the shared iteration counter
      precond_beta(ctx, b.w, b.prec, b.gt, flexible, 0, st, &b == &bs.back() ? bs[0].w.kiter : nullptr);
    }
  }
}

// The captured chunk for this exact set of batches (pointers, shapes, kernel
// choices, options), captured on first use.
int chunk_graph(rve_ctx* ctx, std::vector<Batch>& bs, const rve_opts* o, int flexible, hipGraphExec_t* out) {
  std::vector<long long> key;
  long long tolbits = 0;
  std::memcpy(&tolbits, &o->tol, sizeof tolbits);
  key.insert(key.end(), {(long long)(uintptr_t)ctx->ws, tolbits, o->maxit, flexible, o->stencil_prec, o->scheme,
                         (long long)bs.size()});
  for (auto& b : bs)
    key.insert(key.end(), {b.B, b.n, b.dim, b.prec, (long long)b.base, b.w.stencil, b.w.ustencil,
                           b.w.gemm_variant, b.w.a8 != nullptr, b.w.pdirect, b.w.pdir16});
  auto it = ctx->graph_cache.find(key);
  if (it != ctx->graph_cache.end()) {
    *out = it->second;
    return RVE_OK;
  }
  if (ctx->graph_cache.size() >= 32) clear_graphs(ctx);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  run_chunk(ctx, bs, o, flexible, ctx->cap_stream);
  const hipError_t launch_err = hipGetLastError();
  const hipError_t end_err = hipStreamEndCapture(ctx->cap_stream, &g);
  if (launch_err != hipSuccess || end_err != hipSuccess) {
    fprintf(stderr, "librve: capturing a PCG chunk failed: %s\n",
            hipGetErrorString(launch_err != hipSuccess ? launch_err : end_err));
    if (g) ignore(hipGraphDestroy(g));
    return RVE_EHIP;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  ignore(hipGraphDestroy(g));
  HIP_TRY(ie);
  ctx->graph_cache[key] = ex;
  *out = ex;
  return RVE_OK;
}

// Solve every batch (each B equal-size realizations) together: all batches
// step through the same PCG iterations, sharing one iteration counter and
// one convergence poll. `status_host` (optional) receives the per-item
// statuses, batch after batch.
int solve_batches(rve_ctx* ctx, std::vector<Batch>& bs, double h, const rve_opts* o,
                  std::vector<int>* status_host) {
  const int prec = gemm_prec(o->prec);
  // automatic: standard beta (the flexible form gave the same iteration counts
  // with the BF16/FP32 transforms at contrast 10 and 100)
  const int flexible = o->flexible < 0 ? 0 : (o->flexible != 0);
  const int count_len = o->maxit + kRing;
  size_t total = ctl_bytes(count_len);
  for (auto& b : bs) {
    b.L = plan(b.B, b.n, o->prec, o->stencil_prec, o->scheme, b.dim, &b.w);
    b.base = total;
    total += b.L.total;
  }
  int rc = ensure_ws(ctx, total);
  if (rc) return rc;
  char* ws = static_cast<char*>(ctx->ws);
  int* kiter = reinterpret_cast<int*>(ws);
  int* count = reinterpret_cast<int*>(ws + align_up(256));
  hipStream_t st = ctx->stream;
  for (auto& b : bs) {
    bind(ws + b.base, b.L, &b.w);
    double* a_ws = reinterpret_cast<double*>(ws + b.base + b.L.off_a);
    const size_t cells = (size_t)b.w.N2;
    if (b.a_items.empty()) {
      HIP_TRY(hipMemcpyAsync(a_ws, b.a, (size_t)b.B * cells * 8, hipMemcpyDeviceToDevice, st));
    } else {
      for (int k = 0; k < b.B; ++k)
        HIP_TRY(hipMemcpyAsync(a_ws + k * cells, b.a_items[k], cells * 8, hipMemcpyDeviceToDevice, st));
    }
    b.w.a = a_ws;
    b.w.kiter = kiter;
    b.w.count = count;
    if (!b.status) b.status = reinterpret_cast<int*>(ws + b.base + b.L.off_status);
    Tables* tb = nullptr;
    rc = b.dim == 3 ? build_tables3(ctx, b.n, &tb) : build_tables(ctx, b.n, &tb);
    if (rc) return rc;
    b.gt = gemm_tables(tb, o->prec, o->scheme);
    b.prec = prec;
  }

  // the smallest grid in FP64: one workgroup per system runs the whole PCG
  // in one launch (no iteration chunks, tuning or fold)
  bool small = ctx->small_solver != 0;
  for (auto& b : bs) small = small && small_solver_fits(b.w);
  // two-valued fields (every cell its realization's minimum or maximum, the
  // model of Sec. 2 eqns. Stoch-decomp and coef_diag): the operator kernels
  // read one byte per cell instead of eight, decoded exactly
  bool encode = !small;
  for (auto& b : bs) encode = encode && b.dim == 2 && !b.w.sprec;
  int* not_two_valued = reinterpret_cast<int*>(ws + kTwoValuedFlagOffset);

  launch_ctl_reset(kiter, count, count_len, st);
  for (auto& b : bs) {
    launch_init_state(b.w, st);
    launch_rhs(b.w, st);
    launch_scalar_init(b.w, st);
    if (encode)
      launch_encode_two_valued(b.w, reinterpret_cast<uint8_t*>(ws + b.base + b.L.off_a8), not_two_valued, st);
    launch_meansub(b.w, st);
    launch_scalar_fnorm(b.w, st);
    if (b.w.sprec) {
      HIP_TRY(hipMemcpyAsync(b.w.f, b.w.r, (size_t)b.w.S * b.w.N2 * 8, hipMemcpyDeviceToDevice, st));
      launch_to_f32(b.w.a, const_cast<float*>(b.w.a32), (long long)b.B * b.w.N2, st);
    }
  }
  // (bit 1 of the flag: a field of the solve exceeds the contrast of BF16
  // directions)
  bool low_contrast = false;
  if (encode) {
    HIP_TRY(hipMemcpyAsync(ctx->h_count + 2, not_two_valued, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if ((ctx->h_count[2] & 1) == 0)
      for (auto& b : bs) b.w.a8 = reinterpret_cast<const uint8_t*>(ws + b.base + b.L.off_a8);
    low_contrast = (ctx->h_count[2] & 2) == 0;
  }

  if (small) {
    for (auto& b : bs)
      launch_pcg_small(b.w, static_cast<const double*>(b.gt.q), b.gt.einv64, o->tol, o->maxit, st);
  } else {
  // kernel variants: defaults, or the autotuner's choice for each shape; then
  // z_0 and beta's first call for each batch
  for (auto& b : bs) {
    Work& w = b.w;
    const int n = b.n;
    if (b.dim == 3) {   // one operator-apply shape and one transform variant
      precond_beta(ctx, w, prec, b.gt, flexible, 1, st, nullptr);
      continue;
    }
    const int bb = batch_bucket(b.B);
    // kind 0: FP64 operator-apply shape, 2: FP32 apply, 3: five-point apply
    const TuneKey kst(w.sprec ? 2 : w.scheme ? 3 : 0, n, o->prec, bb), kgm(1, n, o->prec, bb);
    const bool tune_now = ctx->autotune && (!ctx->tune.count(kst) || !ctx->tune.count(kgm)) &&
                          (ctx->force_stencil < 0 || ctx->force_gemm < 0) && count_active(ctx, w) > 0;
    if (ctx->autotune) {
      std::vector<int> gc;
      // the even/odd-folded variant (2) is faster per apply but its extra BF16
      // rounding costs iterations (n = 512: 39.3 vs 38.0; n = 2048: 149 vs
      // 100), which a per-apply timing cannot see: it is used only on request
      // the 16-bit tile variants 1, 4, 5 and 6 accumulate every output and
      // every r.z partial in the same order, so the pick among them cannot
      // change a result; the 64 x 64 kernel (0), which forms r.z from the z
      // it writes instead, is a candidate only where none of them fits
      const bool h16_tiles = gemm_variant_valid(n, prec, 1);
      for (int v : {0, 1, 4, 5, 6})
        if (gemm_variant_valid(n, prec, v) && !(h16_tiles && v == 0)) gc.push_back(v);
      if (ctx->tune.count(kgm) || tune_now)
        w.gemm_variant = tune_pick(ctx, kgm, gc, [&](int v) {
          Work t2 = w;
          t2.gemm_variant = v;
          t2.P_gemm = gemm_tiles_per_system(n, prec, v);
          launch_precond(t2, prec, b.gt, st);
        });
    }
    if (ctx->force_gemm >= 0 && gemm_variant_valid(n, prec, ctx->force_gemm)) w.gemm_variant = ctx->force_gemm;
    w.P_gemm = gemm_tiles_per_system(n, prec, w.gemm_variant);
    // the last transform forms the next direction (standard beta, FP64 apply,
    // 16-bit tile transforms): bit-identical to the apply forming it
    w.pdirect = ctx->direction_update && !flexible && !w.sprec &&
                gemm_variant_writes_direction(n, prec, w.gemm_variant) ? 1 : 0;
    w.m_ring = w.pdirect ? kRing + 1 : kRing;
    // the directions the last transform forms are stored in BF16 (16-bit
    // transforms; they only steer the iteration: x and q = A p see the same
    // rounded p, so r = f - A x still holds to FP64 rounding), on grids up to
    // kDir16MaxN and for fields of contrast up to kDir16MaxContrast
    w.pdir16 =
        w.pdirect && ctx->direction_bf16 && (w.mixed == 2 || w.mixed == 3) && n <= kDir16MaxN && low_contrast ? 1 : 0;
    precond_beta(ctx, w, prec, b.gt, flexible, 1, st, nullptr);
    int sc = stencil_choice_default(n);
    // operator-apply shapes: V in {1, 2, 4}, H in {16, 64}, D in {1, 2, 4}
    std::vector<int> vc;
    for (int v : {1, 2, 4})
      for (int hs : {16, 64})
        for (int dc : {0, 64, 128}) {
          const int c = v + 8 * (hs / 16) + dc;
          if (stencil_choice_valid(n, c)) vc.push_back(c);
        }
    // Each probe of the two stencil passes follows the preconditioner's last
    // transform, as in the solve (rerun here on the first apply's
    // intermediate: it writes the same p_0 or z again), so the operand comes
    // from where the solve finds it; timed alone, shapes without row
    // prefetch probed as fast as the rest, then ran 15 % slower in the solve.
    auto follow_last = [&]() {
      Work v = w;
      v.pdir_first = 1;
      launch_precond(v, prec, b.gt, st, 3);
    };
    if (ctx->autotune) {
      // candidates are timed on probes of iteration 0 that also read the
      // previous direction's slot (zeroed here), i.e. do a later iteration's
      // work; iteration 0 then rewrites everything they wrote
      if (tune_now && !ctx->tune.count(kst)) {
        const size_t slot = (size_t)w.S * w.N2 * (w.pdir16 ? 2 : w.mixed ? 4 : 8);
        HIP_TRY(hipMemsetAsync(static_cast<char*>(w.pring) + (kRing - 1) * slot, 0, slot, st));
      }
      if (ctx->tune.count(kst) || tune_now)
        sc = tune_pick(
            ctx, kst, vc,
            [&](int c) {
              Work t2 = w;
              t2.stencil = c;
              t2.P_st = stencil_tiles_per_realization(n, c);
              launch_stencil_fused(t2, st, 1);
            },
            follow_last);
    }
    if (ctx->force_stencil >= 0 && stencil_choice_valid(n, ctx->force_stencil)) sc = ctx->force_stencil;
    w.stencil = sc;
    w.P_st = stencil_tiles_per_realization(n, sc);
    // FP64 apply: the residual update recomputes A p, in a tile shape of its
    // own (it streams r in and out besides the operand, so its best shape is
    // not the apply's); timed on probes that rewrite r unchanged
    if (!w.sprec) {
      w.qfree = 1;
      const TuneKey kup(w.scheme ? 5 : 4, n, o->prec, bb);
      int uc = sc;
      const bool forced = ctx->force_update >= 0 || ctx->force_stencil >= 0;
      if (ctx->autotune && !forced && (ctx->tune.count(kup) || count_active(ctx, w) > 0))
        uc = tune_pick(
            ctx, kup, vc,
            [&](int c) {
              Work t2 = w;
              t2.ustencil = c;
              t2.P_rr = stencil_tiles_per_realization(n, c);
              launch_update_r(t2, flexible, st, 1);
            },
            follow_last);
      if (ctx->force_update >= 0 && stencil_choice_valid(n, ctx->force_update)) uc = ctx->force_update;
      w.ustencil = uc;
      w.P_rr = stencil_tiles_per_realization(n, uc);
    }
  }

  // iterations in chunks of kRing, replayed from a captured graph unless
  // kernel timing is on; the host polls the count of the chunk before the one
  // just enqueued, so one chunk of work stays queued while it waits
  hipGraphExec_t ex = nullptr;
  if (ctx->graphs && !ctx->timing) {
    rc = chunk_graph(ctx, bs, o, flexible, &ex);
    if (rc) return rc;
  }
  const int max_chunks = (o->maxit + kRing - 1) / kRing;
  const int per_poll = o->check_every > 0 ? std::max(1, (o->check_every + kRing - 1) / kRing) : 1;
  for (int c = 0, polls = 0;; ++c) {
    if (ex)
      HIP_TRY(hipGraphLaunch(ex, st));
    else
      run_chunk(ctx, bs, o, flexible, st);
    const bool last = c + 1 >= max_chunks;
    if (!last && (c + 1) % per_poll != 0) continue;
    const int slot = polls & 1;
    HIP_TRY(hipMemcpyAsync(ctx->h_count + slot, count + (c * kRing + kRing - 1), sizeof(int),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(ctx->chunk_ev[slot], st));
    if (last) {
      HIP_TRY(hipEventSynchronize(ctx->chunk_ev[slot]));
      break;
    }
    if (polls > 0) {
      const int prev = slot ^ 1;
      HIP_TRY(hipEventSynchronize(ctx->chunk_ev[prev]));
      if (ctx->h_count[prev] == 0) break;
    }
    ++polls;
  }
  }   // not small

  for (auto& b : bs) {
    if (!small) {
      // the directions since the last fold
      Timed t(ctx, 6);
      launch_fold_x(b.w, 1, st);
    }
    launch_ahom(b.w, st);
    launch_scalar_ahom(b.w, b.ahom, b.flux, st);
    if (b.phi) launch_phi_out(b.w, b.phi, h, st);
    launch_finalize(b.w, b.iters, b.relres, b.status, st);
  }
  HIP_TRY(hipGetLastError());
  std::vector<int> hs;
  for (auto& b : bs) {
    const size_t o0 = hs.size();
    hs.resize(o0 + b.B);
    HIP_TRY(hipMemcpyAsync(hs.data() + o0, b.status, b.B * sizeof(int), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  harvest_timing(ctx);
  int worst = RVE_OK;
  for (int v : hs) worst = worse(worst, v);
  if (status_host) *status_host = hs;
  return worst;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

void rve_default_opts(rve_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->maxit = 2000;
  o->prec = RVE_FP64;
  o->flexible = -1;
  o->check_every = 0;
  o->stencil_prec = RVE_STENCIL_FP64;
  o->scheme = RVE_SCHEME_Q1;
}

const char* rve_status_string(int s) {
  switch (s) {
    case RVE_OK: return "RVE_OK: converged";
    case RVE_NOT_CONVERGED: return "RVE_NOT_CONVERGED: maxit reached";
    case RVE_BREAKDOWN: return "RVE_BREAKDOWN: non-positive or non-finite curvature in PCG";
    case RVE_EINVAL: return "RVE_EINVAL: invalid argument or coefficient";
    case RVE_EHIP: return "RVE_EHIP: HIP runtime error";
    case RVE_ENOMEM: return "RVE_ENOMEM: device allocation failed";
    default: return "unknown rve status";
  }
}

int rve_create(rve_ctx** out, int device, void* hip_stream) {
  if (!out) return RVE_EINVAL;
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(device));
  rve_ctx* c = new (std::nothrow) rve_ctx();
  if (!c) return RVE_ENOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // the device address of this device's copy of the fixed scratch array
  {
    void* sp = nullptr;
    const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !sp) {
      fprintf(stderr, "librve: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
      delete c;
      return RVE_EHIP;
    }
    c->noalloc_scratch = static_cast<char*>(sp);
  }
  if (const char* tp = std::getenv("RVE_TUNE_CACHE")) c->tune_path = tp;
  load_tune_cache(c);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_count), 4 * sizeof(int), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return RVE_ENOMEM;
  }
  if (hipEventCreateWithFlags(&c->chunk_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->chunk_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    ignore(hipHostFree(c->h_count));
    delete c;
    return RVE_EHIP;
  }
  *out = c;
  return RVE_OK;
}

int rve_destroy(rve_ctx* c) {
  if (!c) return RVE_EINVAL;
  ignore(hipSetDevice(c->device));
  ignore(hipStreamSynchronize(c->stream));
  for (auto& kv : c->tables) {
    ignore(hipFree(kv.second.q64));
    ignore(hipFree(kv.second.q32));
    ignore(hipFree(kv.second.q16));
    ignore(hipFree(kv.second.einv64));
    ignore(hipFree(kv.second.einv32));
    ignore(hipFree(kv.second.ch16));
    ignore(hipFree(kv.second.einv64_fd));
    ignore(hipFree(kv.second.einv32_fd));
    ignore(hipFree(kv.second.sh16));
    ignore(hipFree(kv.second.einv3_64));
    ignore(hipFree(kv.second.einv3_32));
    ignore(hipFree(kv.second.einv3h));
    ignore(hipFree(kv.second.qh));
    ignore(hipFree(kv.second.einvh));
    ignore(hipFree(kv.second.einvh_fd));
    ignore(hipFree(kv.second.sin2));
  }
  clear_graphs(c);
  if (c->ws) ignore(hipFree(c->ws));
  ignore(hipStreamDestroy(c->cap_stream));
  for (auto e : c->timer.pool) ignore(hipEventDestroy(e));
  ignore(hipEventDestroy(c->chunk_ev[0]));
  ignore(hipEventDestroy(c->chunk_ev[1]));
  ignore(hipHostFree(c->h_count));
  if (c->one_out) ignore(hipFree(c->one_out));
  delete c;
  return RVE_OK;
}

int rve_set_stream(rve_ctx* c, void* hip_stream) {
  if (!c) return RVE_EINVAL;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return RVE_OK;
}

int rve_solve_batch(rve_ctx* c, int B, int n, double h, const double* a_dev, const rve_opts* o,
                    double* phi_dev, double* ahom_dev, double* ahom_flux_dev, int* iters_dev,
                    double* relres_dev, int* status_dev) {
  if (!c || B < 1 || !n_supported(n) || !(h > 0.0) || !std::isfinite(h) || !a_dev || !ahom_dev)
    return RVE_EINVAL;
  if (check_opts(o)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  std::vector<Batch> bs(1);
  Batch& b = bs[0];
  b.B = B;
  b.n = n;
  b.a = a_dev;
  b.phi = phi_dev;
  b.ahom = ahom_dev;
  b.flux = ahom_flux_dev;
  b.iters = iters_dev;
  b.relres = relres_dev;
  b.status = status_dev;
  return solve_batches(c, bs, h, o, nullptr);
}

int rve_solve(rve_ctx* c, int n, double h, const double* a_dev, const rve_opts* o, double* phi_dev,
              double* ahom_host, double* ahom_flux_host, int* iters_host, double* relres_host) {
  if (!c || !n_supported(n) || !(h > 0.0) || !std::isfinite(h) || !a_dev || !ahom_host) return RVE_EINVAL;
  if (check_opts(o)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  int rc = ensure_one_out(c);
  if (rc) return rc;
  // staging: [0..3] A_hom, [4..7] flux form, [8..9] relres, then the ints
  // iters[2] and status in the bytes of [10..11]
  double* out = c->one_out;
  std::vector<Batch> bs(1);
  Batch& b = bs[0];
  b.B = 1;
  b.n = n;
  b.a = a_dev;
  b.phi = phi_dev;
  b.ahom = out;
  b.flux = out + 4;
  b.relres = out + 8;
  b.iters = reinterpret_cast<int*>(out + 10);
  b.status = reinterpret_cast<int*>(out + 11);
  rc = solve_batches(c, bs, h, o, nullptr);
  if (rc == RVE_EHIP || rc == RVE_ENOMEM) return rc;
  double host[12];
  HIP_TRY(hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(ahom_host, host, 4 * sizeof(double));
  if (ahom_flux_host) std::memcpy(ahom_flux_host, host + 4, 4 * sizeof(double));
  if (relres_host) std::memcpy(relres_host, host + 8, 2 * sizeof(double));
  if (iters_host) std::memcpy(iters_host, host + 10, 2 * sizeof(int));
  return rc;
}

// Launch-size bound of the 3D kernels: every grid stays below 2^31 workgroups.
static bool fits3(int B, int n) {
  const long long per = std::max<long long>(tiles3(n), gemm_tiles_per_system3(n));
  return (long long)B * 3 * per < (1LL << 31);
}

int rve_solve_batch_3d(rve_ctx* c, int B, int n, double h, const double* a_dev, const rve_opts* o,
                       double* phi_dev, double* ahom_dev, double* ahom_flux_dev, int* iters_dev,
                       double* relres_dev, int* status_dev) {
  if (!c || B < 1 || !n_supported3(n) || !fits3(B, n) || !(h > 0.0) || !std::isfinite(h) || !a_dev ||
      !ahom_dev)
    return RVE_EINVAL;
  if (check_opts(o)) return RVE_EINVAL;
  if (o->stencil_prec != RVE_STENCIL_FP64 || o->scheme != RVE_SCHEME_Q1) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  std::vector<Batch> bs(1);
  Batch& b = bs[0];
  b.B = B;
  b.n = n;
  b.dim = 3;
  b.a = a_dev;
  b.phi = phi_dev;
  b.ahom = ahom_dev;
  b.flux = ahom_flux_dev;
  b.iters = iters_dev;
  b.relres = relres_dev;
  b.status = status_dev;
  return solve_batches(c, bs, h, o, nullptr);
}

int rve_apply_operator_3d(rve_ctx* c, int B, int n, const double* a_dev, const double* u_dev, double* out_dev) {
  if (!c || B < 1 || !n_supported3(n) || !fits3(B, n) || !a_dev || !u_dev || !out_dev || u_dev == out_dev)
    return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_apply_stencil3(B, n, a_dev, u_dev, out_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_apply_precond_3d(rve_ctx* c, int B, int n, const double* a_dev, const double* r_dev, double* z_dev,
                         int prec) {
  if (!c || B < 1 || !n_supported3(n) || !fits3(B, n) || !a_dev || !r_dev || !z_dev || r_dev == z_dev)
    return RVE_EINVAL;
  if (prec < RVE_FP64 || prec > RVE_MIX_FP16) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  Work w;
  const Layout L = plan(B, n, prec, 0, RVE_SCHEME_Q1, 3, &w);
  int rc = ensure_ws(c, L.total);
  if (rc) return rc;
  bind(static_cast<char*>(c->ws), L, &w);
  w.a = a_dev;
  Tables* tb = nullptr;
  rc = build_tables3(c, n, &tb);
  if (rc) return rc;
  // a0 of each realization, exactly as the solver derives it
  launch_init_state(w, c->stream);
  launch_rhs(w, c->stream);
  launch_scalar_init(w, c->stream);
  const GemmTables gt = gemm_tables(tb, prec, RVE_SCHEME_Q1);
  w.r = const_cast<double*>(r_dev);
  w.sys = nullptr;
  if (w.mixed) launch_round_lo(w, c->stream);
  void* z_solver = w.z;
  w.z = w.mixed ? z_solver : (void*)z_dev;
  launch_precond(w, gemm_prec(prec), gt, c->stream);
  if (w.mixed) launch_widen(static_cast<const float*>(w.z), z_dev, (long long)w.S * w.N2, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_solve_uneven(rve_ctx* c, int B, const int* n_host, const int64_t* off, double h,
                     const double* a_dev, const rve_opts* o, double* phi_dev, double* ahom_dev,
                     double* ahom_flux_dev, int* iters_dev, double* relres_dev, int* status_dev) {
  if (!c || B < 1 || !n_host || !off || !(h > 0.0) || !std::isfinite(h) || !a_dev || !ahom_dev)
    return RVE_EINVAL;
  if (check_opts(o)) return RVE_EINVAL;
  // validate sizes and offsets: supported n, increasing, non-overlapping
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) {
    if (!n_supported(n_host[b]) || off[b] < 0) return RVE_EINVAL;
    order[b] = b;
  }
  // off[B] is the total extent of a_dev in elements; items must fit in it and
  // must not overlap each other
  std::sort(order.begin(), order.end(), [&](int x, int y) { return off[x] < off[y]; });
  for (int k = 0; k < B; ++k) {
    const int b = order[k];
    const int64_t end = off[b] + (int64_t)n_host[b] * n_host[b];
    if (end > off[B]) return RVE_EINVAL;
    if (k + 1 < B && end > off[order[k + 1]]) return RVE_EINVAL;
  }
  HIP_TRY(hipSetDevice(c->device));
  // group items by size; each group's items are copied into its workspace,
  // all groups are solved together (one chunk of iterations covers every
  // size), and the outputs, staged per group, are scattered back
  std::map<int, std::vector<int>> groups;
  for (int b = 0; b < B; ++b) groups[n_host[b]].push_back(b);
  size_t bytes = 0;
  for (auto& g : groups) {
    const size_t Bg = g.second.size(), N2 = (size_t)g.first * g.first;
    bytes += (phi_dev ? align_up(2 * Bg * N2 * 8) : 0) + 3 * align_up(Bg * 4 * 8) +
             2 * align_up(Bg * 2 * 4) + align_up(Bg * 4);
  }
  char* stage = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&stage), bytes, c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return RVE_ENOMEM;
  }
  size_t o2 = 0;
  auto take = [&](size_t nb) { char* p = stage + o2; o2 += align_up(nb); return p; };
  std::vector<Batch> bs;
  std::vector<const std::vector<int>*> members;
  for (auto& g : groups) {
    const int n = g.first;
    const std::vector<int>& items = g.second;
    const int Bg = (int)items.size();
    const size_t N2 = (size_t)n * n;
    Batch bt;
    bt.B = Bg;
    bt.n = n;
    for (int k = 0; k < Bg; ++k) bt.a_items.push_back(a_dev + off[items[k]]);
    if (phi_dev) bt.phi = reinterpret_cast<double*>(take(2 * Bg * N2 * 8));
    bt.ahom = reinterpret_cast<double*>(take(Bg * 4 * 8));
    bt.flux = reinterpret_cast<double*>(take(Bg * 4 * 8));
    bt.relres = reinterpret_cast<double*>(take(Bg * 4 * 8));
    bt.iters = reinterpret_cast<int*>(take(Bg * 2 * 4));
    bt.status = reinterpret_cast<int*>(take(Bg * 4));
    bs.push_back(bt);
    members.push_back(&items);
  }
  const int rc = solve_batches(c, bs, h, o, nullptr);
  if (rc == RVE_EHIP || rc == RVE_ENOMEM) {
    ignore(hipFreeAsync(stage, c->stream));
    return rc;
  }
  for (size_t gi = 0; gi < bs.size(); ++gi) {
    const Batch& bt = bs[gi];
    const size_t N2 = (size_t)bt.n * bt.n;
    const std::vector<int>& items = *members[gi];
    for (int k = 0; k < bt.B; ++k) {
      const int b = items[k];
      HIP_TRY(hipMemcpyAsync(ahom_dev + 4 * b, bt.ahom + 4 * k, 32, hipMemcpyDeviceToDevice, c->stream));
      if (ahom_flux_dev)
        HIP_TRY(hipMemcpyAsync(ahom_flux_dev + 4 * b, bt.flux + 4 * k, 32, hipMemcpyDeviceToDevice, c->stream));
      if (relres_dev)
        HIP_TRY(hipMemcpyAsync(relres_dev + 2 * b, bt.relres + 2 * k, 16, hipMemcpyDeviceToDevice, c->stream));
      if (iters_dev)
        HIP_TRY(hipMemcpyAsync(iters_dev + 2 * b, bt.iters + 2 * k, 8, hipMemcpyDeviceToDevice, c->stream));
      if (status_dev)
        HIP_TRY(hipMemcpyAsync(status_dev + b, bt.status + k, 4, hipMemcpyDeviceToDevice, c->stream));
      if (phi_dev)
        HIP_TRY(hipMemcpyAsync(phi_dev + 2 * off[b], bt.phi + 2 * k * N2, 2 * N2 * 8, hipMemcpyDeviceToDevice,
                               c->stream));
    }
  }
  HIP_TRY(hipFreeAsync(stage, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return rc;
}

// Argument checks of the gradient call, and the bytes of
// scratch the call needs (partials, and per-item totals when the caller
// wants only their sum).
int grad_args(rve_ctx* c, int B, int n, const double* a_dev, const double* phi_dev, double h,
              const double* G_dev, double* grad_a_dev, const unsigned char* mask, double a_in,
              double* grad_in_dev, double* grad_in_sum_dev, int scheme, size_t* scratch_bytes) {
  if (!c || B < 1 || !n_supported(n) || !(h > 0.0) || !std::isfinite(h) || !a_dev || !phi_dev || !G_dev ||
      !grad_a_dev)
    return RVE_EINVAL;
  if (scheme != RVE_SCHEME_Q1 && scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  const bool want_in = grad_in_dev || grad_in_sum_dev;
  if (want_in && !mask && !std::isfinite(a_in)) return RVE_EINVAL;
  const size_t P = (size_t)grad_tiles_per_realization(n);
  *scratch_bytes = want_in ? align_up((size_t)B * P * 8) + (grad_in_dev ? 0 : align_up((size_t)B * 8)) : 0;
  return RVE_OK;
}

void grad_launch(rve_ctx* c, int B, int n, const double* a_dev, const double* phi_dev, double h,
                 const double* G_dev, double* grad_a_dev, const unsigned char* mask, double a_in,
                 double* grad_in_dev, double* grad_in_sum_dev, int scheme, char* scratch) {
  const bool want_in = grad_in_dev || grad_in_sum_dev;
  const size_t P = (size_t)grad_tiles_per_realization(n);
  double* part = reinterpret_cast<double*>(scratch);
  double* totals = grad_in_dev ? grad_in_dev
                               : (want_in ? reinterpret_cast<double*>(scratch + align_up((size_t)B * P * 8)) : nullptr);
  launch_grad(B, n, scheme, a_dev, phi_dev, 1.0 / h, G_dev, grad_a_dev, a_in, mask, part, want_in ? 1 : 0,
              c->stream);
  if (want_in) launch_scalar_grad(B, n, part, totals, grad_in_sum_dev, c->stream);
}

int rve_grad(rve_ctx* c, int B, int n, const double* a_dev, const double* phi_dev, double h,
             const double* G_dev, double* grad_a_dev, const unsigned char* incl_mask_dev, double a_in,
             double* grad_in_dev, double* grad_in_sum_dev, int scheme) {
  size_t bytes = 0;
  int rc = grad_args(c, B, n, a_dev, phi_dev, h, G_dev, grad_a_dev, incl_mask_dev, a_in, grad_in_dev,
                     grad_in_sum_dev, scheme, &bytes);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(c->device));
  if (bytes) {
    rc = ensure_ws(c, bytes);
    if (rc) return rc;
  }
  grad_launch(c, B, n, a_dev, phi_dev, h, G_dev, grad_a_dev, incl_mask_dev, a_in, grad_in_dev, grad_in_sum_dev,
              scheme, static_cast<char*>(c->ws));
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_grad_noalloc(rve_ctx* c, int B, int n, const double* a_dev, const double* phi_dev, double h,
                     const double* G_dev, double* grad_a_dev, const unsigned char* incl_mask_dev, double a_in,
                     double* grad_in_dev, double* grad_in_sum_dev, int scheme) {
  size_t bytes = 0;
  const int rc = grad_args(c, B, n, a_dev, phi_dev, h, G_dev, grad_a_dev, incl_mask_dev, a_in, grad_in_dev,
                           grad_in_sum_dev, scheme, &bytes);
  if (rc) return rc;
  if (bytes > kNoAllocScratchBytes) {
    fprintf(stderr, "librve: rve_grad_noalloc needs %zu bytes of scratch for B = %d, n = %d; its fixed "
            "scratch holds %zu (use rve_grad)\n", bytes, B, n, kNoAllocScratchBytes);
    return RVE_EINVAL;
  }
  HIP_TRY(hipSetDevice(c->device));
  // every scratch byte read is written first by the same call (tile partials,
  // then per-item totals), so nothing needs clearing
  grad_launch(c, B, n, a_dev, phi_dev, h, G_dev, grad_a_dev, incl_mask_dev, a_in, grad_in_dev, grad_in_sum_dev,
              scheme, c->noalloc_scratch);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_field_from_mask(rve_ctx* c, int B, long long cells, const unsigned char* mask_dev, const double* a_in_dev,
                        double a_bg, double* a_dev) {
  if (!c || B < 1 || B > 65535 || cells < 1 || !mask_dev || !a_in_dev || !a_dev) return RVE_EINVAL;
  if (!(a_bg > 0.0) || !std::isfinite(a_bg)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_field_from_mask(B, cells, mask_dev, a_in_dev, a_bg, a_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_stats(rve_ctx* c, int N, double L, const double* ahom_dev, double* out_dev) {
  if (!c || N < 2 || !(L > 0.0) || !ahom_dev || !out_dev) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_stats(N, L, ahom_dev, out_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_apply_operator(rve_ctx* c, int B, int n, const double* a_dev, const double* u_dev, double* out_dev,
                       int scheme) {
  if (!c || B < 1 || !n_supported(n) || !a_dev || !u_dev || !out_dev || u_dev == out_dev) return RVE_EINVAL;
  if (scheme != RVE_SCHEME_Q1 && scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_apply_stencil(B, n, scheme, a_dev, u_dev, out_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_apply_precond(rve_ctx* c, int B, int n, const double* a_dev, const double* r_dev, double* z_dev,
                      int prec, int scheme) {
  if (!c || B < 1 || !n_supported(n) || !a_dev || !r_dev || !z_dev || r_dev == z_dev) return RVE_EINVAL;
  if (prec < RVE_FP64 || prec > RVE_MIX_FP16) return RVE_EINVAL;
  if (scheme != RVE_SCHEME_Q1 && scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  Work w;
  const Layout L = plan(B, n, prec, 0, scheme, 2, &w);
  int rc = ensure_ws(c, L.total);
  if (rc) return rc;
  bind(static_cast<char*>(c->ws), L, &w);
  w.a = a_dev;
  Tables* tb = nullptr;
  rc = build_tables(c, n, &tb);
  if (rc) return rc;
  // a0 of each realization, exactly as the solver derives it
  launch_init_state(w, c->stream);
  launch_rhs(w, c->stream);
  launch_scalar_init(w, c->stream);
  const GemmTables gt = gemm_tables(tb, prec, scheme);
  w.r = const_cast<double*>(r_dev);
  w.sys = nullptr;
  if (w.mixed) launch_round_lo(w, c->stream);
  const int gp = gemm_prec(prec);
  if (c->force_gemm >= 0 && gemm_variant_valid(n, gp, c->force_gemm)) {
    w.gemm_variant = c->force_gemm;
    w.P_gemm = gemm_tiles_per_system(n, gp, w.gemm_variant);
  }
  // the solver keeps z in FP32 in the mixed modes; the caller wants FP64
  void* z_solver = w.z;
  w.z = w.mixed ? z_solver : (void*)z_dev;
  launch_precond(w, gp, gt, c->stream);
  if (w.mixed) launch_widen(static_cast<const float*>(w.z), z_dev, (long long)w.S * w.N2, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_dos_moments(rve_ctx* c, int B, int n, int scheme, const double* a_dev, int nv, const double* v_dev,
                    double lmax, int K, double* mu_dev) {
  if (!c || B < 1 || !n_supported(n) || !a_dev || !v_dev || !mu_dev || nv < 2 || nv % 2 || K < 1 || K > 1000000)
    return RVE_EINVAL;
  if (scheme != RVE_SCHEME_Q1 && scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  if (!(lmax > 0.0) || !std::isfinite(lmax)) return RVE_EINVAL;
  if ((long long)B * nv > 65535) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  const long long N2 = (long long)n * n, S = (long long)B * nv;
  const size_t vec = align_up((size_t)(S * N2) * 8);
  const size_t part = align_up((size_t)S * dos_vec_tiles(N2) * 2 * 8);
  int rc = ensure_ws(c, 3 * vec + part);
  if (rc) return rc;
  char* ws = static_cast<char*>(c->ws);
  double* W = reinterpret_cast<double*>(ws);
  double* Wp = reinterpret_cast<double*>(ws + vec);
  double* AW = reinterpret_cast<double*>(ws + 2 * vec);
  double* P = reinterpret_cast<double*>(ws + 3 * vec);
  // probes [B][nv][n][n] -> pair-major [nv/2][B][2][n][n]
  for (int b = 0; b < B; ++b)
    for (int v = 0; v < nv; ++v)
      HIP_TRY(hipMemcpyAsync(W + (((long long)(v / 2) * B + b) * 2 + (v % 2)) * N2,
                             v_dev + ((long long)b * nv + v) * N2, N2 * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(Wp, 0, (size_t)(S * N2) * 8, c->stream));
  launch_dos_moments(B, n, scheme, a_dev, nv, W, Wp, AW, lmax, K, P, mu_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_dos_plan(rve_ctx* c, int B, int n, int scheme, const double* a_dev, double eta, double* lmax_host,
                 int* K_host) {
  if (!c || B < 1 || !n_supported(n) || !a_dev || !lmax_host || !K_host) return RVE_EINVAL;
  if (scheme != RVE_SCHEME_Q1 && scheme != RVE_SCHEME_FD5) return RVE_EINVAL;
  if (!(eta > 0.0) || !std::isfinite(eta)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  int rc = ensure_one_out(c);
  if (rc) return rc;
  const long long total = (long long)B * n * n;
  rc = ensure_ws(c, align_up((size_t)field_max_blocks(total) * 2 * 8));
  if (rc) return rc;
  launch_field_max(a_dev, total, static_cast<double*>(c->ws), c->one_out, c->stream);
  double host[2];
  HIP_TRY(hipMemcpyAsync(host, c->one_out, sizeof host, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (host[1] != 0.0 || !(host[0] > 0.0) || !std::isfinite(host[0])) return RVE_EINVAL;
  // Gershgorin: a row of the Q1 stiffness has diagonal (2/3) sum of its four
  // cells and off-diagonal magnitudes summing to the same, so every
  // eigenvalue is at most (4/3) 4 max a; the five-point operator's rows give
  // 2 * 4 max a
  const double lmax = (scheme == RVE_SCHEME_FD5 ? 8.0 : 16.0 / 3.0) * host[0];
  // enough moments to resolve the width eta: about 6 per eta over [0, lmax]
  const double k = std::min(20000.0, std::max(64.0, 6.0 * lmax / eta));
  *lmax_host = lmax;
  *K_host = (int)k;
  return RVE_OK;
}

int rve_dos_probes(rve_ctx* c, int B, int nv, int n, uint64_t seed, double* v_dev) {
  if (!c || B < 1 || nv < 1 || !n_supported(n) || !v_dev) return RVE_EINVAL;
  const long long total = (long long)B * nv * n * n;
  if (total / nv / B != (long long)n * n || (total + 127) / 128 / kBlock >= (1LL << 31)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_probes(total, (unsigned long long)seed, v_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_sample_fixed_count(rve_ctx* c, int B, int n, int side, uint64_t seed, int64_t first, int K, double a_in,
                           double a_bg, double* a_dev) {
  if (!c || B < 1 || B > 65535 || !n_supported(n) || !sample_side_valid(n, side) || first < 0 || K < 0 ||
      (long long)B * K >= (1LL << 31) * kBlock || !a_dev)
    return RVE_EINVAL;
  if (!(a_in > 0.0) || !(a_bg > 0.0) || !std::isfinite(a_in) || !std::isfinite(a_bg)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  const int rc = ensure_ws(c, align_up((size_t)B * n * n));
  if (rc) return rc;
  launch_sample_fixed(B, n, side, (unsigned long long)seed, (long long)first, K, a_in, a_bg,
                      static_cast<uint8_t*>(c->ws), a_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

uint32_t rve_occupancy_threshold(double mu) {
  if (!(mu > 0.0)) return 0u;
  if (!std::isfinite(mu)) return 0xFFFFFFFFu;
  const double t = std::nearbyint(4294967296.0 * -std::expm1(-mu));
  return t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
}

int rve_dos_eval(rve_ctx* c, int B, int nv, int K, const double* mu_dev, double lmax, double eta, int Q, int nt,
                 const double* t_dev, double* phi_dev) {
  if (Q <= 0 && K >= 1 && K <= 2500000) Q = 4 * K;   // default rule
  if (!c || B < 1 || B > 65535 || nv < 1 || K < 1 || Q < K || Q > 10000000 || nt < 1 || !mu_dev || !t_dev ||
      !phi_dev)
    return RVE_EINVAL;
  if (!(lmax > 0.0) || !std::isfinite(lmax) || !(eta > 0.0) || !std::isfinite(eta)) return RVE_EINVAL;
  if ((nt + kBlock - 1) / kBlock > 2147483647 || (Q + kBlock - 1) / kBlock > 2147483647) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  int rc = ensure_ws(c, align_up((size_t)B * Q * 8));
  if (rc) return rc;
  launch_dos_eval(B, nv, K, mu_dev, lmax, eta, Q, nt, t_dev, static_cast<double*>(c->ws), phi_dev, c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_sample_lattice(rve_ctx* c, int B, int n, int side, uint64_t seed, int64_t first, uint32_t occ_threshold,
                       double a_in, double a_bg, double* a_dev) {
  if (!c || B < 1 || B > 65535 || !n_supported(n) || !sample_side_valid(n, side) || first < 0 || !a_dev)
    return RVE_EINVAL;
  if (!(a_in > 0.0) || !(a_bg > 0.0) || !std::isfinite(a_in) || !std::isfinite(a_bg)) return RVE_EINVAL;
  HIP_TRY(hipSetDevice(c->device));
  launch_sample_lattice(B, n, side, (unsigned long long)seed, (long long)first, occ_threshold, a_in, a_bg, a_dev,
                        c->stream);
  HIP_TRY(hipGetLastError());
  return RVE_OK;
}

int rve_force_variants(rve_ctx* c, int stencil_choice, int gemm_variant, int update_choice) {
  if (!c || stencil_choice < -1 || gemm_variant < -1 || gemm_variant > 7 || update_choice < -1) return RVE_EINVAL;
  // well-formed shape codes (every shape tiles the largest supported grid)
  if (stencil_choice >= 0 && !stencil_choice_valid(kMaxN, stencil_choice)) return RVE_EINVAL;
  if (update_choice >= 0 && !stencil_choice_valid(kMaxN, update_choice)) return RVE_EINVAL;
  c->force_stencil = stencil_choice;
  c->force_gemm = gemm_variant;
  c->force_update = update_choice >= 0 ? update_choice : stencil_choice;
  return RVE_OK;
}

int rve_set_direction_update(rve_ctx* c, int mode) {
  if (!c || (mode != 0 && mode != 1)) return RVE_EINVAL;
  c->direction_update = mode;
  return RVE_OK;
}

int rve_set_direction_bf16(rve_ctx* c, int mode) {
  if (!c || (mode != 0 && mode != 1)) return RVE_EINVAL;
  c->direction_bf16 = mode;
  return RVE_OK;
}

int rve_set_small_solver(rve_ctx* c, int mode) {
  if (!c || (mode != 0 && mode != 1)) return RVE_EINVAL;
  c->small_solver = mode;
  return RVE_OK;
}

int rve_set_graphs(rve_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 1) return RVE_EINVAL;
  c->graphs = mode;
  return RVE_OK;
}

int rve_set_autotune(rve_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 1) return RVE_EINVAL;
  c->autotune = mode;
  return RVE_OK;
}

int rve_get_tuned(rve_ctx* c, int kind, int n, int prec, int B, int* choice) {
  if (!c || !choice || kind < 0 || kind > 5 || B < 1) return RVE_EINVAL;
  auto it = c->tune.find(TuneKey(kind, n, prec, batch_bucket(B)));
  if (it == c->tune.end()) {
    *choice = -1;
    return RVE_NOT_CONVERGED;
  }
  *choice = it->second;
  return RVE_OK;
}

int rve_set_timing(rve_ctx* c, int enable) {
  if (!c) return RVE_EINVAL;
  c->timing = enable != 0;
  for (int k = 0; k < kTimedClasses; ++k) {
    c->timer.ms[k] = 0;
    c->timer.count[k] = 0;
  }
  c->timer.pairs.clear();
  c->timer.used = 0;
  return RVE_OK;
}

int rve_last_timing(rve_ctx* c, double* out_ms, long long* out_counts) {
  if (!c || !out_ms || !out_counts) return RVE_EINVAL;
  for (int k = 0; k < kTimedClasses; ++k) {
    out_ms[k] = c->timer.ms[k];
    out_counts[k] = c->timer.count[k];
  }
  return RVE_OK;
}

}  // extern "C"
