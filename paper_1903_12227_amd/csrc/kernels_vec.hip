// Stencil-shaped and elementwise kernels of the RVE corrector path.
//
// Grid units (h = 1). Cell (i, j) spans nodes i..i+1 (x1) and j..j+1 (x2),
// mod n; arrays are [i][j] with x2 contiguous. A realization b owns the two
// corrector systems s = 2b (direction e1) and s = 2b + 1 (direction e2).
//
// Tile-shaped kernels (RHS, operator apply, A_hom, gradient) use one
// 256-thread workgroup per 64 x 64 tile of a realization: lane = column, the
// four waves take 16-row strips and slide a register window down their
// strip, so every value is loaded from HBM about once and the +-1 column
// neighbours come from the same cache lines. All reductions are written as
// per-workgroup partials and finished in a fixed order (deterministic, no
// floating-point atomics).
#include <type_traits>

#include "launch.h"
#include "stencil2d.h"

namespace rve {

namespace {


// Four consecutive elements of a vector in its storage type, widened to or
// rounded from FP64 (the element index is a multiple of 4).
template <class T> struct V4;
template <> struct V4<double> {
  __device__ static void load(const double* p, double (&v)[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  __device__ static void store(double* p, const double (&v)[4]) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  }
};
template <> struct V4<float> {
  __device__ static void load(const float* p, double (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  __device__ static void store(float* p, const double (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
};
template <> struct V4<__bf16> {
  __device__ static void store(__bf16* p, const double (&v)[4]) {
    struct alignas(8) Pack { __bf16 e[4]; } pk;
#pragma unroll
    for (int k = 0; k < 4; ++k) pk.e[k] = (__bf16)(float)v[k];
    *reinterpret_cast<Pack*>(p) = pk;
  }
};
template <> struct V4<_Float16> {
  __device__ static void store(_Float16* p, const double (&v)[4]) {
    struct alignas(8) Pack { _Float16 e[4]; } pk;
#pragma unroll
    for (int k = 0; k < 4; ++k) pk.e[k] = (_Float16)(float)v[k];
    *reinterpret_cast<Pack*>(p) = pk;
  }
};

// The GEMM-precision residual copy: FP16 copies are written times the
// system's scale, the others as they are (their scale is 1).
template <class LoT> constexpr bool kScaledLo = std::is_same<LoT, _Float16>::value;
template <class LoT>
__device__ inline double lo_scale_of(const SysState& S) {
  if constexpr (kScaledLo<LoT>) return S.lo_next;
  return 1.0;
}
template <class LoT>
__device__ inline void store_lo(LoT* p, const double (&v)[4], double sc) {
  if constexpr (kScaledLo<LoT>) {
    double w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = v[k] * sc;
    V4<LoT>::store(p, w);
  } else {
    V4<LoT>::store(p, v);
  }
}

// Coefficients as the operator kernels read them: FP64 values (AT = CT), or
// one byte per cell for a two-valued field (AT = uint8_t: 1 on cells with the
// realization's largest value, 0 on those with its smallest), decoded
// exactly to those two values.
template <class CT, class AT>
struct CoefDec {
  CT lo = (CT)0, hi = (CT)0;
  __device__ CoefDec(const RealState* real, int b) {
    if constexpr (std::is_same<AT, uint8_t>::value) {
      lo = (CT)real[b].a_min;
      hi = (CT)real[b].a_max;
      // the larger value is held in vector registers (the empty statement
      // only pins it there), so a decode is one select per 32-bit half that
      // reads the smaller value from scalar registers, with no copies
      asm("" : "+v"(hi));
    }
  }
  __device__ CT operator()(AT v) const {
    if constexpr (std::is_same<AT, uint8_t>::value) return v ? hi : lo;
    else return (CT)v;
  }
};

// code[b][e] = 1 where a = max a of realization b, 0 where a = min a; a cell
// with any other value sets bit 0 of *not_two_valued (one atomic per
// workgroup), a realization whose contrast max a / min a exceeds
// kDir16MaxContrast bit 1.
__global__ void __launch_bounds__(kBlock) k_encode_two_valued(const double* __restrict__ a,
                                                               const RealState* __restrict__ real, long long N2,
                                                               uint8_t* __restrict__ code, int* not_two_valued) {
  const int b = blockIdx.y;
  const double lo = real[b].a_min, hi = real[b].a_max;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !(hi <= kDir16MaxContrast * lo)) atomicOr(not_two_valued, 2);
  const long long off = (long long)b * N2;
  const long long stride = (long long)gridDim.x * kBlock * 4;
  int bad = 0;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < N2; i += stride) {
    double v[4];
    V4<double>::load(a + off + i, v);
    uchar4 c;
    c.x = v[0] == hi; c.y = v[1] == hi; c.z = v[2] == hi; c.w = v[3] == hi;
#pragma unroll
    for (int k = 0; k < 4; ++k) bad |= !(v[k] == hi || v[k] == lo);
    *reinterpret_cast<uchar4*>(code + off + i) = c;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(not_two_valued, 1);
}

__global__ void __launch_bounds__(kBlock) k_init_state(SysState* sys, RealState* real, int S, int B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int stride = gridDim.x * kBlock;
  for (int i = t; i < S; i += stride) {
    SysState z{};
    z.lo_scale = 1.0;
    z.lo_next = 1.0;
    sys[i] = z;
  }
  for (int i = t; i < B; i += stride) real[i] = RealState{};
}

// Iteration counter and per-iteration counts of the systems still iterating,
// shared by every batch of one solve.
__global__ void __launch_bounds__(kBlock) k_ctl_reset(int* kiter, int* count, int count_len) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int stride = gridDim.x * kBlock;
  if (t == 0) {
    kiter[0] = 0;
    kiter[16] = 0;   // the not-two-valued flag of the batch encoding (byte 64)
  }
  for (int i = t; i < count_len; i += stride) count[i] = 0;
}


// Galerkin right-hand sides f_i = -int a d(psi)/dx_i, integrated exactly per
// cell (eqn. FEM_discr_RHS): with a11 = a[p][q], a10 = a[p][q-1],
// a01 = a[p-1][q], a00 = a[p-1][q-1],
//   f_1[p][q] = (a11 + a10 - a01 - a00)/2,  f_2[p][q] = (a11 + a01 - a10 - a00)/2.
// Also gathers per-tile sum/min/max of a and a count of invalid cells.
__global__ void __launch_bounds__(kBlock) k_rhs(const double* __restrict__ a, double* __restrict__ r,
                                                 int n, double* __restrict__ part) {
  __shared__ double sh[4 * 6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.z;
  const long long N2 = (long long)n * n;
  const int col = blockIdx.x * kTile + lane, cm = wrap_dec(col, n);
  const int row0 = blockIdx.y * kTile + w * kStrip;
  const double* A = a + (long long)b * N2;
  double* F1 = r + (2LL * b) * N2;
  double* F2 = F1 + N2;
  int rr = wrap_dec(row0, n);
  double a00 = A[(long long)rr * n + cm], a01 = A[(long long)rr * n + col];
  double s[3] = {0.0, 0.0, 0.0};
  double amin = 1.0e308, amax = -1.0e308;
  int bad = 0;
  for (int j = 0; j < kStrip; ++j) {
    const int row = row0 + j;
    const double a10 = A[(long long)row * n + cm], a11 = A[(long long)row * n + col];
    const double f1 = 0.5 * ((a11 + a10) - (a01 + a00));
    const double f2 = 0.5 * ((a11 + a01) - (a10 + a00));
    F1[(long long)row * n + col] = f1;
    F2[(long long)row * n + col] = f2;
    s[0] += f1;
    s[1] += f2;
    s[2] += a11;
    amin = fmin(amin, a11);
    amax = fmax(amax, a11);
    bad += !(a11 > 0.0);   // also catches NaN
    a00 = a10;
    a01 = a11;
  }
  const double vmin = wave_min(amin), vmax = wave_max(amax);
  double badd = (double)bad;
  double v[4] = {s[0], s[1], s[2], badd};
  block_sum<4>(v, sh);
  __shared__ double mm[8];
  if (lane == 0) { mm[w] = vmin; mm[4 + w] = vmax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int P = gridDim.x * gridDim.y;
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    double* o = part + ((long long)b * P + tile) * kMiscNV;
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = fmin(fmin(mm[0], mm[1]), fmin(mm[2], mm[3]));
    o[4] = fmax(fmax(mm[4], mm[5]), fmax(mm[6], mm[7]));
    o[5] = v[3];
  }
}

// Per realization: finish the RHS partials (one wave per realization).
__global__ void k_scalar_init(SysState* sys, RealState* real, const double* __restrict__ part, int P,
                              int n, int scaled) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double s1 = 0, s2 = 0, sa = 0, bad = 0, mn = 1.0e308, mx = -1.0e308;
  for (int t = lane; t < P; t += kWave) {
    const double* o = part + ((long long)b * P + t) * kMiscNV;
    s1 += o[0];
    s2 += o[1];
    sa += o[2];
    mn = fmin(mn, o[3]);
    mx = fmax(mx, o[4]);
    bad += o[5];
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  sa = wave_sum(sa);
  bad = wave_sum(bad);
  mn = wave_min(mn);
  mx = wave_max(mx);
  if (lane == 0) {
    const double N2 = (double)n * (double)n;
    RealState rs;
    rs.a_sum = sa;
    rs.a_min = mn;
    rs.a_max = mx;
    rs.inv_a0 = 2.0 / (mx + mn);
    rs.bad = (int)bad;
    rs.pad = 0;
    real[b] = rs;
    const int valid = (bad == 0.0) && isfinite(sa);
    sys[2 * b].mean_f = s1 / N2;
    sys[2 * b + 1].mean_f = s2 / N2;
    sys[2 * b].valid = valid;
    sys[2 * b + 1].valid = valid;
    // scaled copies: |f - mean f| <= 2 (a_max - a_min), so the first copy
    // stays within +-1/2
    if (scaled && mx > mn) {
      sys[2 * b].lo_next = 0.25 / (mx - mn);
      sys[2 * b + 1].lo_next = 0.25 / (mx - mn);
    }
  }
}

// r <- r - mean(f), x <- 0 (the initial iterate), and in mixed modes the
// GEMM-precision copy of r; partial sums of r.r.
template <class LoT, bool LO>
__global__ void __launch_bounds__(kBlock) k_meansub(double* __restrict__ r, double* __restrict__ x,
                                                     LoT* __restrict__ rlo, const SysState* sys, long long N2,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  const int s = blockIdx.y;
  const double m = sys[s].mean_f, sc = lo_scale_of<LoT>(sys[s]);
  const long long off = (long long)s * N2;
  double acc[1] = {0.0};
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < N2; i += stride) {
    double v[4];
    V4<double>::load(r + off + i, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] -= m;
      acc[0] += v[k] * v[k];
    }
    V4<double>::store(r + off + i, v);
    V4<double>::store(x + off + i, zero);
    if constexpr (LO) store_lo<LoT>(rlo + off + i, v, sc);
  }
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) part[(long long)s * gridDim.x + blockIdx.x] = acc[0];
}

__global__ void k_scalar_fnorm(SysState* sys, const double* __restrict__ part, int P, int scaled,
                               double sqrt_n) {
  const int s = blockIdx.x, lane = threadIdx.x;
  double v = 0;
  for (int t = lane; t < P; t += kWave) v += part[(long long)s * P + t];
  v = wave_sum(v);
  if (lane == 0) {
    SysState& S = sys[s];
    S.fnorm = sqrt(v);
    S.iters = 0;
    S.relres = 0.0;
    // the copy just written carries lo_next; the next one is scaled to the
    // norm of this residual
    S.lo_scale = S.lo_next;
    if (scaled && S.fnorm > 0.0 && isfinite(S.fnorm)) S.lo_next = 0.25 * sqrt_n / S.fnorm;
    if (!S.valid) {
      S.active = 0;
      S.status = -1;   // RVE_EINVAL
    } else if (!(S.fnorm > 0.0)) {
      S.active = 0;    // f = 0 (e.g. a constant field): phi = 0, done
      S.status = 0;
    } else {
      S.active = 1;
      S.status = 0;
    }
  }
}

// q = A p for both systems of a realization (9-point Q1 stencil, or the
// five-point scheme; formulas in stencil2d.h), with partial sums of p.q.

// V consecutive elements of a row, converted to / from the register type S.
template <class T, int V> struct VecIO;
template <int V> struct VecIO<double, V> {
  template <class S> __device__ static void load(const double* p, S* v) {
    if constexpr (V == 1) {
      v[0] = (S)p[0];
    } else {
#pragma unroll
      for (int k = 0; k < V; k += 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + k);
        v[k] = (S)t.x; v[k + 1] = (S)t.y;
      }
    }
  }
  template <class S> __device__ static void store(double* p, const S* v) {
    if constexpr (V == 1) {
      p[0] = (double)v[0];
    } else {
#pragma unroll
      for (int k = 0; k < V; k += 2)
        *reinterpret_cast<double2*>(p + k) = make_double2((double)v[k], (double)v[k + 1]);
    }
  }
};
template <int V> struct VecIO<float, V> {
  template <class S> __device__ static void load(const float* p, S* v) {
    if constexpr (V == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      v[0] = (S)t.x; v[1] = (S)t.y; v[2] = (S)t.z; v[3] = (S)t.w;
    } else if constexpr (V == 2) {
      const float2 t = *reinterpret_cast<const float2*>(p);
      v[0] = (S)t.x; v[1] = (S)t.y;
    } else {
      v[0] = (S)p[0];
    }
  }
  template <class S> __device__ static void store(float* p, const S* v) {
    if constexpr (V == 4) {
      *reinterpret_cast<float4*>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    } else if constexpr (V == 2) {
      *reinterpret_cast<float2*>(p) = make_float2((float)v[0], (float)v[1]);
    } else {
      p[0] = (float)v[0];
    }
  }
};

// Streaming accesses (read once, written once per iteration, no reuse
// within a launch): non-temporal, so they do not displace reused lines in L2.
template <class T, int V>
__device__ inline void load_nt(const T* p, T* v) {
  constexpr int C = (int)(16 / sizeof(T)) < V ? (int)(16 / sizeof(T)) : V;   // elements per load
  typedef T vec_t __attribute__((ext_vector_type(C)));
#pragma unroll
  for (int k = 0; k < V; k += C) {
    if constexpr (C == 1) {
      v[k] = __builtin_nontemporal_load(p + k);
    } else {
      const vec_t t = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(p + k));
#pragma unroll
      for (int e = 0; e < C; ++e) v[k + e] = t[e];
    }
  }
}
template <class T, int V>
__device__ inline void store_nt(T* p, const T* v) {
#pragma unroll
  for (int k = 0; k < V; ++k) __builtin_nontemporal_store(v[k], p + k);
}

// Operator apply over V consecutive columns per lane for both systems of a
// realization. A workgroup covers 64V columns x 4H rows; each of its four
// waves slides a three-row register window down an H-row strip, so every
// value is loaded about once (plus two halo rows per strip) and the +-1
// columns come from the cache lines just loaded. The loads of a row are
// issued D - 1 rows ahead of their use (a ring of D row buffers), so each
// wave keeps D rows of loads in flight (D = 1: each row is loaded just
// before it is used).
// FUSED: the operand is the new search direction
// p_k = z_k + beta_{k-1} p_{k-1} (p_0 = z_0), formed on the fly for the V
// nodes and their neighbours; p_k goes to a ring slot other than p_{k-1}'s
// (neighbouring workgroups still read p_{k-1} at tile edges), and q = A p_k
// is written with partial sums of p_k.q (active systems only). Not FUSED:
// q = A u for a caller's u (the plain operator apply).
//
// One-dimensional grid of gx * gy * B workgroups. The hardware hands
// consecutive workgroup ids to the eight XCDs in turn; the id is remapped so
// that each XCD receives a contiguous run of tiles (all tiles of a few
// realizations, neighbours next to each other in time), and halo lines
// fetched by one tile are found in that XCD's L2 by its neighbours.
//
// FUSED: iteration k is read from *kiter; p_k goes to ring slot k mod m and
// p_{k-1} comes from slot (k - 1) mod m (slots slot_stride elements apart).
// probe = 1 (autotuner timing at k = 0 only) reads p_{k-1} as a later
// iteration would; its outputs are rewritten by the real iteration 0.
// Not FUSED: the operand is p_in.
// SCH selects the operator: 0 the consistent Q1 nine-point stencil, 1 the
// lumped five-point one. wq = 0 (FUSED only) skips the store of q: the
// residual update then recomputes it (k_update_r_st).
// CT is the arithmetic type of the apply (coefficients a, operand, q = A p):
// FP64, or FP32 with p rounded to FP32 before use; the p.q partial sums are
// FP64 either way (the product of two FP32 values is exact in FP64).
// PDIR (FUSED only): the direction p_k is already in ring slot k mod m (the
// last transform formed it); the apply reads it alone and stores nothing but
// the p.q partials (and q with wq).
template <bool FUSED, class PT, class ZT, int V, int D, class CT, int SCH, class AT = CT, bool PDIR = false>
__global__ void __launch_bounds__(kBlock) k_stencil_v(const AT* __restrict__ a, const PT* p_in, PT* ring,
                                                       long long slot_stride, int m, const int* kiter,
                                                       const ZT* __restrict__ z, CT* __restrict__ q, int n,
                                                       int H, const SysState* sys, double* __restrict__ part,
                                                       int probe, int wq, const RealState* real) {
  static_assert(D == 1 || D == 2 || D == 4, "prefetch depth");
  static_assert(FUSED || !PDIR, "PDIR is a mode of the fused apply");
  constexpr bool FORM = FUSED && !PDIR;   // p_k formed here from z_k and p_{k-1}
  __shared__ double sh[4 * 2];
  int first = 0;
  const PT* __restrict__ p_old = p_in;
  PT* __restrict__ p_new = nullptr;
  if constexpr (PDIR) {
    p_old = ring + (long long)(kiter[0] % m) * slot_stride;
  } else if constexpr (FUSED) {
    const int k = kiter[0];
    first = k == 0 && !probe;   // a probe does the work of a later iteration
    p_new = ring + (long long)(k % m) * slot_stride;
    p_old = ring + (long long)((k + m - 1) % m) * slot_stride;
  }
  const int gx = n / (kWave * V), gy = n / (4 * H);
  const unsigned T = gridDim.x, L = blockIdx.x;
  const unsigned t = (T & 7u) ? L : (L & 7u) * (T >> 3) + (L >> 3);
  const int bx = (int)(t % (unsigned)gx);
  const int by = (int)((t / (unsigned)gx) % (unsigned)gy);
  const int b = (int)(t / (unsigned)(gx * gy));
  const int s0 = 2 * b, s1 = s0 + 1;
  const int act0 = FUSED ? sys[s0].active : 1, act1 = FUSED ? sys[s1].active : 1;
  if (!act0 && !act1) return;   // uniform over the workgroup
  const double be[2] = {FORM && !first ? sys[s0].beta : 0.0, FORM && !first ? sys[s1].beta : 0.0};
  const int act[2] = {act0, act1};
  const int lane = threadIdx.x & 63, w = wave_id();
  const long long N2 = (long long)n * n;
  const int c0 = (bx * kWave + lane) * V;
  const int cl = wrap_dec(c0, n), cr = c0 + V == n ? 0 : c0 + V;
  const int row0 = by * 4 * H + w * H;
  const CoefDec<CT, AT> dec(real, b);
  const bool need_p = !FORM || !first;
  // the n x n blocks this workgroup reads and writes; rows are wave-uniform,
  // and the byte offsets of columns c0, c0-1 and c0+V are fixed per lane
  const Plane<AT> Ap(a + (long long)b * N2, n);
  const Plane<PT> Pold[2] = {Plane<PT>(p_old + (long long)s0 * N2, n), Plane<PT>(p_old + (long long)s1 * N2, n)};
  const Plane<PT> Pnew[2] = {Plane<PT>(p_new + (long long)s0 * N2, n), Plane<PT>(p_new + (long long)s1 * N2, n)};
  const Plane<ZT> Zs[2] = {Plane<ZT>(z + (long long)s0 * N2, n), Plane<ZT>(z + (long long)s1 * N2, n)};
  const Plane<CT> Qs[2] = {Plane<CT>(q + (long long)s0 * N2, n), Plane<CT>(q + (long long)s1 * N2, n)};
  const unsigned pc0 = c0 * sizeof(PT), pcl = cl * sizeof(PT), pcr = cr * sizeof(PT);
  const unsigned zc0 = c0 * sizeof(ZT), zcl = cl * sizeof(ZT), zcr = cr * sizeof(ZT);
  const unsigned ac0 = c0 * sizeof(AT), acl = cl * sizeof(AT);
  const unsigned qc0 = c0 * sizeof(CT);

  // raw operand row ro (V + 2 values per system: column c0-1, c0..c0+V-1,
  // c0+V) and coefficient row ra (V + 1 values: c0-1 .. c0+V-1). The operand
  // columns c0 - 1 and c0 + V come from the neighbouring lanes (halo), lanes 0
  // and 63 reading theirs with one load per array (halo_offset): two loads
  // fewer per array and row than loading both neighbour columns
  struct Raw {
    ZT z[2][V + 2];
    PT p[2][V + 2];
    AT a[V + 1];
  };
  const unsigned zch = halo_offset(lane, zcl, zcr), pch = halo_offset(lane, pcl, pcr);
  auto load_raw = [&](Raw& R, int ro, int ra, bool with_a) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if constexpr (FORM) {
        Zs[i].template load<V>(ro, zc0, &R.z[i][1]);
        R.z[i][0] = Zs[i].get(ro, zch);
      }
      if (need_p) {
        Pold[i].template load<V>(ro, pc0, &R.p[i][1]);
        R.p[i][0] = Pold[i].get(ro, pch);
      }
    }
    if (with_a) {
      R.a[0] = Ap.get(ra, acl);
      Ap.template load<V>(ra, ac0, &R.a[1]);
    }
  };
  // the neighbour columns of a loaded row (the halo sits in column 0)
  auto halo = [&](Raw& R) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if constexpr (FORM) {
        const ZT h = R.z[i][0];
        R.z[i][0] = shift_in<kHaloBelow>(h, R.z[i][V]);
        R.z[i][V + 1] = shift_in<kHaloAbove>(h, R.z[i][1]);
      }
      if (need_p) {
        const PT h = R.p[i][0];
        R.p[i][0] = shift_in<kHaloBelow>(h, R.p[i][V]);
        R.p[i][V + 1] = shift_in<kHaloAbove>(h, R.p[i][1]);
      }
    }
  };
  // operand values of system i from a raw row
  auto cook = [&](const Raw& R, int i, CT* u) {
    if constexpr (FORM) {
      if (first) {
#pragma unroll
        for (int k = 0; k < V + 2; ++k) u[k] = (CT)(PT)R.z[i][k];
      } else {
        // p_k is rounded to its storage type (and to CT) before it is used,
        // so q = A p_k, p_k.q and the later x += alpha p_k all see the same
        // direction and the recursive residual follows f - A x
#pragma unroll
        for (int k = 0; k < V + 2; ++k) u[k] = (CT)(PT)fma(be[i], (double)R.p[i][k], (double)R.z[i][k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < V + 2; ++k) u[k] = (CT)R.p[i][k];
    }
  };

  const int rm = wrap_dec(row0, n);
  CT um[2][V + 2], uc[2][V + 2], am[V + 1];
  Raw R[D];
  {
    Raw Ra, Rb;
    load_raw(Ra, rm, rm, true);
    load_raw(Rb, row0, 0, false);
    // the rows of the first D - 1 steps go in flight at once
#pragma unroll
    for (int u = 0; u + 1 < D; ++u) load_raw(R[u], wrap_inc(row0 + u, n), row0 + u, true);
    halo(Ra);
    halo(Rb);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      cook(Ra, i, um[i]);
      cook(Rb, i, uc[i]);
    }
#pragma unroll
    for (int k = 0; k < V + 1; ++k) am[k] = dec(Ra.a[k]);   // a[row-1][c0-1 .. c0+V-1]
  }

  double d[2] = {0.0, 0.0};
  // node row `row`: `use` holds operand row row+1 and coefficient row `row`
  // (with D = 1 it receives them here); `fill` (the buffer of the step
  // before) receives those of step j + D - 1. Past the strip's end that step
  // does not exist and the strip's last rows are loaded again (cache hits,
  // never used): every pass of the loop then issues the same loads, so the
  // waits for a row's data count exactly the loads issued after it instead
  // of draining all of them.
  auto step = [&](int j, Raw& use, Raw& fill) {
    const int row = row0 + j;
    {
      const int rc = row0 + min(j + D - 1, H - 1);   // < n: the strip lies inside the grid
      load_raw(fill, wrap_inc(rc, n), rc, true);
    }
    halo(use);
    CT up[2][V + 2];
#pragma unroll
    for (int i = 0; i < 2; ++i) cook(use, i, up[i]);
    CT ac[V + 1];
#pragma unroll
    for (int k = 0; k < V + 1; ++k) ac[k] = dec(use.a[k]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      CT qv[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const CT sm[3] = {um[i][k], um[i][k + 1], um[i][k + 2]};
        const CT sc[3] = {uc[i][k], uc[i][k + 1], uc[i][k + 2]};
        const CT sp[3] = {up[i][k], up[i][k + 1], up[i][k + 2]};
        if constexpr (SCH == 1)
          qv[k] = fd5_apply<CT>(am[k], am[k + 1], ac[k], ac[k + 1], sm, sc, sp);
        else
          qv[k] = q1_apply<CT>(am[k], am[k + 1], ac[k], ac[k + 1], sm, sc, sp);
      }
      if (act[i]) {
        if (wq) Qs[i].template store<V>(row, qc0, qv);
        if constexpr (FORM) {
          PT pn[V];
#pragma unroll
          for (int k = 0; k < V; ++k) pn[k] = (PT)uc[i][k + 1];
          Pnew[i].template store<V, true>(row, pc0, pn);
        }
      }
#pragma unroll
      for (int k = 0; k < V; ++k) d[i] += (double)uc[i][k + 1] * (double)qv[k];
#pragma unroll
      for (int k = 0; k < V + 2; ++k) {
        um[i][k] = uc[i][k];
        uc[i][k] = up[i][k];
      }
    }
#pragma unroll
    for (int k = 0; k < V + 1; ++k) am[k] = ac[k];
  };
  for (int j = 0; j < H; j += D) {   // H is a multiple of D
#pragma unroll
    for (int u = 0; u < D; ++u) step(j + u, R[u], R[(u + D - 1) % D]);
  }
  if constexpr (FUSED) {
    block_sum<2>(d, sh);
    if (threadIdx.x == 0) {
      const int P = gx * gy;
      const int tile = by * gx + bx;
      part[(long long)s0 * P + tile] = d[0];
      part[(long long)s1 * P + tile] = d[1];
    }
  }
}

// V values of the GEMM-precision residual copy (scaled for FP16).
template <class LoT, int V>
__device__ inline void lo_round_v(LoT* out, const double* v, double sc) {
#pragma unroll
  for (int k = 0; k < V; ++k) out[k] = (LoT)(float)(kScaledLo<LoT> ? v[k] * sc : v[k]);
}

// Residual update in the operator apply's tile shape, with A p_k recomputed:
// r -= alpha_k A p_k for both systems of a realization, r.r partials per tile,
// the GEMM-precision copy of r, and r.z_old partials for the flexible beta.
// The operand is the direction p_k the fused apply stored into ring slot
// k mod m (its values are those the apply used, already rounded to their
// storage type), and A p_k comes from the same coefficient reads and
// arithmetic as there; so the apply need not store q (8 bytes per node and
// system) and this kernel reads p_k (4 bytes with FP32 directions) and the
// coefficients (shared by both systems) instead of q. Tiles, XCD remap and
// the sliding three-row window as in k_stencil_v; each row's r (and z) is
// loaded with the coefficient row, one row ahead with D = 2.
//
// probe = 1 (autotuner timing, before iteration 0): r is rewritten unchanged
// (A p is computed but not applied); the GEMM copy and the partials it writes
// are rewritten by the real iteration 0.
// FLEX: the flexible beta's r.z_old partials (a template parameter, so the
// loop carries no branch around the loads of z).
template <class PT, class ZT, class LoT, bool LO, int V, int D, class CT, int SCH, class AT = CT, bool FLEX = false>
__global__ void __launch_bounds__(kBlock) k_update_r_st(const AT* __restrict__ a, const PT* ring,
                                                         long long slot_stride, int m, const int* kiter,
                                                         const ZT* __restrict__ z, double* __restrict__ r,
                                                         LoT* __restrict__ rlo, int n, int H, const SysState* sys,
                                                         double* __restrict__ part_rr,
                                                         double* __restrict__ part_rzo,
                                                         const RealState* real, int probe) {
  static_assert(D == 1 || D == 2 || D == 4, "prefetch depth");
  __shared__ double sh[4 * 4];
  const PT* __restrict__ pk = ring + (long long)(kiter[0] % m) * slot_stride;
  const int gx = n / (kWave * V), gy = n / (4 * H);
  const unsigned T = gridDim.x, L = blockIdx.x;
  const unsigned t = (T & 7u) ? L : (L & 7u) * (T >> 3) + (L >> 3);
  const int bx = (int)(t % (unsigned)gx);
  const int by = (int)((t / (unsigned)gx) % (unsigned)gy);
  const int b = (int)(t / (unsigned)(gx * gy));
  const int s0 = 2 * b, s1 = s0 + 1;
  const int act[2] = {sys[s0].active, sys[s1].active};
  if (!act[0] && !act[1]) return;   // uniform over the workgroup
  const double al[2] = {sys[s0].alpha, sys[s1].alpha};
  const double sc[2] = {lo_scale_of<LoT>(sys[s0]), lo_scale_of<LoT>(sys[s1])};
  const int lane = threadIdx.x & 63, w = wave_id();
  const long long N2 = (long long)n * n;
  const int c0 = (bx * kWave + lane) * V;
  const int cl = wrap_dec(c0, n), cr = c0 + V == n ? 0 : c0 + V;
  const int row0 = by * 4 * H + w * H;
  const CoefDec<CT, AT> dec(real, b);
  // the n x n blocks (rows wave-uniform, column byte offsets fixed per lane)
  const Plane<AT> Ap(a + (long long)b * N2, n);
  const Plane<PT> P[2] = {Plane<PT>(pk + (long long)s0 * N2, n), Plane<PT>(pk + (long long)s1 * N2, n)};
  const Plane<double> Rs[2] = {Plane<double>(r + (long long)s0 * N2, n), Plane<double>(r + (long long)s1 * N2, n)};
  const Plane<ZT> Zs[2] = {Plane<ZT>(z + (long long)s0 * N2, n), Plane<ZT>(z + (long long)s1 * N2, n)};
  const Plane<LoT> Ls[2] = {Plane<LoT>(rlo + (long long)s0 * N2, n), Plane<LoT>(rlo + (long long)s1 * N2, n)};
  const unsigned pc0 = c0 * sizeof(PT), pcl = cl * sizeof(PT), pcr = cr * sizeof(PT);
  const unsigned ac0 = c0 * sizeof(AT), acl = cl * sizeof(AT);
  const unsigned rc0 = c0 * sizeof(double), zc0 = c0 * sizeof(ZT), lc0 = c0 * sizeof(LoT);
  // a system that has stopped iterating has its r (and z, and the GEMM copy)
  // neither read nor written: its accesses go past the block instead of
  // sitting behind a branch, so every step issues the same memory
  // instructions and the waits for a row count exactly the ones after it
  const unsigned off_i[2] = {act[0] ? 0u : kPastBlock, act[1] ? 0u : kPastBlock};

  // operand row ro (V + 2 values per system), coefficient row ra (V + 1
  // values) and, with_r, that row's r (and z for the flexible beta). The
  // neighbour columns are loaded here, not taken from the neighbouring lanes
  // as in k_stencil_v: that measured 1 % slower in this pass.
  struct Raw {
    PT p[2][V + 2];
    AT a[V + 1];
    double r[2][V];
    ZT z[2][V];
  };
  auto load_raw = [&](Raw& R, int ro, int ra, bool with_a, bool with_r, unsigned past) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      P[i].template load<V>(ro, pc0, &R.p[i][1]);
      R.p[i][0] = P[i].get(ro, pcl);
      R.p[i][V + 1] = P[i].get(ro, pcr);
    }
    if (with_a) {
      R.a[0] = Ap.get(ra, acl);
      Ap.template load<V>(ra, ac0, &R.a[1]);
    }
    if (with_r) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        Rs[i].template load<V, true>(ra, rc0 + (off_i[i] | past), R.r[i]);
        if constexpr (FLEX) Zs[i].template load<V>(ra, zc0 + (off_i[i] | past), R.z[i]);
      }
    }
  };
  auto cook = [&](const Raw& R, int i, CT* u) {
#pragma unroll
    for (int k = 0; k < V + 2; ++k) u[k] = (CT)R.p[i][k];
  };

  const int rm = wrap_dec(row0, n);
  CT um[2][V + 2], uc[2][V + 2], am[V + 1];
  Raw R[D];
  {
    Raw Ra, Rb;
    load_raw(Ra, rm, rm, true, false, 0);
    load_raw(Rb, row0, 0, false, false, 0);
#pragma unroll
    for (int u = 0; u + 1 < D; ++u) load_raw(R[u], wrap_inc(row0 + u, n), row0 + u, true, true, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      cook(Ra, i, um[i]);
      cook(Rb, i, uc[i]);
    }
#pragma unroll
    for (int k = 0; k < V + 1; ++k) am[k] = dec(Ra.a[k]);
  }

  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // r.r and r.z_old of both systems
  auto step = [&](int j, Raw& use, Raw& fill) {
    const int row = row0 + j;
    // as in k_stencil_v, the loads of step j + D - 1 are issued on every
    // step; past the strip's end the rows of p and a are loaded again (cache
    // hits) and those of r and z not at all (their offsets go past the block)
    {
      const bool past = j + D - 1 >= H;
      const int rc = row0 + min(j + D - 1, H - 1);
      load_raw(fill, wrap_inc(rc, n), rc, true, true, past ? kPastBlock : 0u);
    }
    CT up[2][V + 2];
#pragma unroll
    for (int i = 0; i < 2; ++i) cook(use, i, up[i]);
    CT ac[V + 1];
#pragma unroll
    for (int k = 0; k < V + 1; ++k) ac[k] = dec(use.a[k]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      CT qv[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const CT sm[3] = {um[i][k], um[i][k + 1], um[i][k + 2]};
        const CT sc3[3] = {uc[i][k], uc[i][k + 1], uc[i][k + 2]};
        const CT sp[3] = {up[i][k], up[i][k + 1], up[i][k + 2]};
        if constexpr (SCH == 1)
          qv[k] = fd5_apply<CT>(am[k], am[k + 1], ac[k], ac[k + 1], sm, sc3, sp);
        else
          qv[k] = q1_apply<CT>(am[k], am[k + 1], ac[k], ac[k + 1], sm, sc3, sp);
      }
      {
        double rv[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
          // a probe keeps r exactly (the ring slot it reads may not hold a
          // direction yet, so q is not used at all)
          rv[k] = probe ? use.r[i][k] : fma(-al[i], (double)qv[k], use.r[i][k]);
          if (act[i]) acc[i] += rv[k] * rv[k];
        }
        Rs[i].template store<V, true>(row, rc0 + off_i[i], rv);
        if constexpr (LO) {
          LoT lv[V];
          lo_round_v<LoT, V>(lv, rv, sc[i]);
          Ls[i].template store<V>(row, lc0 + off_i[i], lv);
        }
        if constexpr (FLEX) {
          if (act[i]) {
#pragma unroll
            for (int k = 0; k < V; ++k) acc[2 + i] += rv[k] * (double)use.z[i][k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < V + 2; ++k) {
        um[i][k] = uc[i][k];
        uc[i][k] = up[i][k];
      }
    }
#pragma unroll
    for (int k = 0; k < V + 1; ++k) am[k] = ac[k];
  };
  for (int j = 0; j < H; j += D) {   // H is a multiple of D
#pragma unroll
    for (int u = 0; u < D; ++u) step(j + u, R[u], R[(u + D - 1) % D]);
  }
  block_sum<4>(acc, sh);
  if (threadIdx.x == 0) {
    const int Pt = gx * gy;
    const int tile = by * gx + bx;
    part_rr[(long long)s0 * Pt + tile] = acc[0];
    part_rr[(long long)s1 * Pt + tile] = acc[1];
    part_rzo[(long long)s0 * Pt + tile] = acc[2];
    part_rzo[(long long)s1 * Pt + tile] = acc[3];
  }
}

__global__ void k_scalar_alpha(SysState* sys, const double* __restrict__ part, int P, double* alpha_hist,
                               int m, const int* kiter) {
  const int s = blockIdx.x, lane = threadIdx.x;
  if (!sys[s].active) return;
  const int slot = kiter[0] % m;
  double v = 0;
  for (int t = lane; t < P; t += kWave) v += part[(long long)s * P + t];
  v = wave_sum(v);
  if (lane == 0) {
    SysState& S = sys[s];
    if (!(v > 0.0) || !isfinite(v)) {
      S.active = 0;
      S.status = 2;   // RVE_BREAKDOWN
      S.alpha = 0.0;
    } else {
      S.alpha = S.rz / v;
    }
    alpha_hist[(long long)s * m + slot] = S.alpha;
  }
}

// r -= alpha q, partial sums of r.r (and of r.z for the flexible beta); in
// mixed modes also the GEMM-precision copy of the new r. (Used with the fused
// stencil, which applies the x update.)
template <class ZT, class LoT, bool LO, class QT>
__global__ void __launch_bounds__(kBlock) k_update_r(double* __restrict__ r, const QT* __restrict__ q,
                                                      const ZT* __restrict__ z, LoT* __restrict__ rlo,
                                                      const SysState* sys, long long N2,
                                                      double* __restrict__ part_rr,
                                                      double* __restrict__ part_rzo, int flexible) {
  __shared__ double sh[4 * 2];
  const int s = blockIdx.y;
  if (!sys[s].active) return;
  const double al = sys[s].alpha, sc = lo_scale_of<LoT>(sys[s]);
  const long long off = (long long)s * N2;
  double acc[2] = {0.0, 0.0};
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < N2; i += stride) {
    double rv[4], qv[4];
    V4<double>::load(r + off + i, rv);
    V4<QT>::load(q + off + i, qv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rv[k] = fma(-al, qv[k], rv[k]);
      acc[0] += rv[k] * rv[k];
    }
    V4<double>::store(r + off + i, rv);
    if constexpr (LO) store_lo<LoT>(rlo + off + i, rv, sc);
    if (flexible) {
      double zv[4];
      V4<ZT>::load(z + off + i, zv);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[1] += rv[k] * zv[k];
    }
  }
  block_sum<2>(acc, sh);
  if (threadIdx.x == 0) {
    part_rr[(long long)s * gridDim.x + blockIdx.x] = acc[0];
    part_rzo[(long long)s * gridDim.x + blockIdx.x] = acc[1];
  }
}

// x += alpha_j p_j for j = j0 .. min(j1, iters) - 1 in increasing j, each
// direction read from its ring slot j mod m (m >= kRing, hi - j0 <= kRing). A system's iters counts the
// iterations that produced a direction with a valid step length, so the
// direction of a breakdown (alpha = 0) is never folded in.
//
// final = 0: the fold at the start of iteration k (a multiple of kRing), over
// the kRing directions before it; final = 1: the fold after the last
// iteration K, over the directions since the last multiple of kRing.
template <class PT>
__global__ void __launch_bounds__(kBlock) k_fold_x(double* __restrict__ x, const PT* __restrict__ ring,
                                                    long long slot_stride, int m,
                                                    const double* __restrict__ alpha_hist, const SysState* sys,
                                                    long long N2, const int* kiter, int final) {
  // folds happen every kRing iterations; the ring may hold more slots
  // (m = kRing + 1 when the last transform writes the next direction early)
  const int s = blockIdx.y;
  const int k = kiter[0];
  const int j0 = final ? (k > 0 ? ((k - 1) / kRing) * kRing : 0) : (k > kRing ? k - kRing : 0);
  const int j1 = k;
  const int hi = min(min(j1, sys[s].iters), j0 + kRing);
  if (hi <= j0) return;
  const long long off = (long long)s * N2;
  const long long stride = (long long)gridDim.x * kBlock * 4;
  // all (at most kRing) directions are loaded before the first fma, so each
  // lane has them in flight together; indices past the range repeat the last
  // direction (a cache hit) and are not used
  double al[kRing];
  long long so[kRing];
#pragma unroll
  for (int t = 0; t < kRing; ++t) {
    const int slot = min(j0 + t, hi - 1) % m;
    al[t] = alpha_hist[(long long)s * m + slot];
    so[t] = slot * slot_stride + off;
  }
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < N2; i += stride) {
    double xv[4], pv[kRing][4];
    load_nt<double, 4>(x + off + i, xv);
#pragma unroll
    for (int t = 0; t < kRing; ++t) {
      PT pt[4];
      load_nt<PT, 4>(ring + so[t] + i, pt);
#pragma unroll
      for (int k = 0; k < 4; ++k) pv[t][k] = (double)pt[k];
    }
#pragma unroll
    for (int t = 0; t < kRing; ++t)
      if (j0 + t < hi) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xv[k] = fma(al[t], pv[t][k], xv[k]);
      }
    store_nt<double, 4>(x + off + i, xv);
  }
}

__global__ void k_scalar_conv(SysState* sys, const double* __restrict__ part, int P, double tol, int maxit,
                              int* count, const int* kiter, int scaled, double sqrt_n) {
  // one wave per system; blockDim = 64
  const int s = blockIdx.x, lane = threadIdx.x;
  if (!sys[s].active) return;
  int* count_slot = count + kiter[0];
  double v = 0;
  for (int t = lane; t < P; t += kWave) v += part[(long long)s * P + t];
  v = wave_sum(v);
  if (lane == 0) {
    SysState& S0 = sys[s];
    S0.iters += 1;
    S0.relres = sqrt(v) / S0.fnorm;
    // the residual copy written this iteration carries lo_next; scale the
    // next one to this residual's norm
    S0.lo_scale = S0.lo_next;
    if (scaled && v > 0.0 && isfinite(v)) S0.lo_next = 0.25 * sqrt_n / sqrt(v);
    if (S0.relres <= tol) {
      S0.active = 0;
      S0.status = 0;
    } else if (!isfinite(S0.relres)) {
      S0.active = 0;
      S0.status = 2;
    } else if (S0.iters >= maxit) {
      S0.active = 0;
      S0.status = 1;   // RVE_NOT_CONVERGED
    } else {
      atomicAdd(count_slot, 1);
    }
  }
}

// advance (may be null): the shared iteration counter, advanced once by the
// last batch's beta of an iteration (no block of this kernel reads it)
__global__ void k_scalar_beta(SysState* sys, const double* __restrict__ part_rz, int Pz,
                              const double* __restrict__ part_rzo, int Po, int flexible, int first,
                              int* advance) {
  const int s = blockIdx.x, lane = threadIdx.x;
  if (advance && s == 0 && lane == 0) advance[0] += 1;
  if (!sys[s].active) return;
  double v = 0, o = 0;
  for (int t = lane; t < Pz; t += kWave) v += part_rz[(long long)s * Pz + t];
  if (flexible && !first)
    for (int t = lane; t < Po; t += kWave) o += part_rzo[(long long)s * Po + t];
  v = wave_sum(v);
  o = wave_sum(o);
  if (lane == 0) {
    SysState& S = sys[s];
    S.beta = first ? 0.0 : (v - o) / S.rz;
    S.rz = v;
    if (!(v > 0.0) || !isfinite(v)) {   // the preconditioner must stay positive
      S.active = 0;
      S.status = 2;
    }
  }
}

// rlo = r rounded to the GEMM precision (for applying the preconditioner to a
// caller's residual outside the solver).
template <class LoT>
__global__ void __launch_bounds__(kBlock) k_round_lo(const double* __restrict__ r, LoT* __restrict__ rlo,
                                                      long long total) {
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < total; i += stride) {
    double v[4];
    V4<double>::load(r + i, v);
    V4<LoT>::store(rlo + i, v);
  }
}

__global__ void __launch_bounds__(kBlock) k_widen(const float* __restrict__ in, double* __restrict__ out,
                                                   long long total) {
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < total; i += stride) {
    double v[4];
    V4<float>::load(in + i, v);
    V4<double>::store(out + i, v);
  }
}

// Exact cell integrals for bilinear phi on the unit cell, corners
// u00 = phi[i][j], u01 = phi[i][j+1], u10 = phi[i+1][j], u11 = phi[i+1][j+1]:
// d1 phi is linear in the x2-local coordinate t between b1 = u10 - u00 (t=0)
// and t1 = u11 - u01 (t=1), so int d1u d1v = (b1u b1v + t1u t1v)/3 +
// (b1u t1v + t1u b1v)/6 and int d1u = (b1u + t1u)/2; d2 likewise.
struct CellGrad {
  double b1, t1, b2, t2;
  __device__ CellGrad(double u00, double u01, double u10, double u11)
      : b1(u10 - u00), t1(u11 - u01), b2(u01 - u00), t2(u11 - u10) {}
  __device__ double D1() const { return 0.5 * (b1 + t1); }
  __device__ double D2() const { return 0.5 * (b2 + t2); }
};
// Lumped five-point scheme: the cell's share of the edge quadrature is half
// of each of its four edges, so int d1u d1v -> (b1u b1v + t1u t1v)/2 and
// likewise along x2; the averages D1, D2 are unchanged.
template <int SCH>
__device__ inline double grad_dot(const CellGrad& u, const CellGrad& v) {
  if constexpr (SCH == 1)
    return 0.5 * ((u.b1 * v.b1 + u.t1 * v.t1) + (u.b2 * v.b2 + u.t2 * v.t2));
  return kThird * ((u.b1 * v.b1 + u.t1 * v.t1) + (u.b2 * v.b2 + u.t2 * v.t2)) +
         kSixth * ((u.b1 * v.t1 + u.t1 * v.b1) + (u.b2 * v.t2 + u.t2 * v.b2));
}
// E_ij(e) = int_e (e_i + grad phi_i).(e_j + grad phi_j) in the scheme's quadrature.
template <int SCH>
struct CellEnergy {
  double e11, e12, e22;
  __device__ CellEnergy(const CellGrad& u, const CellGrad& v) {
    e11 = 1.0 + 2.0 * u.D1() + grad_dot<SCH>(u, u);
    e12 = u.D2() + v.D1() + grad_dot<SCH>(u, v);
    e22 = 1.0 + 2.0 * v.D2() + grad_dot<SCH>(v, v);
  }
};

// Per-tile partials of sum_e a_e E_ij(e) (energy form), of the flux-form
// integrands a(delta_ij + d_j phi_i), and of sum phi_i.
template <int SCH>
__global__ void __launch_bounds__(kBlock) k_ahom(const double* __restrict__ a, const double* __restrict__ x,
                                                  int n, double* __restrict__ part) {
  __shared__ double sh[4 * 9];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.z;
  const long long N2 = (long long)n * n;
  const int col = blockIdx.x * kTile + lane, cp = wrap_inc(col, n);
  const int row0 = blockIdx.y * kTile + w * kStrip;
  const double* A = a + (long long)b * N2;
  const double* X0 = x + (2LL * b) * N2;
  const double* X1 = X0 + N2;
  long long o = (long long)row0 * n;
  double u00 = X0[o + col], u01 = X0[o + cp], v00 = X1[o + col], v01 = X1[o + cp];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < kStrip; ++j) {
    const int row = row0 + j;
    const long long on = (long long)wrap_inc(row, n) * n;
    const double u10 = X0[on + col], u11 = X0[on + cp], v10 = X1[on + col], v11 = X1[on + cp];
    const double ae = A[(long long)row * n + col];
    const CellGrad gu(u00, u01, u10, u11), gv(v00, v01, v10, v11);
    const CellEnergy<SCH> E(gu, gv);
    acc[0] += ae * E.e11;
    acc[1] += ae * E.e12;
    acc[2] += ae * E.e22;
    acc[3] += ae * (1.0 + gu.D1());
    acc[4] += ae * gu.D2();
    acc[5] += ae * gv.D1();
    acc[6] += ae * (1.0 + gv.D2());
    acc[7] += u00;
    acc[8] += v00;
    u00 = u10; u01 = u11; v00 = v10; v01 = v11;
  }
  block_sum<9>(acc, sh);
  if (threadIdx.x == 0) {
    const int P = gridDim.x * gridDim.y;
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    double* out = part + ((long long)b * P + tile) * kMiscNV;
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = acc[k];
  }
}

__global__ void k_scalar_ahom(SysState* sys, const double* __restrict__ part, int P, int n,
                              double* __restrict__ ahom, double* __restrict__ ahom_flux) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = lane; t < P; t += kWave) {
    const double* o = part + ((long long)b * P + t) * kMiscNV;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] += o[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
    const double inv = 1.0 / ((double)n * (double)n);
    double* A = ahom + 4LL * b;
    A[0] = v[0] * inv;
    A[1] = v[1] * inv;
    A[2] = v[1] * inv;
    A[3] = v[2] * inv;
    if (ahom_flux) {
      double* F = ahom_flux + 4LL * b;
      F[0] = v[3] * inv;
      F[1] = v[4] * inv;
      F[2] = v[5] * inv;
      F[3] = v[6] * inv;
    }
    sys[2 * b].mean_x = v[7] * inv;
    sys[2 * b + 1].mean_x = v[8] * inv;
  }
}

__global__ void __launch_bounds__(kBlock) k_phi_out(const double* __restrict__ x, double* __restrict__ phi,
                                                     const SysState* sys, long long N2, double h) {
  const int s = blockIdx.y;
  const double m = sys[s].mean_x;
  const long long off = (long long)s * N2;
  const long long stride = (long long)gridDim.x * kBlock * 2;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 2; i < N2; i += stride) {
    const double2 xv = *reinterpret_cast<const double2*>(x + off + i);
    double2 o;
    o.x = h * (xv.x - m);
    o.y = h * (xv.y - m);
    *reinterpret_cast<double2*>(phi + off + i) = o;
  }
}

__global__ void k_finalize(const SysState* sys, int B, int* iters, double* relres, int* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const SysState& s0 = sys[2 * b];
  const SysState& s1 = sys[2 * b + 1];
  if (iters) {
    iters[2 * b] = s0.iters;
    iters[2 * b + 1] = s1.iters;
  }
  if (relres) {
    relres[2 * b] = s0.relres;
    relres[2 * b + 1] = s1.relres;
  }
  if (status) {
    // errors (negative codes) dominate; otherwise the larger warning code
    const int c0 = s0.status, c1 = s1.status;
    status[b] = (c0 < 0 || c1 < 0) ? min(c0, c1) : max(c0, c1);
  }
}

// grad[e] = sum_ij G_ij dA_ij/da_e = (G11 E11 + (G12 + G21) E12 + G22 E22)/n^2,
// plus per-tile partial sums over the inclusion cells: those with
// mask[e] != 0, or (mask == nullptr) those with a_e == a_in.
template <int SCH>
__global__ void __launch_bounds__(kBlock) k_grad(const double* __restrict__ a, const double* __restrict__ phi,
                                                  double inv_h, const double* __restrict__ G,
                                                  double* __restrict__ grad, double a_in,
                                                  const unsigned char* __restrict__ mask, int n,
                                                  double* __restrict__ part, int want_in) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.z;
  const long long N2 = (long long)n * n;
  const int col = blockIdx.x * kTile + lane, cp = wrap_inc(col, n);
  const int row0 = blockIdx.y * kTile + w * kStrip;
  const double* A = a + (long long)b * N2;
  const double* X0 = phi + (2LL * b) * N2;
  const double* X1 = X0 + N2;
  double* Gr = grad + (long long)b * N2;
  const double inv_n2 = 1.0 / ((double)n * (double)n);
  const double g11 = G[4 * b] * inv_n2, g12 = (G[4 * b + 1] + G[4 * b + 2]) * inv_n2, g22 = G[4 * b + 3] * inv_n2;
  long long o = (long long)row0 * n;
  double u00 = X0[o + col] * inv_h, u01 = X0[o + cp] * inv_h;
  double v00 = X1[o + col] * inv_h, v01 = X1[o + cp] * inv_h;
  double acc[1] = {0.0};
  for (int j = 0; j < kStrip; ++j) {
    const int row = row0 + j;
    const long long on = (long long)wrap_inc(row, n) * n;
    const double u10 = X0[on + col] * inv_h, u11 = X0[on + cp] * inv_h;
    const double v10 = X1[on + col] * inv_h, v11 = X1[on + cp] * inv_h;
    const CellEnergy<SCH> E(CellGrad(u00, u01, u10, u11), CellGrad(v00, v01, v10, v11));
    const double g = g11 * E.e11 + g12 * E.e12 + g22 * E.e22;
    const long long oc = (long long)row * n + col;
    Gr[oc] = g;
    if (want_in && (mask ? mask[(long long)b * N2 + oc] != 0 : A[oc] == a_in)) acc[0] += g;
    u00 = u10; u01 = u11; v00 = v10; v01 = v11;
  }
  if (want_in) {
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) {
      const int P = gridDim.x * gridDim.y;
      part[(long long)b * P + blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
    }
  }
}

__global__ void k_scalar_grad(const double* __restrict__ part, int P, double* grad_in) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double v = 0;
  for (int t = lane; t < P; t += kWave) v += part[(long long)b * P + t];
  v = wave_sum(v);
  if (lane == 0) grad_in[b] = v;
}

// out[0] = sum_b v[b], one wave, fixed order.
__global__ void k_sum_items(const double* __restrict__ v, int B, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double s = 0;
  for (int b = lane; b < B; b += kWave) s += v[b];
  s = wave_sum(s);
  if (lane == 0) out[0] = s;
}

// a[b][e] = mask[b][e] ? a_in[b] : a_bg (the covered set of eqn. Stoch-decomp
// carries the inclusion value, eqn. ahm_coef).
__global__ void __launch_bounds__(kBlock) k_field_from_mask(const unsigned char* __restrict__ mask,
                                                             const double* __restrict__ a_in, double a_bg,
                                                             long long N2, double* __restrict__ a) {
  const int b = blockIdx.y;
  const double ain = a_in[b];
  const long long off = (long long)b * N2;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < N2; i += stride)
    a[off + i] = mask[off + i] ? ain : a_bg;
}

// Ensemble statistics in one workgroup (fixed-order reductions).
__global__ void __launch_bounds__(kBlock) k_stats(const double* __restrict__ A, int N, double L,
                                                   double* __restrict__ out) {
  __shared__ double sh[4 * 18];
  __shared__ double mean[4];
  double s[4] = {0, 0, 0, 0};
  for (int t = threadIdx.x; t < N; t += kBlock)
    for (int k = 0; k < 4; ++k) s[k] += A[4LL * t + k];
  block_sum<4>(s, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) mean[k] = s[k] / N;
  __syncthreads();
  double c[18];
  for (int k = 0; k < 18; ++k) c[k] = 0.0;
  for (int t = threadIdx.x; t < N; t += kBlock) {
    double d[4], raw[4];
    for (int k = 0; k < 4; ++k) {
      raw[k] = A[4LL * t + k];
      d[k] = raw[k] - mean[k];
    }
    // q[(i,k),(j,l)] = cov(A_ij, A_kl): row (i,k) -> 2i+k, col (j,l) -> 2j+l
    for (int i = 0; i < 2; ++i)
      for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
          for (int l = 0; l < 2; ++l) c[(2 * i + k) * 4 + (2 * j + l)] += d[2 * i + j] * d[2 * k + l];
    c[16] += raw[1] * raw[1];
    const double dd = raw[0] - raw[3];
    c[17] += dd * dd;
  }
  block_sum<18>(c, sh);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) out[k] = mean[k];
    // centred variances are the diagonal covariances cov(A_ij, A_ij)
    // var(A_ij) = cov(A_ij, A_ij) sits at row (i,i), column (j,j)
    out[4] = c[0 * 4 + 0] / (N - 1);            // A11: row (0,0), col (0,0)
    out[5] = c[0 * 4 + 3] / (N - 1);            // A12: row (0,0), col (1,1)
    out[6] = c[3 * 4 + 0] / (N - 1);            // A21: row (1,1), col (0,0)
    out[7] = c[3 * 4 + 3] / (N - 1);            // A22: row (1,1), col (1,1)
    out[8] = sqrt(c[16] / N);
    out[9] = sqrt(c[17] / N);
    const double scale = L * L / (N - 1);
    for (int k = 0; k < 16; ++k) out[10 + k] = scale * c[k];
  }
}

inline int vec_blocks(long long N2) {
  long long nb = (N2 + 4LL * kBlock - 1) / (4LL * kBlock);
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return (int)nb;
}

}  // namespace

// ---------------------------------------------------------------- launchers

void launch_init_state(const Work& w, hipStream_t st) {
  int blocks = (w.S + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(kBlock), 0, st, w.sys, w.real, w.S, w.B);
}

void launch_encode_two_valued(const Work& w, uint8_t* code, int* not_two_valued, hipStream_t st) {
  long long blocks = (w.N2 / 4 + kBlock - 1) / kBlock;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_encode_two_valued, dim3((unsigned)blocks, w.B), dim3(kBlock), 0, st, w.a, w.real, w.N2, code,
                     not_two_valued);
}

void launch_ctl_reset(int* kiter, int* count, int count_len, hipStream_t st) {
  int blocks = (count_len + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_ctl_reset, dim3(blocks), dim3(kBlock), 0, st, kiter, count, count_len);
}


void launch_rhs(const Work& w, hipStream_t st) {
  if (w.dim == 3) return launch_rhs3(w, st);
  dim3 g(w.n / kTile, w.n / kTile, w.B);
  hipLaunchKernelGGL(k_rhs, g, dim3(kBlock), 0, st, w.a, w.r, w.n, w.part_misc);
}

void launch_scalar_init(const Work& w, hipStream_t st) {
  if (w.dim == 3) return launch_scalar_init3(w, st);
  hipLaunchKernelGGL(k_scalar_init, dim3(w.B), dim3(kWave), 0, st, w.sys, w.real, w.part_misc, w.P_tile, w.n,
                     (int)(w.mixed == 3));
}

void launch_meansub(const Work& w, hipStream_t st) {
  const dim3 g(w.P_vec, w.S), blk(kBlock);
  if (w.mixed == 0)
    hipLaunchKernelGGL((k_meansub<double, false>), g, blk, 0, st, w.r, w.x, (double*)nullptr, w.sys, w.N2,
                       w.part_rr);
  else if (w.mixed == 1)
    hipLaunchKernelGGL((k_meansub<float, true>), g, blk, 0, st, w.r, w.x, (float*)w.rlo, w.sys, w.N2,
                       w.part_rr);
  else if (w.mixed == 3)
    hipLaunchKernelGGL((k_meansub<_Float16, true>), g, blk, 0, st, w.r, w.x, (_Float16*)w.rlo, w.sys, w.N2,
                       w.part_rr);
  else
    hipLaunchKernelGGL((k_meansub<__bf16, true>), g, blk, 0, st, w.r, w.x, (__bf16*)w.rlo, w.sys, w.N2,
                       w.part_rr);
}

void launch_scalar_fnorm(const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_fnorm, dim3(w.S), dim3(kWave), 0, st, w.sys, w.part_rr, w.P_vec,
                     (int)(w.mixed == 3), sqrt((double)w.N2));
}


// Default operator-apply shape: the widest column count that divides the
// grid, 16-row strips.
int stencil_choice_default(int n) { return (n % 256 == 0 ? 4 : n % 128 == 0 ? 2 : 1) + 8 * (kStrip / 16); }
bool stencil_choice_valid(int n, int c) {
  if (c < 0 || c >= 256 || (c & 192) == 192) return false;
  const int V = stencil_choice_V(c), H = stencil_choice_H(c);
  if (!(V == 1 || V == 2 || V == 4) || !(H == 16 || H == 32 || H == 64)) return false;
  return n % (kWave * V) == 0 && n % (4 * H) == 0;
}

template <bool FUSED, class PT, class ZT, int D, class CT, int SCH, class AT, bool PDIR>
void launch_stencil_d(int B, int n, int V, int H, const AT* a, const PT* pin, PT* ring, long long slot_stride,
                      int m, const int* kiter, const ZT* z, CT* q, const SysState* sys, double* part,
                      int probe, int wq, const RealState* real, hipStream_t st) {
  const dim3 g((unsigned)((n / (kWave * V)) * (n / (4 * H)) * B)), blk(kBlock);
  if (V == 4)
    hipLaunchKernelGGL((k_stencil_v<FUSED, PT, ZT, 4, D, CT, SCH, AT, PDIR>), g, blk, 0, st, a, pin, ring,
                       slot_stride, m, kiter, z, q, n, H, sys, part, probe, wq, real);
  else if (V == 2)
    hipLaunchKernelGGL((k_stencil_v<FUSED, PT, ZT, 2, D, CT, SCH, AT, PDIR>), g, blk, 0, st, a, pin, ring,
                       slot_stride, m, kiter, z, q, n, H, sys, part, probe, wq, real);
  else
    hipLaunchKernelGGL((k_stencil_v<FUSED, PT, ZT, 1, D, CT, SCH, AT, PDIR>), g, blk, 0, st, a, pin, ring,
                       slot_stride, m, kiter, z, q, n, H, sys, part, probe, wq, real);
}

template <bool FUSED, class PT, class ZT, class CT, int SCH, class AT = CT, bool PDIR = false>
void launch_stencil_t(int B, int n, int c, const AT* a, const PT* pin, PT* ring, long long slot_stride, int m,
                      const int* kiter, const ZT* z, CT* q, const SysState* sys, double* part, int probe,
                      hipStream_t st, int wq = 1, const RealState* real = nullptr) {
  const int V = stencil_choice_V(c), H = stencil_choice_H(c), D = stencil_choice_D(c);
  if (D == 4)
    launch_stencil_d<FUSED, PT, ZT, 4, CT, SCH, AT, PDIR>(B, n, V, H, a, pin, ring, slot_stride, m, kiter, z, q,
                                                          sys, part, probe, wq, real, st);
  else if (D == 2)
    launch_stencil_d<FUSED, PT, ZT, 2, CT, SCH, AT, PDIR>(B, n, V, H, a, pin, ring, slot_stride, m, kiter, z, q,
                                                          sys, part, probe, wq, real, st);
  else
    launch_stencil_d<FUSED, PT, ZT, 1, CT, SCH, AT, PDIR>(B, n, V, H, a, pin, ring, slot_stride, m, kiter, z, q,
                                                          sys, part, probe, wq, real, st);
}

template <class PT, int SCH, bool PDIR>
void launch_stencil_fused_m(const Work& w, int probe, hipStream_t st) {
  const long long slot = (long long)w.S * w.N2;
  // two-valued fields: one byte per cell instead of eight
  if (w.a8)
    launch_stencil_t<true, PT, PT, double, SCH, uint8_t, PDIR>(w.B, w.n, w.stencil, w.a8, (const PT*)nullptr,
                                                               (PT*)w.pring, slot, w.m_ring, w.kiter, (const PT*)w.z,
                                                               w.q, w.sys, w.part_pq, probe, st, !w.qfree, w.real);
  else
    launch_stencil_t<true, PT, PT, double, SCH, double, PDIR>(w.B, w.n, w.stencil, w.a, (const PT*)nullptr,
                                                              (PT*)w.pring, slot, w.m_ring, w.kiter, (const PT*)w.z,
                                                              w.q, w.sys, w.part_pq, probe, st, !w.qfree, w.real);
}

template <class PT, int SCH>
void launch_stencil_fused_s(const Work& w, int probe, hipStream_t st) {
  if (w.pdirect) launch_stencil_fused_m<PT, SCH, true>(w, probe, st);
  else launch_stencil_fused_m<PT, SCH, false>(w, probe, st);
}

template <class PT>
void launch_stencil_fused_p(const Work& w, int probe, hipStream_t st) {
  const long long slot = (long long)w.S * w.N2;
  if (w.sprec)   // FP32 apply: the Q1 operator only
    launch_stencil_t<true, PT, PT, float, 0>(w.B, w.n, w.stencil, w.a32, (const PT*)nullptr, (PT*)w.pring, slot,
                                             w.m_ring, w.kiter, (const PT*)w.z, (float*)w.q, w.sys, w.part_pq,
                                             probe, st);
  else if (w.scheme == 1)
    launch_stencil_fused_s<PT, 1>(w, probe, st);
  else
    launch_stencil_fused_s<PT, 0>(w, probe, st);
}

void launch_stencil_fused(const Work& w, hipStream_t st, int probe) {
  if (w.dim == 3) return launch_stencil3_fused(w, st, probe);
  // iteration k (read on the device) writes p_k into ring slot k mod m and
  // reads p_{k-1} from the previous slot
  if (w.mixed == 0)
    launch_stencil_fused_p<double>(w, probe, st);
  else if (w.pdir16 && w.scheme == 1)
    launch_stencil_fused_m<__bf16, 1, true>(w, probe, st);
  else if (w.pdir16)
    launch_stencil_fused_m<__bf16, 0, true>(w, probe, st);
  else
    launch_stencil_fused_p<float>(w, probe, st);
}

int stencil_tiles_per_realization(int n, int c) {
  return (n / (kWave * stencil_choice_V(c))) * (n / (4 * stencil_choice_H(c)));
}

template <class PT, class LoT, bool LO, int D, int SCH, class AT, bool FLEX>
void launch_update_r_st_a(const Work& w, const AT* a, int probe, hipStream_t st) {
  const int V = stencil_choice_V(w.ustencil), H = stencil_choice_H(w.ustencil);
  const dim3 g((unsigned)((w.n / (kWave * V)) * (w.n / (4 * H)) * w.B)), blk(kBlock);
  const long long slot = (long long)w.S * w.N2;
  const PT* ring = (const PT*)w.pring;
  const PT* z = (const PT*)w.z;
  LoT* rlo = (LoT*)w.rlo;
  if (V == 4)
    hipLaunchKernelGGL((k_update_r_st<PT, PT, LoT, LO, 4, D, double, SCH, AT, FLEX>), g, blk, 0, st, a, ring, slot,
                       w.m_ring, (const int*)w.kiter, z, w.r, rlo, w.n, H, w.sys, w.part_rr, w.part_rzo, w.real,
                       probe);
  else if (V == 2)
    hipLaunchKernelGGL((k_update_r_st<PT, PT, LoT, LO, 2, D, double, SCH, AT, FLEX>), g, blk, 0, st, a, ring, slot,
                       w.m_ring, (const int*)w.kiter, z, w.r, rlo, w.n, H, w.sys, w.part_rr, w.part_rzo, w.real,
                       probe);
  else
    hipLaunchKernelGGL((k_update_r_st<PT, PT, LoT, LO, 1, D, double, SCH, AT, FLEX>), g, blk, 0, st, a, ring, slot,
                       w.m_ring, (const int*)w.kiter, z, w.r, rlo, w.n, H, w.sys, w.part_rr, w.part_rzo, w.real,
                       probe);
}

template <class PT, class LoT, bool LO, int D, int SCH, bool FLEX>
void launch_update_r_st_d(const Work& w, int probe, hipStream_t st) {
  if (w.a8) launch_update_r_st_a<PT, LoT, LO, D, SCH, uint8_t, FLEX>(w, w.a8, probe, st);
  else launch_update_r_st_a<PT, LoT, LO, D, SCH, double, FLEX>(w, w.a, probe, st);
}

template <class PT, class LoT, bool LO, int SCH, bool FLEX>
void launch_update_r_st_s(const Work& w, int probe, hipStream_t st) {
  const int D = stencil_choice_D(w.ustencil);
  if (D == 4) launch_update_r_st_d<PT, LoT, LO, 4, SCH, FLEX>(w, probe, st);
  else if (D == 2) launch_update_r_st_d<PT, LoT, LO, 2, SCH, FLEX>(w, probe, st);
  else launch_update_r_st_d<PT, LoT, LO, 1, SCH, FLEX>(w, probe, st);
}

template <class PT, class LoT, bool LO>
void launch_update_r_st_l(const Work& w, int flexible, int probe, hipStream_t st) {
  if (w.scheme == 1) {
    if (flexible) launch_update_r_st_s<PT, LoT, LO, 1, true>(w, probe, st);
    else launch_update_r_st_s<PT, LoT, LO, 1, false>(w, probe, st);
  } else {
    if (flexible) launch_update_r_st_s<PT, LoT, LO, 0, true>(w, probe, st);
    else launch_update_r_st_s<PT, LoT, LO, 0, false>(w, probe, st);
  }
}

// the residual update with A p_k recomputed (w.qfree: FP64 operator apply,
// two dimensions) in its own tile shape w.ustencil; r.r and r.z_old partials
// per tile of that shape (w.P_rr). FP64 directions go with the FP64 GEMM
// copy-free path, FP32 ones with an FP32, FP16 or BF16 copy of r; BF16
// ones (only where the last transform forms them, so never with the
// flexible beta) with a BF16 or FP16 copy.
void launch_update_r_st(const Work& w, int flexible, int probe, hipStream_t st) {
  if (w.mixed == 0) launch_update_r_st_l<double, double, false>(w, flexible, probe, st);
  else if (w.pdir16 && w.mixed == 3) launch_update_r_st_l<__bf16, _Float16, true>(w, 0, probe, st);
  else if (w.pdir16) launch_update_r_st_l<__bf16, __bf16, true>(w, 0, probe, st);
  else if (w.mixed == 1) launch_update_r_st_l<float, float, true>(w, flexible, probe, st);
  else if (w.mixed == 3) launch_update_r_st_l<float, _Float16, true>(w, flexible, probe, st);
  else launch_update_r_st_l<float, __bf16, true>(w, flexible, probe, st);
}

template <class QT>
void launch_update_r_q(const Work& w, int flexible, hipStream_t st) {
  const dim3 g(w.P_vec, w.S), blk(kBlock);
  const QT* q = reinterpret_cast<const QT*>(w.q);
  if (w.mixed == 0)
    hipLaunchKernelGGL((k_update_r<double, double, false, QT>), g, blk, 0, st, w.r, q, (const double*)w.z,
                       (double*)nullptr, w.sys, w.N2, w.part_rr, w.part_rzo, flexible);
  else if (w.mixed == 1)
    hipLaunchKernelGGL((k_update_r<float, float, true, QT>), g, blk, 0, st, w.r, q, (const float*)w.z,
                       (float*)w.rlo, w.sys, w.N2, w.part_rr, w.part_rzo, flexible);
  else if (w.mixed == 3)
    hipLaunchKernelGGL((k_update_r<float, _Float16, true, QT>), g, blk, 0, st, w.r, q, (const float*)w.z,
                       (_Float16*)w.rlo, w.sys, w.N2, w.part_rr, w.part_rzo, flexible);
  else
    hipLaunchKernelGGL((k_update_r<float, __bf16, true, QT>), g, blk, 0, st, w.r, q, (const float*)w.z,
                       (__bf16*)w.rlo, w.sys, w.N2, w.part_rr, w.part_rzo, flexible);
}

void launch_update_r(const Work& w, int flexible, hipStream_t st, int probe) {
  if (w.qfree) {
    launch_update_r_st(w, flexible, probe, st);
    return;
  }
  // q = A p is FP32 with the FP32 operator apply
  if (w.sprec)
    launch_update_r_q<float>(w, flexible, st);
  else
    launch_update_r_q<double>(w, flexible, st);
}

// r = f - A x for every active system, and its GEMM-precision copy: the
// residual replacement of the FP32 operator apply (A x in FP64 in q).
template <class LoT, bool LO>
__global__ void __launch_bounds__(kBlock) k_replace_r(double* __restrict__ r, const double* __restrict__ f,
                                                       const double* __restrict__ ax, LoT* __restrict__ rlo,
                                                       const SysState* sys, long long N2) {
  const int s = blockIdx.y;
  if (!sys[s].active) return;
  const double sc = lo_scale_of<LoT>(sys[s]);
  const long long off = (long long)s * N2;
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < N2; i += stride) {
    double fv[4], qv[4];
    V4<double>::load(f + off + i, fv);
    V4<double>::load(ax + off + i, qv);
#pragma unroll
    for (int k = 0; k < 4; ++k) fv[k] -= qv[k];
    V4<double>::store(r + off + i, fv);
    if constexpr (LO) store_lo<LoT>(rlo + off + i, fv, sc);
  }
}

void launch_replace_r(const Work& w, hipStream_t st) {
  // A x (FP64) into q, then r = f - A x
  launch_apply_stencil(w.B, w.n, 0, w.a, w.x, w.q, st);
  const dim3 g(w.P_vec, w.S), blk(kBlock);
  if (w.mixed == 0)
    hipLaunchKernelGGL((k_replace_r<double, false>), g, blk, 0, st, w.r, (const double*)w.f, (const double*)w.q,
                       (double*)nullptr, w.sys, w.N2);
  else if (w.mixed == 1)
    hipLaunchKernelGGL((k_replace_r<float, true>), g, blk, 0, st, w.r, (const double*)w.f, (const double*)w.q,
                       (float*)w.rlo, w.sys, w.N2);
  else if (w.mixed == 3)
    hipLaunchKernelGGL((k_replace_r<_Float16, true>), g, blk, 0, st, w.r, (const double*)w.f, (const double*)w.q,
                       (_Float16*)w.rlo, w.sys, w.N2);
  else
    hipLaunchKernelGGL((k_replace_r<__bf16, true>), g, blk, 0, st, w.r, (const double*)w.f, (const double*)w.q,
                       (__bf16*)w.rlo, w.sys, w.N2);
}

__global__ void __launch_bounds__(kBlock) k_to_f32(const double* __restrict__ in, float* __restrict__ out,
                                                    long long total) {
  const long long stride = (long long)gridDim.x * kBlock * 4;
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; i < total; i += stride) {
    double v[4];
    V4<double>::load(in + i, v);
    V4<float>::store(out + i, v);
  }
}

void launch_to_f32(const double* in, float* out, long long total, hipStream_t st) {
  long long nb = (total + 4LL * kBlock - 1) / (4LL * kBlock);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, total);
}

void launch_fold_x(const Work& w, int final, hipStream_t st) {
  const dim3 g(w.P_vec, w.S), blk(kBlock);
  const long long slot = (long long)w.S * w.N2;
  if (w.mixed == 0)
    hipLaunchKernelGGL((k_fold_x<double>), g, blk, 0, st, w.x, (const double*)w.pring, slot, w.m_ring,
                       w.alpha_hist, w.sys, w.N2, (const int*)w.kiter, final);
  else if (w.pdir16)
    hipLaunchKernelGGL((k_fold_x<__bf16>), g, blk, 0, st, w.x, (const __bf16*)w.pring, slot, w.m_ring,
                       w.alpha_hist, w.sys, w.N2, (const int*)w.kiter, final);
  else
    hipLaunchKernelGGL((k_fold_x<float>), g, blk, 0, st, w.x, (const float*)w.pring, slot, w.m_ring,
                       w.alpha_hist, w.sys, w.N2, (const int*)w.kiter, final);
}

void launch_apply_stencil(int B, int n, int scheme, const double* a, const double* u, double* out, hipStream_t st) {
  if (scheme == 1)
    launch_stencil_t<false, double, double, double, 1>(B, n, stencil_choice_default(n), a, u, (double*)nullptr, 0,
                                                       1, (const int*)nullptr, (const double*)nullptr, out,
                                                       (const SysState*)nullptr, (double*)nullptr, 0, st);
  else
    launch_stencil_t<false, double, double, double, 0>(B, n, stencil_choice_default(n), a, u, (double*)nullptr, 0,
                                                       1, (const int*)nullptr, (const double*)nullptr, out,
                                                       (const SysState*)nullptr, (double*)nullptr, 0, st);
}

void launch_scalar_alpha(const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_alpha, dim3(w.S), dim3(kWave), 0, st, w.sys, w.part_pq, w.P_st, w.alpha_hist,
                     w.m_ring, (const int*)w.kiter);
}


void launch_scalar_conv(const Work& w, double tol, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_conv, dim3(w.S), dim3(kWave), 0, st, w.sys, w.part_rr, w.P_rr, tol, maxit,
                     w.count, (const int*)w.kiter, (int)(w.mixed == 3), sqrt((double)w.N2));
}

__global__ void k_advance(int* kiter) {
  if (threadIdx.x == 0) kiter[0] += 1;
}

void launch_advance(int* kiter, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(kWave), 0, st, kiter);
}

void launch_scalar_beta(const Work& w, int flexible, int first, hipStream_t st, int* advance) {
  hipLaunchKernelGGL(k_scalar_beta, dim3(w.S), dim3(kWave), 0, st, w.sys, w.part_rz, w.P_gemm, w.part_rzo,
                     w.P_rr, flexible, first, advance);
}

void launch_round_lo(const Work& w, hipStream_t st) {
  const long long total = (long long)w.S * w.N2;
  long long nb = (total + 4LL * kBlock - 1) / (4LL * kBlock);
  if (nb > 4096) nb = 4096;
  if (w.mixed == 1)
    hipLaunchKernelGGL((k_round_lo<float>), dim3((unsigned)nb), dim3(kBlock), 0, st, w.r, (float*)w.rlo, total);
  else if (w.mixed == 3)
    hipLaunchKernelGGL((k_round_lo<_Float16>), dim3((unsigned)nb), dim3(kBlock), 0, st, w.r, (_Float16*)w.rlo,
                       total);
  else if (w.mixed == 2)
    hipLaunchKernelGGL((k_round_lo<__bf16>), dim3((unsigned)nb), dim3(kBlock), 0, st, w.r, (__bf16*)w.rlo,
                       total);
}

void launch_widen(const float* in, double* out, long long total, hipStream_t st) {
  long long nb = (total + 4LL * kBlock - 1) / (4LL * kBlock);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, total);
}


void launch_ahom(const Work& w, hipStream_t st) {
  if (w.dim == 3) return launch_ahom3(w, st);
  dim3 g(w.n / kTile, w.n / kTile, w.B);
  if (w.scheme == 1)
    hipLaunchKernelGGL(k_ahom<1>, g, dim3(kBlock), 0, st, w.a, w.x, w.n, w.part_misc);
  else
    hipLaunchKernelGGL(k_ahom<0>, g, dim3(kBlock), 0, st, w.a, w.x, w.n, w.part_misc);
}

void launch_scalar_ahom(const Work& w, double* ahom, double* ahom_flux, hipStream_t st) {
  if (w.dim == 3) return launch_scalar_ahom3(w, ahom, ahom_flux, st);
  hipLaunchKernelGGL(k_scalar_ahom, dim3(w.B), dim3(kWave), 0, st, w.sys, w.part_misc, w.P_tile, w.n, ahom,
                     ahom_flux);
}

void launch_phi_out(const Work& w, double* phi, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_phi_out, dim3(w.P_vec, w.S), dim3(kBlock), 0, st, w.x, phi, w.sys, w.N2, h);
}

void launch_finalize(const Work& w, int* iters, double* relres, int* status, hipStream_t st) {
  if (w.dim == 3) return launch_finalize3(w, iters, relres, status, st);
  hipLaunchKernelGGL(k_finalize, dim3((w.B + kBlock - 1) / kBlock), dim3(kBlock), 0, st, w.sys, w.B, iters,
                     relres, status);
}

void launch_grad(int B, int n, int scheme, const double* a, const double* phi, double inv_h, const double* G,
                 double* grad, double a_in, const unsigned char* mask, double* part, int want_in, hipStream_t st) {
  dim3 g(n / kTile, n / kTile, B);
  if (scheme == 1)
    hipLaunchKernelGGL(k_grad<1>, g, dim3(kBlock), 0, st, a, phi, inv_h, G, grad, a_in, mask, n, part, want_in);
  else
    hipLaunchKernelGGL(k_grad<0>, g, dim3(kBlock), 0, st, a, phi, inv_h, G, grad, a_in, mask, n, part, want_in);
}

int grad_tiles_per_realization(int n) { return (n / kTile) * (n / kTile); }

void launch_scalar_grad(int B, int n, const double* part, double* grad_in, double* grad_in_sum, hipStream_t st) {
  const int P = grad_tiles_per_realization(n);
  hipLaunchKernelGGL(k_scalar_grad, dim3(B), dim3(kWave), 0, st, part, P, grad_in);
  if (grad_in_sum) hipLaunchKernelGGL(k_sum_items, dim3(1), dim3(kWave), 0, st, grad_in, B, grad_in_sum);
}

void launch_field_from_mask(int B, long long N2, const unsigned char* mask, const double* a_in, double a_bg,
                            double* a, hipStream_t st) {
  long long blocks = (N2 + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_field_from_mask, dim3((unsigned)blocks, B), dim3(kBlock), 0, st, mask, a_in, a_bg, N2, a);
}

void launch_stats(int N, double L, const double* ahom, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(kBlock), 0, st, ahom, N, L, out);
}

int vec_blocks_per_system(long long N2) { return vec_blocks(N2); }

}  // namespace rve
