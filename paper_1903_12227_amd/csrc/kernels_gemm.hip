// Preconditioner apply z = (a0 A_Delta)^+ r by Kronecker diagonalisation,
// as dense transform GEMMs on the MFMA units (gfx950).
//
// A_Delta = K (x) M + M (x) K is the constant-coefficient periodic Q1
// operator (grid units): K = circ(-1, 2, -1), M = circ(1, 4, 1)/6. Both are
// symmetric circulants, so the symmetric orthogonal Hartley matrix
// Q[k][j] = cas(2 pi k j / n)/sqrt(n) (cas = cos + sin, Q = Q^T, Q^2 = I)
// diagonalises both factors, and for an n x n residual R
//     Z = Q [ (Q R Q) ./ (a0 E) ] Q,  E[k][l] = (8 - 2c_k - 2c_l - 4 c_k c_l)/3,
// c_k = cos(2 pi k / n), with the (0,0) entry of 1/E set to zero (the
// pseudo-inverse on the mean-zero subspace; Sec. 3.5 uses B = a0 A_Delta +
// delta I with delta -> 0).
//
// Every GEMM here has the same shape: out_s = (X_s Q)^T for each system s,
// X_s row-major with the contraction index contiguous. Since Q is symmetric,
// two such GEMMs give ((X Q)^T Q)^T = Q X Q, so the four transforms are four
// launches of one kernel; the first reads the FP64 residual and converts,
// the second scales by 1/(a0 E), the fourth writes z in FP64 and emits
// partial sums of r.z.
//
// Three dimensions (eqn. As_Kron_d): A_Delta = K (x) M (x) M + M (x) K (x) M
// + M (x) M (x) K is diagonalised by Q (x) Q (x) Q with
// E[k][l][m] = kappa_k mu_l mu_m + mu_k kappa_l mu_m + mu_k mu_l kappa_m,
// kappa = 2 - 2c, mu = (4 + 2c)/6. Viewing an n x n x n array as an n^2 x n
// matrix (x3 contiguous), out = (X Q)^T transforms the last axis and rotates
// the axes ([i][j][k] -> [k][i][j]), so three such GEMMs transform every
// axis and restore the layout: six launches of the same kernel (D = 3, row
// count n^2), the third scaling by 1/(a0 E).
//
// Tiling: 256 threads (2 x 2 waves) per 64 x 64 output tile; each wave owns
// a 32 x 32 block = 2 x 2 MFMA 16x16 tiles. Operand tiles are staged through
// LDS with the next K slice prefetched into registers; the output tile is
// transposed through LDS so global stores are contiguous. Tiles are ordered
// so that the n/64 tiles sharing one A row-block are consecutive and land on
// one XCD (its L2 then holds that row-block once).
#include <type_traits>

#include "launch.h"

namespace rve {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64;

// MFMA precision traits. Lane layouts (wave64, 16x16 output):
//   operands: lane l supplies row/column l%16 at contraction slice l/16
//             (FP64/FP32: one value; BF16: 8 consecutive values);
//   FP64 accumulator register i of lane l: row (l/16) + 4i, column l%16;
//   FP32 accumulator register i of lane l: row 4(l/16) + i, column l%16.
struct TrF64 {
  using op_t = double;
  using acc_t = double;
  using accv_t = v4d;
  static constexpr int BK = 16, KM = 4, PAD = 1;
  __device__ static accv_t mma(const op_t* a, const op_t* b, accv_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(*a, *b, c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
struct TrF32 {
  using op_t = float;
  using acc_t = float;
  using accv_t = v4f;
  static constexpr int BK = 16, KM = 4, PAD = 1;
  __device__ static accv_t mma(const op_t* a, const op_t* b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
struct TrBF16 {
  using op_t = __bf16;
  using acc_t = float;
  using accv_t = v4f;
  static constexpr int BK = 64, KM = 32, PAD = 8;
  __device__ static accv_t mma(const op_t* a, const op_t* b, accv_t c) {
    const v8bf av = *reinterpret_cast<const v8bf*>(a);
    const v8bf bv = *reinterpret_cast<const v8bf*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// FP16 operands (16x16x32, FP32 accumulation; same lane layouts as BF16).
// The FP16 path keeps every operand in range by scaling: the residual copy
// is stored times a per-system factor sigma (0.25 sqrt(N) / ||r||, so its
// 2-norm is about sqrt(N)/4), the symbol's reciprocal is stored as
// E_min / E <= 1, and since the transforms are orthogonal no entry of any
// intermediate exceeds the 2-norm of the scaled input; the last transform
// multiplies by 1 / (sigma E_min a0).
struct TrF16 {
  using op_t = _Float16;
  using acc_t = float;
  using accv_t = v4f;
  static constexpr int BK = 64, KM = 32, PAD = 8;
  __device__ static accv_t mma(const op_t* a, const op_t* b, accv_t c) {
    const v8h av = *reinterpret_cast<const v8h*>(a);
    const v8h bv = *reinterpret_cast<const v8h*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
  __device__ static int acc_row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <class T> __device__ inline T cvt(double v);
template <> __device__ inline double cvt<double>(double v) { return v; }
template <> __device__ inline float cvt<float>(double v) { return (float)v; }
template <> __device__ inline __bf16 cvt<__bf16>(double v) { return (__bf16)(float)v; }
template <> __device__ inline _Float16 cvt<_Float16>(double v) { return (_Float16)(float)v; }
template <class T> __device__ inline T cvtf(float v);
template <> __device__ inline float cvtf<float>(float v) { return v; }
template <> __device__ inline __bf16 cvtf<__bf16>(float v) { return (__bf16)v; }
template <> __device__ inline _Float16 cvtf<_Float16>(float v) { return (_Float16)v; }

enum Epi { kEpiStore = 0, kEpiEinv = 1, kEpiZ = 2 };

// The r.z partials of the last transform read the residual the transforms
// started from: FP64 r with FP64 transforms, else its GEMM-precision copy
// (the values the preconditioner was actually applied to).
__device__ inline double widen(double v) { return v; }
__device__ inline double widen(float v) { return (double)v; }
__device__ inline double widen(__bf16 v) { return (double)(float)v; }
__device__ inline double widen(_Float16 v) { return (double)(float)v; }

// Epilogue factors of the scaled (FP16) path: the scaling transform skips
// 1/a0, the last one multiplies z by 1 / (sigma E_min a0) and the r.z partial
// sum (taken against the scaled residual copy) by 1 / sigma. Unscaled paths:
// sigma = E_min = 1 and 1/a0 in the scaling transform, exactly as before.
struct EpiScale {
  double z = 1.0, dot = 1.0;
  __device__ EpiScale(int scaled, const SysState* sys, const RealState* real, int s, int r, double emin) {
    if (scaled) {
      const double sig = sys ? sys[s].lo_scale : 1.0;
      z = real[r].inv_a0 / (sig * emin);
      dot = 1.0 / sig;
    }
  }
};

// The last transform may write the next search direction instead of z (the
// driver's pdirect mode): p = z at the first apply, else
// p_{k+1} = z_{k+1} + beta_k p_k with beta_k from the system state, rounded to
// the direction type exactly as the operator apply would form it, into ring
// slot k+1 mod m (k from the iteration counter; the first apply writes slot
// k mod m). ring == nullptr: z is written as usual.
struct PDir {
  void* ring = nullptr;
  long long slot = 0;   // elements per ring slot
  int m = 1;
  const int* kiter = nullptr;
  int first = 0;
};

// Elements of one K-slice per thread: (BM x BK) / 256.
template <class Tr> struct Stage {
  static constexpr int PER = (BM * Tr::BK) / kBlock;   // 4 (FP64/FP32) or 16 (BF16)
  static constexpr int TPR = Tr::BK / PER;              // threads per row: 4
};

// D = 2: each system is n x n; D = 3: each system is an n^2 x n matrix
// (rows R = n^2) and its output (X Q)^T is n x n^2; D systems per realization.
template <class Tr, class InT, int EPI, class ZT = double, class RT = double, int D = 2>
__global__ void __launch_bounds__(kBlock) k_hartley(const InT* __restrict__ X, const typename Tr::op_t* __restrict__ Qm,
                                                     void* __restrict__ out_v, int n, int S, const SysState* sys,
                                                     const RealState* real, const void* __restrict__ einv_v,
                                                     const RT* __restrict__ rres, double* __restrict__ part,
                                                     double emin) {
  static_assert(D == 2 || D == 3, "dimension");
  constexpr int scaled = std::is_same<Tr, TrF16>::value;   // FP16: scaled operands
  using op_t = typename Tr::op_t;
  using acc_t = typename Tr::acc_t;
  using accv_t = typename Tr::accv_t;
  constexpr int BK = Tr::BK, KM = Tr::KM, LDA = BK + Tr::PAD;
  constexpr int PER = Stage<Tr>::PER, TPR = Stage<Tr>::TPR;
  constexpr int LDC = BM + 1;
  constexpr size_t kOpBytes = 2 * (size_t)BM * LDA * sizeof(op_t);
  constexpr size_t kCBytes = (size_t)BN * LDC * sizeof(acc_t);
  __shared__ __attribute__((aligned(16))) unsigned char smem[kOpBytes > kCBytes ? kOpBytes : kCBytes];
  __shared__ double red[4];
  op_t* As = reinterpret_cast<op_t*>(smem);
  op_t* Bs = As + BM * LDA;
  acc_t* Cs = reinterpret_cast<acc_t*>(smem);

  const long long R = D == 3 ? (long long)n * n : (long long)n;   // rows of X per system
  const int NB = n / BN, MB = (int)(R / BM);
  const long long T = (long long)S * MB * NB;
  long long t = blockIdx.x;
  if ((T & 7) == 0) t = (t & 7) * (T >> 3) + (t >> 3);   // XCD-contiguous tile ranges
  const int nb = (int)(t % NB);
  const long long rest = t / NB;
  const int mb = (int)(rest % MB);
  const int s = (int)(rest / MB);
  if (sys && !sys[s].active) return;

  const long long N2 = R * n;   // elements per system
  const InT* Xs = X + (long long)s * N2 + (long long)mb * BM * n;
  const op_t* Qs = Qm + (long long)nb * BN * n;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int ld_row = tid / TPR, ld_col = (tid % TPR) * PER;

  InT ra[PER];
  op_t rb[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      ra[e] = Xs[(long long)ld_row * n + k0 + ld_col + e];
      rb[e] = Qs[(long long)ld_row * n + k0 + ld_col + e];
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      if constexpr (sizeof(InT) == sizeof(op_t)) As[ld_row * LDA + ld_col + e] = (op_t)ra[e];
      else As[ld_row * LDA + ld_col + e] = cvt<op_t>((double)ra[e]);
      Bs[ld_row * LDA + ld_col + e] = rb[e];
    }
  };

  accv_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  // operand fragment base: row (l%16), contraction offset (l/16) * (KM/4)
  const int frow = lane & 15, fk = (lane >> 4) * (KM / 4);

  gload(0);
  sstore();
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += BK) {
    const bool more = k0 + BK < n;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += KM) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const op_t* pa = As + (wm * 32 + i * 16 + frow) * LDA + kk + fk;
          const op_t* pb = Bs + (wn * 32 + j * 16 + frow) * LDA + kk + fk;
          acc[i][j] = Tr::mma(pa, pb, acc[i][j]);
        }
    }
    __syncthreads();
    if (more) {
      sstore();
      __syncthreads();
    }
  }

  // accumulators -> LDS, transposed: Cs[col][row]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * 32 + i * 16 + Tr::acc_row(lane, e);
        const int col = wn * 32 + j * 16 + (lane & 15);
        Cs[col * LDC + row] = acc[i][j][e];
      }
  __syncthreads();

  // output tile: BN rows (l) of BM contiguous values (m); 4 threads per row
  const int orow = tid >> 2, oc0 = (tid & 3) * 16;
  const long long obase = (long long)s * N2 + (long long)(nb * BN + orow) * R + mb * BM + oc0;
  double dot = 0.0;
  acc_t scale = (acc_t)1;
  const int rz = D == 2 ? (s >> 1) : s / 3;
  if constexpr (EPI == kEpiEinv) scale = scaled ? (acc_t)1 : (acc_t)real[rz].inv_a0;
  const EpiScale es(EPI == kEpiZ ? scaled : 0, sys, real, s, rz, emin);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acc_t v = Cs[orow * LDC + oc0 + e];
    if constexpr (EPI == kEpiEinv) {
      const acc_t* einv = reinterpret_cast<const acc_t*>(einv_v);
      v = v * einv[(long long)(nb * BN + orow) * R + mb * BM + oc0 + e] * scale;
    }
    if constexpr (EPI == kEpiZ) {
      ZT* out = reinterpret_cast<ZT*>(out_v);
      ZT zs;
      if constexpr (scaled) zs = (ZT)((double)v * es.z);
      else zs = (ZT)v;
      out[obase + e] = zs;
      dot += (double)zs * widen(rres[obase + e]);
    } else {
      op_t* out = reinterpret_cast<op_t*>(out_v);
      if constexpr (sizeof(acc_t) == sizeof(op_t)) out[obase + e] = (op_t)v;
      else out[obase + e] = cvtf<op_t>(v);
    }
  }
  if constexpr (EPI == kEpiZ) {
    double d[1] = {dot};
    block_sum<1>(d, red);
    if (tid == 0) part[(long long)s * ((long long)MB * NB) + (long long)mb * NB + nb] = scaled ? d[0] * es.dot : d[0];
  }
}

// 16-bit transform GEMM (BF16 or FP16 operands, FP32 accumulation) with a
// 128 x 128 output tile (n % 128 == 0): 2 x 2 waves of 64 x 64, i.e. 4 x 4
// MFMA 16x16x32 blocks per wave, so each operand fragment read from LDS
// feeds four MFMAs. Two operand pipelines (PIPE):
//   0: 64-wide K slices (operand tiles 128 x 64, row stride 144 B:
//      conflict-free 16-byte fragment reads) loaded with 16-byte global
//      loads, the next slice prefetched into registers while the current
//      one feeds the MFMAs; two barriers per slice.
//   1: 32-wide K slices loaded by the load unit straight into LDS
//      (global_load_lds, 16 bytes per lane), double-buffered: the next
//      slice is in flight while the current one feeds the MFMAs; one
//      barrier per slice and no staging registers. One load instruction of
//      a wave fills 1 KB of LDS contiguously (lane l at byte 16 l), so the
//      tile cannot be padded; instead the four 16-byte chunks of each
//      64-byte row are XOR-swizzled by (row / 2) mod 4, which keeps the
//      fragment reads conflict-free.
// Both accumulate over k in the same order (ascending 32-wide MFMA steps),
// so they give identical outputs. The output (transposed) is stored straight
// from the accumulators: each lane holds four consecutive output columns of
// one output row per MFMA block; for 16-bit output lanes 16 apart swap half
// of each block pair, so a wave's store covers 16 rows x 64 bytes (as the
// FP32 z does with four values per lane), and no LDS round trip or barrier
// is needed.
// Three waves per SIMD (142 VGPRs with PIPE 0) hide more of the load latency
// than two; four with 32-wide register-staged slices measured slower.
constexpr int TM = 128, TN = 128, TK = 64, TLDA = TK + 8, TLDC = TM + 4;
constexpr int DK = 32;   // K slice of the LDS-DMA pipeline

template <class T> struct H16;
template <> struct H16<__bf16> {
  typedef v8bf v8;
  __device__ static v4f mma(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <> struct H16<_Float16> {
  typedef v8h v8;
  __device__ static v4f mma(v8h a, v8h b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// 16 bytes per lane from global memory into LDS at lds_wave + 16 * lane
// (lds_wave must be the same in every lane of the wave).
template <class T>
__device__ inline void lds_dma16(const T* src, T* lds_wave) {
  typedef __attribute__((address_space(3))) void lds_void;
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void*)lds_wave, 16, 0, 0);
}

// One 32-wide K step of a wave's 4 x 4 MFMA blocks: the eight fragment
// reads (rd(0, i): A rows 16 i.., rd(1, j): B rows 16 j..) are all issued
// before the first MFMA, and a scheduling barrier keeps them there; left to
// itself the compiler reused one register set for the A fragments and waited
// for each read in turn, exposing the LDS latency four times per step.
// GROUPED = false (for the register-tight 256 x 128 tile) reads the A
// fragments one at a time, 16 fewer live registers.
// BI (4 or 8) is the wave's count of 16-row A blocks; grouped reads go four
// A fragments at a time.
template <class T, bool GROUPED = true, int BI = 4, class RD>
__device__ inline void h16_kstep(v4f (&acc)[BI][4], RD rd) {
  typedef typename H16<T>::v8 v8t;
  v8t bf[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bf[j] = rd(1, j);
  if constexpr (GROUPED) {
#pragma unroll
    for (int g = 0; g < BI; g += 4) {
      v8t af[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = rd(0, g + i);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[g + i][j] = H16<T>::mma(af[i], bf[j], acc[g + i][j]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      const v8t af = rd(0, i);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = H16<T>::mma(af, bf[j], acc[i][j]);
    }
  }
}

// WMR is the number of wave rows (64 rows each, 128 with BI = 8): 2 (128 x
// 128 tile, 256 threads,
// three waves per SIMD) or 4 (256 x 128 tile, 512 threads, four waves per
// SIMD, PIPE 0 only): the taller tile loads a quarter fewer operand bytes per
// output, which is what the load path of this kernel is short of. At 128
// VGPRs it reads the A fragments one at a time; the EPI 1 epilogue, and the
// EPI 2 one with the scaled FP16 operands, spill there, so those transforms
// stay at WMR = 2.
// WNR is the number of 64-column wave columns: 2, or 4 with WMR = 4 (a
// 256 x 256 tile, 1024 threads: a third fewer operand bytes per output
// than 256 x 128).
// BI = 8 (with WMR = 2, WNR = 4) gives each wave 128 rows instead of 64: the
// same 256 x 256 tile from 8 waves at two per SIMD, a quarter fewer LDS
// fragment reads per K slice than 16 waves of 64 x 64, and the registers
// for grouped reads.
template <class T, int EPI, class ZT, int PIPE = 0, int WMR = 2, int WNR = 2, int BI = 4>
__global__ void __launch_bounds__(64 * WMR * WNR)
__attribute__((amdgpu_waves_per_eu(BI == 8 ? 2 : WMR * WNR == 4 ? 3 : 4, BI == 8 ? 2 : WMR * WNR == 4 ? 3 : 4)))
k_hartley_h16(const T* __restrict__ X, const T* __restrict__ Qm, void* __restrict__ out_v, int n, int S,
              const SysState* sys, const RealState* real, const float* __restrict__ sin2,
              double* __restrict__ part, double emin, int fd, PDir pd) {
  static_assert(PIPE == 0 || PIPE == 1 || PIPE == 2, "operand pipeline");
  static_assert((BI == 4 && ((WMR == 2 && WNR == 2) || (WMR == 4 && (WNR == 2 || WNR == 4) && PIPE == 0))) ||
                    (BI == 8 && WMR == 2 && WNR == 4 && (PIPE == 0 || PIPE == 2)),
                "tile shape");
  static_assert(PIPE != 2 || BI == 8, "the four-stage ring is built for the 8-wave 256 x 256 tile");
  typedef typename H16<T>::v8 v8t;
  constexpr int scaled = std::is_same<T, _Float16>::value;   // FP16: scaled operands
  constexpr int WR = 16 * BI;   // rows of a wave's block
  constexpr int TMR = WR * WMR, TNR = 64 * WNR, NTH = 64 * WMR * WNR, NW = WMR * WNR;
  constexpr bool T256 = PIPE == 0 && TMR == 256 && TNR == 256;
  // the 256 x 256 tile stages its operands in two LDS buffers (147 KB): the
  // next slice is stored while other waves still read the current one, one
  // barrier per K slice instead of two; the smaller tiles keep one buffer
  // (two would cost them a workgroup per CU)
  constexpr int NSTG = T256 ? 2 : 1;
  constexpr size_t kStage = (size_t)(TMR + TNR) * TLDA;
  // operands loaded straight into LDS (PIPE 1, 2): a ring of NRING stages
  // of 32-wide K slices
  constexpr int NRING = PIPE == 2 ? 4 : 2;
  constexpr size_t kSmem =
      PIPE == 0 ? NSTG * kStage * sizeof(T) : (size_t)NRING * (TMR + TNR) * DK * sizeof(T);
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
  T* As = reinterpret_cast<T*>(smem);

  // Tiles of this workgroup: local indices li, li + lstep, ... below lend,
  // counted from tile base. With NT and the grid multiples of 8, workgroup b
  // (on XCD b % 8) takes tiles from range b % 8 of eight contiguous ones, so
  // the tiles that share operand rows meet in one XCD's L2. One workgroup
  // per tile (the grid must then cover every tile), except the plain
  // transform in 256 x 256 tiles (PERS): there the grid may be smaller (one
  // workgroup per CU), and each workgroup loads the first K slice of its
  // next tile while it computes the last slice of this one and stores its
  // outputs. The scaling transform does so too in the 8-wave shape, which
  // has the registers for it; in the 16-wave one its epilogue spilled under
  // the loop, and the last transform gained nothing from it in either.
  constexpr bool PERS = T256 && (EPI == kEpiStore || (EPI == kEpiEinv && BI == 8));
  const int NB = n / TNR, MB = n / TMR;
  const long long NT = (long long)S * MB * NB, N2 = (long long)n * n;
  long long base = 0, li = blockIdx.x, lend = NT, lstep = gridDim.x;
  if ((NT & 7) == 0 && (gridDim.x & 7) == 0) {
    base = (long long)(blockIdx.x & 7) * (NT >> 3);
    li = blockIdx.x >> 3;
    lend = NT >> 3;
    lstep = gridDim.x >> 3;
  }
  // first local index at or after l whose system is active (lend if none)
  auto seek = [&](long long l) {
    while (l < lend && sys && !sys[(base + l) / ((long long)MB * NB)].active) l += lstep;
    return l;
  };

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WNR, wn = w % WNR;
  const int frow = lane & 15;

  constexpr int TPR = TK / 8;                 // threads per staged row (8 elements each)
  constexpr int RPP = NTH / TPR;              // rows per staging pass: 8 / WNR passes
                                              // for A, 8 / WMR for B (4 or 2)
  constexpr int PA = TMR / RPP, PB = TNR / RPP;
  static_assert(PIPE == 1 || ((PA == 2 || PA == 4) && (PB == 2 || PB == 4)), "staging passes");
  const int lr = tid / TPR, lc = (tid % TPR) * 8;
  const int loff = lr * n + lc;   // (lr < 128 and n <= 4096: well inside 32 bits)
  const long long rstep = (long long)RPP * n;
  // register staging of the next K slice in named registers (plain code:
  // arrays or lambdas put it in scratch)
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define RVE_GLOAD(xp, qp, k0)                                         \
  do {                                                                \
    ra0 = *reinterpret_cast<const uint4*>((xp) + (k0));               \
    ra1 = *reinterpret_cast<const uint4*>((xp) + rstep + (k0));       \
    if constexpr (PA == 4) {                                          \
      ra2 = *reinterpret_cast<const uint4*>((xp) + 2 * rstep + (k0)); \
      ra3 = *reinterpret_cast<const uint4*>((xp) + 3 * rstep + (k0)); \
    }                                                                 \
    rb0 = *reinterpret_cast<const uint4*>((qp) + (k0));               \
    rb1 = *reinterpret_cast<const uint4*>((qp) + rstep + (k0));       \
    if constexpr (PB == 4) {                                          \
      rb2 = *reinterpret_cast<const uint4*>((qp) + 2 * rstep + (k0)); \
      rb3 = *reinterpret_cast<const uint4*>((qp) + 3 * rstep + (k0)); \
    }                                                                 \
  } while (0)
#define RVE_SSTORE(Ad)                                                \
  do {                                                                \
    T* const Bd = (Ad) + TMR * TLDA;                                  \
    *reinterpret_cast<uint4*>((Ad) + lr * TLDA + lc) = ra0;           \
    *reinterpret_cast<uint4*>((Ad) + (lr + RPP) * TLDA + lc) = ra1;   \
    if constexpr (PA == 4) {                                          \
      *reinterpret_cast<uint4*>((Ad) + (lr + 2 * RPP) * TLDA + lc) = ra2; \
      *reinterpret_cast<uint4*>((Ad) + (lr + 3 * RPP) * TLDA + lc) = ra3; \
    }                                                                 \
    *reinterpret_cast<uint4*>(Bd + lr * TLDA + lc) = rb0;             \
    *reinterpret_cast<uint4*>(Bd + (lr + RPP) * TLDA + lc) = rb1;     \
    if constexpr (PB == 4) {                                          \
      *reinterpret_cast<uint4*>(Bd + (lr + 2 * RPP) * TLDA + lc) = rb2; \
      *reinterpret_cast<uint4*>(Bd + (lr + 3 * RPP) * TLDA + lc) = rb3; \
    }                                                                 \
  } while (0)

  bool pref = false;   // the first K slice of the tile is already in LDS
  int cur = 0;         // operand buffer of the current K slice (two stages)
  for (li = seek(li); li < lend;) {
    const long long t = base + li;
    const int nb = (int)(t % NB);
    const long long rest = t / NB;
    const int mb = (int)(rest % MB);
    const int s = (int)(rest / MB);
    const long long lnext = PERS ? seek(li + lstep) : lend;
    const T* Xs = X + (long long)s * N2 + (long long)mb * TMR * n;
    const T* Qs = Qm + (long long)nb * TNR * n;

    v4f acc[BI][4];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.f;

    if constexpr (PIPE == 0) {
      // (the empty asm keeps the per-lane offset out of the loop-invariant
      // addresses the compiler would hoist out of the tile loop and spill)
      int lo = loff;
      if constexpr (PERS) asm volatile("" : "+v"(lo));
      const T* xa = Xs + lo;
      const T* qa = Qs + lo;
      const int fk = (lane >> 4) * 8;
      if (!pref) {
        RVE_GLOAD(xa, qa, 0);
        RVE_SSTORE(As + cur * kStage);
      }
      __syncthreads();
      for (int k0 = 0; k0 < n; k0 += TK) {
        const bool more = k0 + TK < n;
        // last slice: load the first slice of the next tile instead (stored
        // to the free buffer like any other, before the epilogue)
        const bool ahead = PERS && !more && lnext < lend;
        if (more) {
          RVE_GLOAD(xa, qa, k0 + TK);
        } else if constexpr (PERS) {
          if (ahead) {
            // (the empty asm keeps the next tile's addresses here, out of
            // the registers live across the loop)
            int lo = loff;
            asm volatile("" : "+v"(lo));
            const long long tn = base + lnext, rn = tn / NB;
            const T* xn = X + (rn / MB) * N2 + (rn % MB) * TMR * n + lo;
            const T* qn = Qm + (tn % NB) * TNR * n + lo;
            RVE_GLOAD(xn, qn, 0);
          }
        }
        const T* Ab = As + cur * kStage;
        const T* Bb = Ab + TMR * TLDA;
#pragma unroll
        for (int kk = 0; kk < TK; kk += 32)
          h16_kstep<T, NW == 4 || BI == 8, BI>(acc, [&](int isb, int q) {
            const T* row = isb ? Bb + (wn * 64 + q * 16 + frow) * TLDA : Ab + (wm * WR + q * 16 + frow) * TLDA;
            return *reinterpret_cast<const v8t*>(row + kk + fk);
          });
        if constexpr (NSTG == 2) {
          // the other buffer was last read before the previous barrier
          if (more || ahead) RVE_SSTORE(As + (cur ^ 1) * kStage);
          __syncthreads();
          cur ^= 1;
        } else {
          __syncthreads();
          if (more) {
            RVE_SSTORE(As);
            __syncthreads();
          }
        }
      }
      pref = PERS && lnext < lend;   // (already in buffer cur)
    } else {
      // stage b holds the A tile (TMR x 32) then the B tile (TNR x 32);
      // 16-byte chunk g of a tile sits at LDS chunk g and holds row g / 4, K
      // chunk (g % 4) ^ ((row / 2) % 4). Lane l of wave w loads chunks
      // 128 w + l and 128 w + 64 + l of both tiles (4 waves: 128 rows,
      // 8 waves: 256 rows), four load instructions per wave and slice.
      constexpr int kA = TMR * DK, kBuf = (TMR + TNR) * DK;
      const int g0 = 128 * w + lane, g1 = g0 + 64;
      const int r0 = g0 >> 2, r1 = g1 >> 2;
      const int c0 = (g0 & 3) ^ ((r0 >> 1) & 3), c1 = (g1 & 3) ^ ((r1 >> 1) & 3);
      const T* xa0 = Xs + (long long)r0 * n + 8 * c0;
      const T* xa1 = Xs + (long long)r1 * n + 8 * c1;
      const T* qa0 = Qs + (long long)r0 * n + 8 * c0;
      const T* qa1 = Qs + (long long)r1 * n + 8 * c1;
      auto issue = [&](int b, int k0) {
        T* base = As + b * kBuf + 1024 * w;
        lds_dma16(xa0 + k0, base);
        lds_dma16(xa1 + k0, base + 512);
        lds_dma16(qa0 + k0, base + kA);
        lds_dma16(qa1 + k0, base + kA + 512);
      };
      // fragment reads: row (.. + frow), K chunk lane / 16 of the slice
      const int fc = (lane >> 4) ^ ((frow >> 1) & 3);
      const int nk = n / DK;
      for (int k = 0; k < NRING - 1 && k < nk; ++k) issue(k, k * DK);
      for (int ks = 0; ks < nk; ++ks) {
        // this wave's loads of slice ks have landed (loads complete in the
        // order they were issued: waiting until at most the four loads of
        // each later slice still in flight remain) and its reads of slice
        // ks - 1 are done; after the barrier the same holds for every wave,
        // so slice ks is complete and the stage of slice ks - 1 is free for
        // slice ks + NRING - 1
        const int ahead = NRING - 2 < nk - 1 - ks ? NRING - 2 : nk - 1 - ks;
        if (ahead >= 2)
          asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        else if (ahead == 1)
          asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        else
          asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (ks + NRING - 1 < nk) issue((ks + NRING - 1) % NRING, (ks + NRING - 1) * DK);
        const T* Ab = As + (ks % NRING) * kBuf;
        const T* Bb = Ab + kA;
        h16_kstep<T, true, BI>(acc, [&](int isb, int q) {
          const T* row = isb ? Bb + (wn * 64 + q * 16 + frow) * DK : Ab + (wm * WR + q * 16 + frow) * DK;
          return *reinterpret_cast<const v8t*>(row + fc * 8);
        });
      }
    }

    // EPI 1 scales output (l, m) by f / E(l, m), E formed from s_k =
    // sin^2(pi k / n) (no cancellation near the zero mode): the Q1 symbol
    // (8 - 2c_l - 2c_m - 4 c_l c_m)/3 = 4 (s_l + s_m) - (16/3) s_l s_m, the
    // five-point one (2 - 2c_l) + (2 - 2c_m) = 4 (s_l + s_m); E(0, 0) = 0 gives
    // 0 (the pseudo-inverse). f = 1/a0, or E_min for the scaled FP16 operands.
    // It also forms the r.z partials: its input X = (R Q)^T, so its product
    // X Q is the two-dimensional transform R^ = Q R Q of the residual copy R,
    // its output U = R^ ./ (a0 E) (as stored), and z = Q U Q; since Q is
    // symmetric and orthogonal, r.z = sum R^ .* U (FP64 sum). With the scaled
    // FP16 operands R = sigma r and U = R^ E_min / E, so the sum is multiplied
    // by 1 / (sigma^2 E_min a0).
    float fscale = 1.f, cq = 0.f;
    double dfac = 1.0;
    if constexpr (EPI == kEpiEinv) {
      fscale = scaled ? (float)emin : (float)real[s >> 1].inv_a0;
      cq = fd ? 0.f : 16.f / 3.f;
      if constexpr (scaled) {
        const double sig = sys ? sys[s].lo_scale : 1.0;
        dfac = real[s >> 1].inv_a0 / (sig * sig * emin);
      }
    }
    const EpiScale es(EPI == kEpiZ ? scaled : 0, sys, real, s, s >> 1, emin);
    // pdirect: where this tile's direction goes, and the old one
    ZT* pnew = nullptr;
    const ZT* pold = nullptr;
    double pbeta = 0.0;
    if constexpr (EPI == kEpiZ) {
      if (pd.ring) {
        const int kk = pd.kiter[0];
        ZT* ring = reinterpret_cast<ZT*>(pd.ring);
        pnew = ring + (long long)((pd.first ? kk : kk + 1) % pd.m) * pd.slot;
        if (!pd.first) {
          pold = ring + (long long)(kk % pd.m) * pd.slot;
          pbeta = sys[s].beta;
        }
      }
    }
    // r.z partials per 64 x 64 output block (a wave's block, or each half of
    // the 128-row block with BI = 8), accumulated per lane in the same order
    // (j, then i, then e) in every tile shape: the partials do not depend on
    // the tile variant
    double dot[BI / 4];
#pragma unroll
    for (int hh = 0; hh < BI / 4; ++hh) dot[hh] = 0.0;
    // straight from the accumulators: block (i, j) of lane l holds output
    // row nb TNR + 64 wn + 16 j + l % 16 at the four consecutive columns
    // mb TMR + WR wm + 16 i + 4 (l / 16) + e
    const int lr = lane & 15, m4 = 4 * (lane >> 4);
    if constexpr (EPI == kEpiZ) {
      // z of block (i, j) (scaled FP16 operands: times 1 / (sigma E_min a0))
      // rounded to its type, plus beta_k p_k when this transform forms the
      // next direction
      ZT* const zo = pnew ? pnew : reinterpret_cast<ZT*>(out_v);
      auto zoff = [&](int i, int j) {
        return (long long)s * N2 + ((long long)nb * TNR + wn * 64 + j * 16 + lr) * n +
               (long long)mb * TMR + wm * WR + i * 16 + m4;
      };
      const ZT kNoP[4] = {0, 0, 0, 0};
      // BF16 directions: p = z + beta p_k of block (i, j) in FP64, rounded
      // to FP32, then to BF16 (the empty asm keeps the two roundings apart:
      // left free, the compiler merged them into one for some elements and
      // not others, differently per tile shape), as two words
      typedef unsigned u2 __attribute__((ext_vector_type(2)));
      typedef unsigned u4 __attribute__((ext_vector_type(4)));
      struct alignas(8) Z4 { ZT e[4]; };
      auto pbits = [&](int i, int j, bool with_p, const ZT (&po)[4]) {
        u2 bits = {0u, 0u};
        if constexpr (sizeof(ZT) == 2) {
          Z4 st;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double zd = scaled ? (double)acc[i][j][e] * es.z : (double)acc[i][j][e];
            float f = (float)(with_p ? fma(pbeta, (double)po[e], zd) : zd);
            asm("" : "+v"(f));
            st.e[e] = (ZT)f;
          }
          bits = __builtin_bit_cast(u2, st);
        }
        return bits;
      };
      // BF16 directions, blocks i and i + 1 of block row j stored together,
      // 16 bytes per lane (lanes 16 apart swap half their words, as in the
      // 16-bit transforms' epilogue: 64 contiguous bytes per row and store)
      auto ppair = [&](int i, int j, bool with_p, const ZT (&pa)[4], const ZT (&pb)[4]) {
        const bool odd = (lane >> 4) & 1;
        const u2 a = pbits(i, j, with_p, pa), b = pbits(i + 1, j, with_p, pb);
        const u2 send = odd ? a : b;
        u2 got;
        got.x = __shfl_xor(send.x, 16, kWave);
        got.y = __shfl_xor(send.y, 16, kWave);
        u4 o4;
        o4.x = odd ? got.x : a.x;
        o4.y = odd ? got.y : a.y;
        o4.z = odd ? b.x : got.x;
        o4.w = odd ? b.y : got.y;
        *reinterpret_cast<u4*>(zo + (zoff(i, j) - m4 + (odd ? 16 : 0) + 8 * (lane >> 5))) = o4;
      };
      auto zput = [&](int i, int j, bool with_p, const ZT (&po)[4]) {
        const long long o = zoff(i, j);
        if constexpr (sizeof(ZT) == 2) {
          *reinterpret_cast<u2*>(zo + o) = pbits(i, j, with_p, po);
          return;
        }
        ZT zs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (scaled) zs[e] = (ZT)((double)acc[i][j][e] * es.z);
          else zs[e] = (ZT)acc[i][j][e];
        }
        if (with_p) {
#pragma unroll
          for (int e = 0; e < 4; ++e) zs[e] = (ZT)fma(pbeta, (double)po[e], (double)zs[e]);
        }
        if constexpr (sizeof(ZT) == 4) {
          float4 st;
          st.x = zs[0]; st.y = zs[1]; st.z = zs[2]; st.w = zs[3];
          *reinterpret_cast<float4*>(zo + o) = st;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) zo[o + e] = zs[e];
        }
      };
      // (the scaled FP16 path in the 16-wave tile keeps one p_k load per
      // block: at 128 registers the row form spills)
      constexpr bool kRows = (sizeof(ZT) == 4 || sizeof(ZT) == 2) && !(scaled && NW == 16);
      // four values of p_k in one load: 16 bytes (FP32) or 8 (BF16)
      using P4 = typename std::conditional<sizeof(ZT) == 4, float4, uint2>::type;
      auto p4dec = [](const P4& v, ZT (&o)[4]) {
        if constexpr (sizeof(ZT) == 4) {
          o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
        } else {
          struct Z4 { ZT e[4]; };
          const Z4 t = __builtin_bit_cast(Z4, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = t.e[e];
        }
      };
      if constexpr (kRows) {
        if (pold) {
          // p_k is loaded a block row at a time (one branch for the whole
          // epilogue), and where the registers allow, row j + 1 before the
          // stores of row j: a wait for loads issued after a store waits for
          // the store too (one in-order counter). Loaded block by block, each
          // block was a full round trip. (The scaled FP16 path, with its FP64
          // products, would spill with two rows of p_k in flight.)
          constexpr bool kAhead = !scaled;
          P4 po[2][BI];
          auto fetch = [&](int j, P4 (&dst)[BI]) {
            if constexpr (sizeof(ZT) == 2) {
              // BF16: 16 bytes per lane at the position the pair store
              // writes (64 contiguous bytes per row), lane halves swapped
              // back when the row is used (pget)
              const bool odd = (lane >> 4) & 1;
#pragma unroll
              for (int i = 0; i < BI; i += 2) {
                const u4 v = *reinterpret_cast<const u4*>(pold + (zoff(i, j) - m4 + (odd ? 16 : 0) + 8 * (lane >> 5)));
                dst[i] = P4{v.x, v.y};
                dst[i + 1] = P4{v.z, v.w};
              }
            } else {
#pragma unroll
              for (int i = 0; i < BI; ++i) dst[i] = *reinterpret_cast<const P4*>(pold + zoff(i, j));
            }
          };
          // BF16: this lane's values of blocks i and i + 1 from a pair load
          // (even lanes hold their own block-i values and their partner's,
          // odd lanes their partner's block-(i + 1) values and their own)
          auto pget = [&](const P4& lo, const P4& hi, ZT (&pa)[4], ZT (&pb)[4]) {
            const bool odd = (lane >> 4) & 1;
            const P4 send = odd ? lo : hi;
            P4 got;
            got.x = __shfl_xor(send.x, 16, kWave);
            got.y = __shfl_xor(send.y, 16, kWave);
            p4dec(odd ? got : lo, pa);
            p4dec(odd ? hi : got, pb);
          };
          if constexpr (kAhead) fetch(0, po[0]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            // (one block row at a time: hoisting the next rows' address and
            // FP64 work spills the tighter tiles)
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kAhead) {
              if (j + 1 < 4) fetch(j + 1, po[(j + 1) & 1]);
            } else {
              fetch(j, po[j & 1]);
            }
            if constexpr (sizeof(ZT) == 2) {
#pragma unroll
              for (int i = 0; i < BI; i += 2) {
                ZT pa[4], pb[4];
                pget(po[j & 1][i], po[j & 1][i + 1], pa, pb);
                ppair(i, j, true, pa, pb);
              }
            } else {
#pragma unroll
              for (int i = 0; i < BI; ++i) {
                ZT pk4[4];
                p4dec(po[j & 1][i], pk4);
                zput(i, j, true, pk4);
              }
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (sizeof(ZT) == 2) {
#pragma unroll
              for (int i = 0; i < BI; i += 2) ppair(i, j, false, kNoP, kNoP);
            } else {
#pragma unroll
              for (int i = 0; i < BI; ++i) zput(i, j, false, kNoP);
            }
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < BI; ++i) {
            ZT pk4[4] = {0, 0, 0, 0};
            if (pold) {
              if constexpr (sizeof(ZT) == 4) {
                const float4 pv = *reinterpret_cast<const float4*>(pold + zoff(i, j));
                pk4[0] = pv.x; pk4[1] = pv.y; pk4[2] = pv.z; pk4[3] = pv.w;
              } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) pk4[e] = pold[zoff(i, j) + e];
              }
            }
            zput(i, j, pold != nullptr, pk4);
          }
      }
    }
    // The scaling transform's symbol values depend on the output row (one
    // per block row j) and on the four output columns of block i. The 8-wave
    // tiles load all of them before the first store: loaded per block, each
    // block pair waited for its loads and with them (one in-order counter)
    // for the previous pair's store.
    constexpr bool kPreSym = EPI == kEpiEinv && BI == 8;
    float sl_pre[kPreSym ? 4 : 1];
    float4 sm_pre[kPreSym ? BI : 1];
    if constexpr (kPreSym) {
#pragma unroll
      for (int j = 0; j < 4; ++j) sl_pre[j] = sin2[nb * TNR + wn * 64 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < BI; ++i) sm_pre[i] = *reinterpret_cast<const float4*>(sin2 + mb * TMR + wm * WR + i * 16 + m4);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // (the 16-wave tile has no registers to spare for hoisting every block's
      // loads of the scaling epilogue to the top)
      if constexpr (EPI == kEpiEinv && NW == 16) __builtin_amdgcn_sched_barrier(0);
      const long long l = (long long)nb * TNR + wn * 64 + j * 16 + lr;
      if constexpr (EPI != kEpiZ) {
        // 16-bit output of block (i, j), rounded (and scaled by f / E in the
        // scaling transform, which adds its products to the r.z partial), as
        // two words. The empty asm pins the rounded bits: every later use
        // (store, lane swap, r.z product) reads them, so the compiler cannot
        // redo a conversion with another instruction sequence, and every tile
        // shape stores the same bits.
        typedef T v4t __attribute__((ext_vector_type(4)));
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        auto block = [&](int i) {
          const long long m = (long long)mb * TMR + wm * WR + i * 16 + m4;
          const float r[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
          float v[4] = {r[0], r[1], r[2], r[3]};
          if constexpr (EPI == kEpiEinv) {
            float sl;
            float4 sm4;
            if constexpr (kPreSym) {
              sl = sl_pre[j];
              sm4 = sm_pre[i];
            } else {
              sl = sin2[l];
              sm4 = *reinterpret_cast<const float4*>(sin2 + m);
            }
            const float sm[4] = {sm4.x, sm4.y, sm4.z, sm4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float E = 4.f * (sl + sm[e]) - cq * sl * sm[e];
              v[e] *= E > 0.f ? fscale * __builtin_amdgcn_rcpf(E) : 0.f;
            }
            // (the scaled values are rounded to FP32 before the conversion:
            // left free, the compiler fuses some of the FP16 multiplies and
            // conversions into one rounding and not others, differently in
            // each tile shape)
            asm("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
          }
          v4t pk;
#pragma unroll
          for (int e = 0; e < 4; ++e) pk[e] = (T)v[e];
          u2 bits = __builtin_bit_cast(u2, pk);
          asm("" : "+v"(bits));
          if constexpr (EPI == kEpiEinv) {
            const v4t q = __builtin_bit_cast(v4t, bits);
#pragma unroll
            for (int e = 0; e < 4; ++e) dot[i >> 2] += (double)r[e] * (double)(float)q[e];
          }
          return bits;
        };
        // Blocks i and i + 1 are stored together, 16 bytes per lane: lane
        // group g = lane / 16 holds four values of block i at column offset
        // 4 g and four of block i + 1 at 16 + 4 g. Even groups swap their
        // block-(i + 1) values for the block-i values of the odd group above
        // (lane + 16), so group 0 stores columns 0-7 of block i, group 2
        // columns 8-15, group 1 columns 16-23 (block i + 1) and group 3
        // 24-31: each row gets 64 contiguous bytes per instruction, which
        // the memory system writes about 1.5 times faster than the 32-byte
        // pieces of 8-byte stores (measured with the same tile pattern).
        const bool odd = (lane >> 4) & 1;
#pragma unroll
        for (int i = 0; i < BI; i += 2) {
          // (keeps each pair's symbol loads with the pair in the scaling
          // transform, whose tall tiles otherwise spill)
          if constexpr (EPI == kEpiEinv) __builtin_amdgcn_sched_barrier(0);
          const u2 a = block(i);
          const u2 b = block(i + 1);
          const u2 send = odd ? a : b;
          u2 got;
          got.x = __shfl_xor(send.x, 16, kWave);
          got.y = __shfl_xor(send.y, 16, kWave);
          // words 0-1: the lower four columns, 2-3: the upper four
          u4 o4;
          o4.x = odd ? got.x : a.x;
          o4.y = odd ? got.y : a.y;
          o4.z = odd ? b.x : got.x;
          o4.w = odd ? b.y : got.y;
          const long long m = (long long)mb * TMR + wm * WR + i * 16 + (odd ? 16 : 0) + 8 * (lane >> 5);
          *reinterpret_cast<u4*>(reinterpret_cast<T*>(out_v) + (long long)s * N2 + l * n + m) = o4;
        }
      }
    }
    if constexpr (EPI == kEpiEinv) {
      // one wave sum per 64 x 64 block, stored at [s][l block][m block]
      const int nbl = n >> 6;
#pragma unroll
      for (int hh = 0; hh < BI / 4; ++hh) {
        const double d = wave_sum(dot[hh]);
        if (lane == 0) {
          const int lblk = (nb * TNR + wn * 64) >> 6, mblk = (mb * TMR + wm * WR + hh * 64) >> 6;
          part[(long long)s * nbl * nbl + (long long)lblk * nbl + mblk] = d * dfac;
        }
      }
    }
    li = lnext;
  }
#undef RVE_GLOAD
#undef RVE_SSTORE
}

// Even/odd-folded BF16 transform (n % 256 == 0), half the MFMA work of
// k_hartley_bf16 for the same output. Q = c + s with
// c[t][k] = cos(2 pi t k / n)/sqrt(n) even and s[t][k] = sin(2 pi t k / n)/sqrt(n)
// odd under t -> n - t and under k -> n - k. For 0 <= k < n/2 and h = n/2:
//   C[r][k] = sum_{t<h} Xe[r][t] c[t][k] + (-1)^k X[r][h]/sqrt(n),
//   S[r][k] = sum_{t<h} Xo[r][t] s[t][k],
// with Xe[t] = X[t] + X[n-t], Xo[t] = X[t] - X[n-t] for t >= 1, Xe[0] = X[0],
// Xo[0] = 0; then (X Q)[r][k] = C + S and (X Q)[r][n-k] = C - S. The one
// output row these miss, (X Q)[r][h] = sum_j (-1)^j X[r][j]/sqrt(n), is the
// alternating sum of the folded operand plus (-1)^h X[r][h], accumulated by
// the tiles of the first column block while they fold. The folded operand
// is rounded to BF16 once more than the plain transform's input.
// Tile: 128 rows r x 128 columns k < h, two accumulator sets (C and S) per
// wave, operand tiles Xe, Xo, c, s of 128 x 32 BF16 in LDS; the epilogue
// writes output rows k and n - k transposed through LDS (as the 64 x 64
// kernel does).
constexpr int SK = 32, SLDA = SK + 8;   // K slice and operand row stride of the folded kernel

template <int EPI, class ZT, class RT = double>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_hartley_bf16_sym(const __bf16* __restrict__ X, const __bf16* __restrict__ Ch, const __bf16* __restrict__ Sh,
                   void* __restrict__ out_v, int n, int S, const SysState* sys, const RealState* real,
                   const float* __restrict__ einv, const RT* __restrict__ rres, double* __restrict__ part) {
  constexpr int kOp = TM * SLDA;   // elements of one operand tile
  constexpr size_t kOpBytes = 4 * (size_t)kOp * sizeof(__bf16);
  constexpr size_t kCBytes = 2 * (size_t)64 * TLDC * sizeof(float);
  __shared__ __attribute__((aligned(16))) unsigned char smem[kOpBytes > kCBytes ? kOpBytes : kCBytes];
  __shared__ float hrow[TM];
  __shared__ double red[4];
  __bf16* Ae = reinterpret_cast<__bf16*>(smem);
  __bf16* Ao = Ae + kOp;
  __bf16* Bc = Ao + kOp;
  __bf16* Bsn = Bc + kOp;
  float* Cp = reinterpret_cast<float*>(smem);
  float* Cm = Cp + 64 * TLDC;

  const int h = n / 2;
  const int NB = h / TN, MB = n / TM;
  const long long T = (long long)S * MB * NB;
  long long tt = blockIdx.x;
  if ((T & 7) == 0) tt = (tt & 7) * (T >> 3) + (tt >> 3);   // XCD-contiguous tile ranges
  const int nb = (int)(tt % NB);
  const long long rest = tt / NB;
  const int mb = (int)(rest % MB);
  const int s = (int)(rest / MB);
  if (sys && !sys[s].active) return;

  const long long N2 = (long long)n * n;
  const __bf16* Xs = X + (long long)s * N2 + (long long)mb * TM * n;
  const __bf16* Cq = Ch + (long long)nb * TN * h;
  const __bf16* Sq = Sh + (long long)nb * TN * h;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lr = tid >> 2, lc = (tid & 3) * 8;   // rows lr and lr + 64, 8 values each
  const float isq = (float)(1.0 / sqrt((double)n));
  if (tid < TM) hrow[tid] = (float)Xs[(long long)tid * n + h] * isq;   // read after the first barrier

  // register staging of the next K slice: forward and mirrored row chunks of
  // X (the mirrored chunk [n-t0-8, n-t0) plus the single value X[n-t0]) and
  // the c / s table rows
  uint4 fa0, fa1, ma0, ma1, rc0, rc1, rs0, rs1;
  __bf16 ea0, ea1;
  float alt0 = 0.f, alt1 = 0.f;   // alternating row sums (first column block)
  const long long r64 = 64LL * n;
  const __bf16* xr = Xs + (long long)lr * n;
  const __bf16* cr = Cq + (long long)lr * h + lc;
  const __bf16* sr = Sq + (long long)lr * h + lc;
  const long long h64 = 64LL * h;
#define RVE_SYM_GLOAD(t0)                                                                     \
  do {                                                                                       \
    const int tf = (t0) + lc, tm = n - (t0) - lc;                                            \
    const int te = tf == 0 ? 0 : tm;                                                         \
    fa0 = *reinterpret_cast<const uint4*>(xr + tf);                                          \
    fa1 = *reinterpret_cast<const uint4*>(xr + r64 + tf);                                    \
    ma0 = *reinterpret_cast<const uint4*>(xr + tm - 8);                                      \
    ma1 = *reinterpret_cast<const uint4*>(xr + r64 + tm - 8);                                \
    ea0 = xr[te];                                                                            \
    ea1 = xr[r64 + te];                                                                      \
    rc0 = *reinterpret_cast<const uint4*>(cr + (t0));                                        \
    rc1 = *reinterpret_cast<const uint4*>(cr + h64 + (t0));                                  \
    rs0 = *reinterpret_cast<const uint4*>(sr + (t0));                                        \
    rs1 = *reinterpret_cast<const uint4*>(sr + h64 + (t0));                                  \
  } while (0)
  // fold one staged row chunk (row lr + 64 i) into Xe / Xo and store it
  auto fold = [&](int t0, int i, const uint4& f4, const uint4& m4, __bf16 ev, float& alt) {
    const v8bf f = __builtin_bit_cast(v8bf, f4), m = __builtin_bit_cast(v8bf, m4);
    v8bf ve, vo;
    float sum = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = t0 + lc + e;
      const float xf = (float)f[e];
      const float xm = e == 0 ? (float)ev : (float)m[8 - e];
      ve[e] = (__bf16)(t == 0 ? xf : xf + xm);
      vo[e] = (__bf16)(t == 0 ? 0.f : xf - xm);
      sum += (t & 1) ? -(float)ve[e] : (float)ve[e];
    }
    if (nb == 0) alt += sum;
    *reinterpret_cast<v8bf*>(Ae + (lr + 64 * i) * SLDA + lc) = ve;
    *reinterpret_cast<v8bf*>(Ao + (lr + 64 * i) * SLDA + lc) = vo;
  };
#define RVE_SYM_SSTORE(t0)                                                                    \
  do {                                                                                       \
    fold((t0), 0, fa0, ma0, ea0, alt0);                                                      \
    fold((t0), 1, fa1, ma1, ea1, alt1);                                                      \
    *reinterpret_cast<uint4*>(Bc + lr * SLDA + lc) = rc0;                                    \
    *reinterpret_cast<uint4*>(Bc + (lr + 64) * SLDA + lc) = rc1;                             \
    *reinterpret_cast<uint4*>(Bsn + lr * SLDA + lc) = rs0;                                   \
    *reinterpret_cast<uint4*>(Bsn + (lr + 64) * SLDA + lc) = rs1;                            \
  } while (0)

  v4f accc[4][4], accs[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        accc[i][j][e] = 0.f;
        accs[i][j][e] = 0.f;
      }

  const int frow = lane & 15, fk = (lane >> 4) * 8;
  RVE_SYM_GLOAD(0);
  RVE_SYM_SSTORE(0);
  __syncthreads();
  for (int t0 = 0; t0 < h; t0 += SK) {
    const bool more = t0 + SK < h;
    if (more) RVE_SYM_GLOAD(t0 + SK);
    {
      v8bf bq[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bq[j] = *reinterpret_cast<const v8bf*>(Bc + (wn * 64 + j * 16 + frow) * SLDA + fk);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const v8bf ae = *reinterpret_cast<const v8bf*>(Ae + (wm * 64 + i * 16 + frow) * SLDA + fk);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          accc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ae, bq[j], accc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) bq[j] = *reinterpret_cast<const v8bf*>(Bsn + (wn * 64 + j * 16 + frow) * SLDA + fk);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const v8bf ao = *reinterpret_cast<const v8bf*>(Ao + (wm * 64 + i * 16 + frow) * SLDA + fk);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          accs[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao, bq[j], accs[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) {
      RVE_SYM_SSTORE(t0 + SK);
      __syncthreads();
    }
  }
#undef RVE_SYM_GLOAD
#undef RVE_SYM_SSTORE

  float scale = 1.f;
  if constexpr (EPI == kEpiEinv) scale = (float)real[s >> 1].inv_a0;
  double dot = 0.0;
  // one output value at (output row krow, column col) through the epilogue
  auto emit1 = [&](long long krow, long long col, float v) {
    const long long idx = (long long)s * N2 + krow * n + col;
    if constexpr (EPI == kEpiEinv) v *= einv[krow * n + col] * scale;
    if constexpr (EPI == kEpiZ) {
      const ZT zs = (ZT)v;
      reinterpret_cast<ZT*>(out_v)[idx] = zs;
      dot += (double)zs * widen(rres[idx]);
    } else {
      reinterpret_cast<__bf16*>(out_v)[idx] = (__bf16)v;
    }
  };
  // 32 consecutive values of output row krow from column m0
  auto emit32 = [&](long long krow, long long m0, float* v) {
    const long long obase = (long long)s * N2 + krow * n + m0;
    if constexpr (EPI == kEpiEinv) {
#pragma unroll
      for (int e = 0; e < 32; e += 4) {
        const float4 g = *reinterpret_cast<const float4*>(einv + krow * n + m0 + e);
        v[e] *= g.x * scale; v[e + 1] *= g.y * scale; v[e + 2] *= g.z * scale; v[e + 3] *= g.w * scale;
      }
    }
    if constexpr (EPI == kEpiZ) {
      ZT* out = reinterpret_cast<ZT*>(out_v) + obase;
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        const ZT zs = (ZT)v[e];
        out[e] = zs;
        dot += (double)zs * widen(rres[obase + e]);
      }
    } else {
      __bf16* out = reinterpret_cast<__bf16*>(out_v) + obase;
#pragma unroll
      for (int e = 0; e < 32; e += 8) {
        v8bf pk;
#pragma unroll
        for (int k = 0; k < 8; ++k) pk[k] = (__bf16)v[e + k];
        *reinterpret_cast<v8bf*>(out + e) = pk;
      }
    }
  };

  // output row h: alternating row sums (first column block), summed over the
  // 8 lanes that folded the row's chunks
  if (nb == 0) {
    float al[2] = {alt0, alt1};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      al[i] += __shfl_xor(al[i], 1, 4);
      al[i] += __shfl_xor(al[i], 2, 4);
    }
    if ((tid & 3) == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = lr + 64 * i;
        const float xh = (float)Xs[(long long)row * n + h];
        emit1(h, (long long)mb * TM + row, (al[i] + ((h & 1) ? -xh : xh)) * isq);
      }
    }
  }

  // rows k (C + S) and n - k (C - S) of the 128 columns of this tile, in two
  // halves of 64 columns, transposed through LDS; k = 0 has no mirror row
  const int orow = tid >> 2, oc0 = (tid & 3) * 32;
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    if (wn == hh) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int rl = wm * 64 + i * 16 + 4 * (lane >> 4) + e;
            const int kl = j * 16 + (lane & 15);
            // (-1)^k X[r][h]/sqrt(n): k has the parity of the lane
            const float c = accc[i][j][e] + ((lane & 1) ? -hrow[rl] : hrow[rl]);
            Cp[kl * TLDC + rl] = c + accs[i][j][e];
            Cm[kl * TLDC + rl] = c - accs[i][j][e];
          }
    }
    __syncthreads();
    const long long k = (long long)nb * TN + hh * 64 + orow;
    const long long m0 = (long long)mb * TM + oc0;
    float v[32];
#pragma unroll
    for (int e = 0; e < 32; e += 4) {
      const float4 c = *reinterpret_cast<const float4*>(Cp + orow * TLDC + oc0 + e);
      v[e] = c.x; v[e + 1] = c.y; v[e + 2] = c.z; v[e + 3] = c.w;
    }
    emit32(k, m0, v);
    if (k != 0) {
#pragma unroll
      for (int e = 0; e < 32; e += 4) {
        const float4 c = *reinterpret_cast<const float4*>(Cm + orow * TLDC + oc0 + e);
        v[e] = c.x; v[e + 1] = c.y; v[e + 2] = c.z; v[e + 3] = c.w;
      }
      emit32(n - k, m0, v);
    }
    __syncthreads();
  }
  if constexpr (EPI == kEpiZ) {
    double d[1] = {dot};
    block_sum<1>(d, red);
    if (tid == 0) part[(long long)s * (MB * NB) + mb * NB + nb] = d[0];
  }
}

bool big_bf16_tiles(int n, int prec) { return (prec == kGemmBF16 || prec == kGemmF16) && n % TM == 0; }
bool folded_bf16_tiles(int n, int prec) { return prec == kGemmBF16 && n % (2 * TN) == 0; }

// The four (2D) transforms with the 64 x 64 kernel.
template <class Tr, class ZT>
void run_precond(const Work& w, const GemmTables& t, hipStream_t st, int phase) {
  using op_t = typename Tr::op_t;
  const int n = w.n;
  const long long T = (long long)w.S * (n / BM) * (n / BN);
  const dim3 grid((unsigned)T), block(kBlock);
  const op_t* Q = reinterpret_cast<const op_t*>(t.q);
  const void* einv = std::is_same<typename Tr::acc_t, double>::value ? (const void*)t.einv64 : (const void*)t.einv32;
  op_t* u1 = reinterpret_cast<op_t*>(w.u1);
  op_t* u2 = reinterpret_cast<op_t*>(w.u2);
  const double em = t.emin;
  // T1 = (R Q)^T, from the FP64 residual or from its GEMM-precision copy
  if (phase >= 0 && phase != 0) {
  } else if (w.rlo)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore>), grid, block, 0, st, (const op_t*)w.rlo, Q, (void*)u1,
                       n, w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  else
    hipLaunchKernelGGL((k_hartley<Tr, double, kEpiStore>), grid, block, 0, st, w.r, Q, (void*)u1, n, w.S,
                       w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  // W = (Q R Q) ./ (a0 E)
  if (phase < 0 || phase == 1)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiEinv>), grid, block, 0, st, u1, Q, (void*)u2, n, w.S, w.sys,
                       w.real, einv, (const double*)nullptr, nullptr, em);
  // T3 = (W Q)^T
  if (phase < 0 || phase == 2)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore>), grid, block, 0, st, u2, Q, (void*)u1, n, w.S, w.sys,
                       w.real, nullptr, (const double*)nullptr, nullptr, em);
  // z = Q W Q, partial sums of r.z
  if (phase >= 0 && phase != 3) {
  } else if (w.rlo)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiZ, ZT, op_t>), grid, block, 0, st, u1, Q, w.z, n, w.S, w.sys,
                       w.real, nullptr, (const op_t*)w.rlo, w.part_rz, em);
  else
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiZ, ZT, double>), grid, block, 0, st, u1, Q, w.z, n, w.S, w.sys,
                       w.real, nullptr, w.r, w.part_rz, em);
}

// Three dimensions: six transforms out = (X Q)^T of the n^2 x n views; the
// third scales by 1/(a0 E), the sixth writes z with partial sums of r.z.
template <class Tr, class ZT>
void run_precond3(const Work& w, const GemmTables& t, hipStream_t st, int phase) {
  using op_t = typename Tr::op_t;
  const int n = w.n;
  const long long T = (long long)w.S * gemm_tiles_per_system3(n);
  const dim3 grid((unsigned)T), block(kBlock);
  const op_t* Q = reinterpret_cast<const op_t*>(t.q);
  const void* einv =
      std::is_same<typename Tr::acc_t, double>::value ? (const void*)t.einv3_64 : (const void*)t.einv3_32;
  op_t* u1 = reinterpret_cast<op_t*>(w.u1);
  op_t* u2 = reinterpret_cast<op_t*>(w.u2);
  const double em = t.emin;
  auto on = [&](int ph) { return phase < 0 || phase == ph; };
  if (!on(0)) {
  } else if (w.rlo)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore, double, double, 3>), grid, block, 0, st, (const op_t*)w.rlo,
                       Q, (void*)u1, n, w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  else
    hipLaunchKernelGGL((k_hartley<Tr, double, kEpiStore, double, double, 3>), grid, block, 0, st, w.r, Q, (void*)u1,
                       n, w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  if (on(1))
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore, double, double, 3>), grid, block, 0, st, u1, Q, (void*)u2, n,
                       w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  if (on(2))
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiEinv, double, double, 3>), grid, block, 0, st, u2, Q, (void*)u1, n,
                       w.S, w.sys, w.real, einv, (const double*)nullptr, nullptr, em);
  if (on(3))
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore, double, double, 3>), grid, block, 0, st, u1, Q, (void*)u2, n,
                       w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  if (on(4))
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiStore, double, double, 3>), grid, block, 0, st, u2, Q, (void*)u1, n,
                       w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr, em);
  if (!on(5)) {
  } else if (w.rlo)
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiZ, ZT, op_t, 3>), grid, block, 0, st, u1, Q, w.z, n, w.S, w.sys,
                       w.real, nullptr, (const op_t*)w.rlo, w.part_rz, em);
  else
    hipLaunchKernelGGL((k_hartley<Tr, op_t, kEpiZ, ZT, double, 3>), grid, block, 0, st, u1, Q, w.z, n, w.S, w.sys,
                       w.real, nullptr, w.r, w.part_rz, em);
}

// The four transforms with the 16-bit kernel (T = BF16 or FP16), operand
// pipeline PIPE and 64 WMR x 128 tiles.
template <class T, class ZT, int PIPE, int WMR = 2, int WNR = 2, int BI = 4>
void run_precond_h16(const Work& w, const GemmTables& t, hipStream_t st, int phase) {
  const int n = w.n;
  constexpr int TMR = 16 * BI * WMR, TNR = 64 * WNR;
  const long long NT = (long long)w.S * (n / TMR) * (n / TNR);
  const long long NT2 = (long long)w.S * (n / TM) * (n / TN);
  constexpr bool big = TMR == 256 && TNR == 256;
  // The plain transforms in 256 x 256 tiles run one workgroup per CU (a
  // multiple of 8 of them, one set per XCD), each looping over at least four
  // tiles; with fewer tiles one workgroup per tile balances better. The
  // other launches take one workgroup per tile.
  const long long G = big && PIPE == 0 && t.cus >= 8 && NT >= 4LL * (t.cus & ~7) ? (long long)(t.cus & ~7) : NT;
  const dim3 gridp((unsigned)G), grid((unsigned)NT), block(64 * WMR * WNR), grid2((unsigned)NT2), block2(kBlock);
  const T* Q = reinterpret_cast<const T*>(t.q);
  T* u1 = reinterpret_cast<T*>(w.u1);
  T* u2 = reinterpret_cast<T*>(w.u2);
  const double em = t.emin;
  // Tile shape of each transform: the plain ones always take 64 WMR x 64 WNR.
  // The epilogues of the scaling transform (which also forms the r.z
  // partials) and of the last one (z) spill in 256 x 128 tiles (the latter
  // only with the scaled FP16 operands), so there those stay at 128 x 128;
  // the 256 x 256 tile has the registers for all four.
  constexpr int WE = big ? WMR : 2, WEN = big ? WNR : 2, BE = big ? BI : 4;
  constexpr bool tallz = big || !std::is_same<T, _Float16>::value;
  constexpr int WZ = tallz ? WMR : 2, WZN = tallz ? WNR : 2, BZ = tallz ? BI : 4;
  PDir none, pd;
  if (w.pdirect) {
    pd.ring = w.pring;
    pd.slot = (long long)w.S * w.N2;
    pd.m = w.m_ring;
    pd.kiter = w.kiter;
    pd.first = w.pdir_first;
  }
  if (phase < 0 || phase == 0)
    hipLaunchKernelGGL((k_hartley_h16<T, kEpiStore, float, PIPE, WMR, WNR, BI>), gridp, block, 0, st, (const T*)w.rlo, Q,
                       (void*)u1, n, w.S, w.sys, w.real, nullptr, nullptr, em, 0, none);
  if (phase < 0 || phase == 1)
    hipLaunchKernelGGL((k_hartley_h16<T, kEpiEinv, float, PIPE, WE, WEN, BE>), big ? (BI == 8 ? gridp : grid) : grid2, big ? block : block2, 0,
                       st, u1, Q, (void*)u2, n, w.S, w.sys, w.real, t.sin2, w.part_rz, em, t.fd, none);
  if (phase < 0 || phase == 2)
    hipLaunchKernelGGL((k_hartley_h16<T, kEpiStore, float, PIPE, WMR, WNR, BI>), gridp, block, 0, st, u2, Q, (void*)u1, n,
                       w.S, w.sys, w.real, nullptr, nullptr, em, 0, none);
  if (phase < 0 || phase == 3)
    hipLaunchKernelGGL((k_hartley_h16<T, kEpiZ, ZT, PIPE, WZ, WZN, BZ>), tallz ? grid : grid2, tallz ? block : block2, 0,
                       st, u1, Q, w.z, n, w.S, w.sys, w.real, nullptr, nullptr, em, 0, pd);
}

template <class ZT>
void run_precond_bf16_sym(const Work& w, const GemmTables& t, hipStream_t st, int phase) {
  const int n = w.n;
  const long long T = (long long)w.S * (n / TM) * (n / (2 * TN));
  const dim3 grid((unsigned)T), block(kBlock);
  __bf16* u1 = reinterpret_cast<__bf16*>(w.u1);
  __bf16* u2 = reinterpret_cast<__bf16*>(w.u2);
  if (phase < 0 || phase == 0)
    hipLaunchKernelGGL((k_hartley_bf16_sym<kEpiStore, float>), grid, block, 0, st, (const __bf16*)w.rlo, t.ch16,
                       t.sh16, (void*)u1, n, w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr);
  if (phase < 0 || phase == 1)
    hipLaunchKernelGGL((k_hartley_bf16_sym<kEpiEinv, float>), grid, block, 0, st, (const __bf16*)u1, t.ch16,
                       t.sh16, (void*)u2, n, w.S, w.sys, w.real, t.einv32, (const double*)nullptr, nullptr);
  if (phase < 0 || phase == 2)
    hipLaunchKernelGGL((k_hartley_bf16_sym<kEpiStore, float>), grid, block, 0, st, (const __bf16*)u2, t.ch16,
                       t.sh16, (void*)u1, n, w.S, w.sys, w.real, nullptr, (const double*)nullptr, nullptr);
  if (phase < 0 || phase == 3)
    hipLaunchKernelGGL((k_hartley_bf16_sym<kEpiZ, ZT, __bf16>), grid, block, 0, st, (const __bf16*)u1, t.ch16,
                       t.sh16, w.z, n, w.S, w.sys, w.real, nullptr, (const __bf16*)w.rlo, w.part_rz);
}

}  // namespace

size_t gemm_elem_size(int prec) {
  return prec == kGemmF64 ? sizeof(double) : prec == kGemmF32 ? sizeof(float) : 2;
}

bool gemm_variant_valid(int n, int prec, int variant) {
  return variant == 0 || ((variant == 1 || variant == 3) && big_bf16_tiles(n, prec)) ||
         (variant == 2 && folded_bf16_tiles(n, prec)) ||
         ((variant >= 4 && variant <= 7) && big_bf16_tiles(n, prec) && n % 256 == 0);
}

bool gemm_variant_writes_direction(int n, int prec, int variant) {
  return (prec == kGemmBF16 || prec == kGemmF16) && variant != 0 && variant != 2 &&
         gemm_variant_valid(n, prec, variant);
}

int gemm_tiles_per_system(int n, int prec, int variant) {
  // r.z partials per system: one per 64 x 64 output block for the 64 x 64
  // kernel and every 16-bit tile variant (1, 3, 4, 5, 6 write the same
  // values), one per folded 128 x 256 tile for variant 2
  (void)prec;
  return variant == 2 ? (n / TM) * (n / (2 * TN)) : (n / BM) * (n / BN);
}

int gemm_tiles_per_system_max(int n) { return (n / BM) * (n / BN); }

int gemm_tiles_per_system3(int n) { return (n / BM) * n * (n / BN); }

int precond_phases(const Work& w) { return w.dim == 3 ? 6 : 4; }

void launch_precond(const Work& w, int prec, const GemmTables& t, hipStream_t st, int phase) {
  // z is FP64 with FP64 transforms and FP32 in the mixed modes
  if (w.dim == 3) {
    if (prec == kGemmF64)
      run_precond3<TrF64, double>(w, t, st, phase);
    else if (prec == kGemmF32)
      run_precond3<TrF32, float>(w, t, st, phase);
    else if (prec == kGemmF16)
      run_precond3<TrF16, float>(w, t, st, phase);
    else
      run_precond3<TrBF16, float>(w, t, st, phase);
  } else if (prec == kGemmF64) {
    run_precond<TrF64, double>(w, t, st, phase);
  } else if (prec == kGemmF32) {
    run_precond<TrF32, float>(w, t, st, phase);
  } else if (prec == kGemmF16) {
    if (w.pdir16 && w.gemm_variant == 1)
      run_precond_h16<_Float16, __bf16, 0>(w, t, st, phase);
    else if (w.pdir16 && w.gemm_variant == 3)
      run_precond_h16<_Float16, __bf16, 1>(w, t, st, phase);
    else if (w.pdir16 && w.gemm_variant == 7)
      run_precond_h16<_Float16, __bf16, 2, 2, 4, 8>(w, t, st, phase);
    else if (w.pdir16 && w.gemm_variant == 4)
      run_precond_h16<_Float16, __bf16, 0, 4>(w, t, st, phase);
    else if (w.pdir16 && w.gemm_variant == 5)
      run_precond_h16<_Float16, __bf16, 0, 4, 4>(w, t, st, phase);
    else if (w.pdir16 && w.gemm_variant == 6)
      run_precond_h16<_Float16, __bf16, 0, 2, 4, 8>(w, t, st, phase);
    else if (w.gemm_variant == 1)
      run_precond_h16<_Float16, float, 0>(w, t, st, phase);
    else if (w.gemm_variant == 3)
      run_precond_h16<_Float16, float, 1>(w, t, st, phase);
    else if (w.gemm_variant == 4)
      run_precond_h16<_Float16, float, 0, 4>(w, t, st, phase);
    else if (w.gemm_variant == 5)
      run_precond_h16<_Float16, float, 0, 4, 4>(w, t, st, phase);
    else if (w.gemm_variant == 6)
      run_precond_h16<_Float16, float, 0, 2, 4, 8>(w, t, st, phase);
    else if (w.gemm_variant == 7)
      run_precond_h16<_Float16, float, 2, 2, 4, 8>(w, t, st, phase);
    else
      run_precond<TrF16, float>(w, t, st, phase);
  } else if (w.gemm_variant == 2) {
    run_precond_bf16_sym<float>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 1) {
    run_precond_h16<__bf16, __bf16, 0>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 3) {
    run_precond_h16<__bf16, __bf16, 1>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 7) {
    run_precond_h16<__bf16, __bf16, 2, 2, 4, 8>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 4) {
    run_precond_h16<__bf16, __bf16, 0, 4>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 5) {
    run_precond_h16<__bf16, __bf16, 0, 4, 4>(w, t, st, phase);
  } else if (w.pdir16 && w.gemm_variant == 6) {
    run_precond_h16<__bf16, __bf16, 0, 2, 4, 8>(w, t, st, phase);
  } else if (w.gemm_variant == 1) {
    run_precond_h16<__bf16, float, 0>(w, t, st, phase);
  } else if (w.gemm_variant == 3) {
    run_precond_h16<__bf16, float, 1>(w, t, st, phase);
  } else if (w.gemm_variant == 4) {
    run_precond_h16<__bf16, float, 0, 4>(w, t, st, phase);
  } else if (w.gemm_variant == 5) {
    run_precond_h16<__bf16, float, 0, 4, 4>(w, t, st, phase);
  } else if (w.gemm_variant == 6) {
    run_precond_h16<__bf16, float, 0, 2, 4, 8>(w, t, st, phase);
  } else if (w.gemm_variant == 7) {
    run_precond_h16<__bf16, float, 2, 2, 4, 8>(w, t, st, phase);
  } else {
    run_precond<TrBF16, float>(w, t, st, phase);
  }
}

}  // namespace rve
