// Shared device-side definitions for the librve kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rve {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per workgroup in every kernel
constexpr int kTile = 64;            // node/cell tile edge of the stencil-shaped kernels
constexpr int kStrip = kTile / 4;    // rows per wave in those kernels (4 waves per tile)

// Per corrector system (2 per realization) PCG state, in device memory.
struct SysState {
  double rz;        // r.z of the current direction
  double alpha;
  double beta;
  double fnorm;     // ||f||_2 of the mean-zero right-hand side
  double relres;    // last recursive ||r||/||f||
  double mean_f;    // mean of the raw right-hand side (removed once)
  double mean_x;    // mean of the final iterate (removed on output)
  int active;       // 1 while the system iterates
  int iters;
  int status;       // enum rve_status
  int valid;        // coefficient field passed the device check
  // Scale of the GEMM-precision residual copy (read with FP16 transforms
  // only; 1 otherwise): lo_scale is the factor of the copy the transforms
  // read, lo_next the one the next copy is written with (0.25 sqrt(N) / ||r||
  // of the latest residual norm).
  double lo_scale;
  double lo_next;
};

// Per realization quantities.
struct RealState {
  double a_sum;
  double a_min;
  double a_max;
  double inv_a0;    // 1 / ((a_max + a_min)/2)
  int bad;          // count of cells with a <= 0 or NaN
  int pad;
};

// Deterministic wave64 sum: a fixed butterfly over xor distances 32..1.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
  return v;
}

// Sum of NV values over a 256-thread block, fixed order; result valid in
// thread 0 only. `sh` must hold 4*NV doubles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[w * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((sh[k] + sh[NV + k]) + (sh[2 * NV + k] + sh[3 * NV + k]));
  }
}

__device__ inline int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ inline int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// One n x n block (a system's vector or a realization's coefficients) read and
// written through a buffer resource: the block's base and size sit in scalar
// registers, a row is addressed by a wave-uniform byte offset (scalar) and a
// column by a per-lane 32-bit byte offset that stays fixed down a strip, so no
// access needs per-lane 64-bit address arithmetic. An access beyond the block
// reads 0 and writes nothing. NT: streaming (non-temporal) access.
// AUX: the cache policy bits (2: non-temporal).
template <int NB, int AUX>
__device__ inline auto buf_load_bytes(__amdgpu_buffer_rsrc_t rs, unsigned vo, unsigned so) {
  if constexpr (NB == 1) return __builtin_amdgcn_raw_buffer_load_b8(rs, vo, so, AUX);
  else if constexpr (NB == 2) return __builtin_amdgcn_raw_buffer_load_b16(rs, vo, so, AUX);
  else if constexpr (NB == 4) return __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, AUX);
  else if constexpr (NB == 8) return __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, AUX);
  else return __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, AUX);
}
template <int AUX, class W>
__device__ inline void buf_store_bytes(W v, __amdgpu_buffer_rsrc_t rs, unsigned vo, unsigned so) {
  constexpr int NB = (int)sizeof(W);
  if constexpr (NB == 1) __builtin_amdgcn_raw_buffer_store_b8(__builtin_bit_cast(unsigned char, v), rs, vo, so, AUX);
  else if constexpr (NB == 2) __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), rs, vo, so, AUX);
  else if constexpr (NB == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, vo, so, AUX);
  else if constexpr (NB == 8) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, vo, so, AUX);
  } else {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rs, vo, so, AUX);
  }
}

// A byte offset past the end of every block: a load there returns 0 and a
// store there is dropped, without a memory access (used to switch accesses
// off without a branch around them).
constexpr unsigned kPastBlock = 0x80000000u;

template <class T>
struct Plane {
  template <int C> struct alignas(sizeof(T) * C) Run { T e[C]; };
  __amdgpu_buffer_rsrc_t rs;
  unsigned row_bytes;
  __device__ Plane(const T* base, int n)
      : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, n * n * (int)sizeof(T), 0x00020000)),
        row_bytes((unsigned)n * (unsigned)sizeof(T)) {}
  // element at byte offset col of row `row`
  __device__ T get(int row, unsigned col) const {
    return __builtin_bit_cast(T, buf_load_bytes<sizeof(T), 0>(rs, col, (unsigned)row * row_bytes));
  }
  // V consecutive elements from byte offset col of row `row`, in loads of at
  // most 16 bytes
  template <int V, bool NT = false>
  __device__ void load(int row, unsigned col, T* v) const {
    constexpr int C = (int)(16 / sizeof(T)) < V ? (int)(16 / sizeof(T)) : V;
#pragma unroll
    for (int k = 0; k < V; k += C) {
      const Run<C> t = __builtin_bit_cast(
          Run<C>, buf_load_bytes<sizeof(T) * C, NT ? 2 : 0>(rs, col + k * (unsigned)sizeof(T), (unsigned)row * row_bytes));
#pragma unroll
      for (int e = 0; e < C; ++e) v[k + e] = t.e[e];
    }
  }
  // V consecutive elements to byte offset col of row `row`, in stores of at
  // most 8 bytes. (A buffer store of more than 8 bytes with the row offset
  // in a scalar register needs a wait state before its data registers are
  // overwritten, which the compiler does not insert for that form on this
  // target; the two stencil passes then stored values rewritten by the
  // following instruction. Stores of 8 bytes have no such hazard.)
  template <int V, bool NT = false>
  __device__ void store(int row, unsigned col, const T* v) const {
    constexpr int C = (int)(8 / sizeof(T)) < V ? (int)(8 / sizeof(T)) : V;
#pragma unroll
    for (int k = 0; k < V; k += C) {
      Run<C> t;
#pragma unroll
      for (int e = 0; e < C; ++e) t.e[e] = v[k + e];
      buf_store_bytes<NT ? 2 : 0>(t, rs, col + k * (unsigned)sizeof(T), (unsigned)row * row_bytes);
    }
  }
};

// Neighbour columns from the neighbouring lanes. Lane l of a wave holds
// columns c0 .. c0 + V - 1 of a row, with c0 = (64 band + l) V; column c0 - 1
// is the last column of lane l - 1 and column c0 + V the first of lane
// l + 1, which a DPP wave shift brings over. Lanes 0 and 63, whose
// neighbours lie in another band, keep `halo` (kHaloBelow: lane 0 takes the
// lower neighbour; kHaloAbove: lane 63 the upper one).
constexpr int kHaloBelow = 0x138;   // DPP wave_shr:1, lane l reads lane l - 1
constexpr int kHaloAbove = 0x130;   // DPP wave_shl:1, lane l reads lane l + 1
template <int CTRL, class T>
__device__ inline T shift_in(T halo, T v) {
  static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "16-, 32- or 64-bit values");
  if constexpr (sizeof(T) == 2) {
    const int h = __builtin_bit_cast(unsigned short, halo), x = __builtin_bit_cast(unsigned short, v);
    return __builtin_bit_cast(T, (unsigned short)__builtin_amdgcn_update_dpp(h, x, CTRL, 0xf, 0xf, false));
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, halo), __builtin_bit_cast(int, v),
                                                             CTRL, 0xf, 0xf, false));
  } else {
    typedef int i2 __attribute__((ext_vector_type(2)));
    const i2 h = __builtin_bit_cast(i2, halo), x = __builtin_bit_cast(i2, v);
    i2 r;
    r.x = __builtin_amdgcn_update_dpp(h.x, x.x, CTRL, 0xf, 0xf, false);
    r.y = __builtin_amdgcn_update_dpp(h.y, x.y, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(T, r);
  }
}
// The byte offset a lane reads a row's neighbour columns from: column c0 - 1
// in lane 0, c0 + V in lane 63, past the block (no access) in every other.
__device__ inline unsigned halo_offset(int lane, unsigned below, unsigned above) {
  return lane == 0 ? below : lane == kWave - 1 ? above : kPastBlock;
}

// The wave's index within its workgroup, as a wave-uniform (scalar) value.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)); }

}  // namespace rve
