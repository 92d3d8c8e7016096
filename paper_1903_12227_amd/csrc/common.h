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

}  // namespace rve
