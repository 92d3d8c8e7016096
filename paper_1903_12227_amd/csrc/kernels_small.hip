// Single-workgroup PCG for small grids (n = 64, FP64): one 256-thread
// workgroup runs the whole iteration of one corrector system (Sec. 3.5: PCG
// with the constant-coefficient periodic preconditioner) without leaving
// the kernel, so a solve costs one launch instead of about ten per
// iteration. The 64 x 64 system lives on the chip: the cells and the Hartley
// matrix in LDS, the vectors x, r, p, z in registers (each thread owns one
// column and a 16-row strip of nodes), and two 64 x 64 LDS buffers serve as
// the operand for the stencil's neighbours and for the transforms.
//
// Preconditioner: the four transforms out = (X Q)^T of the batched path, as
// FP64 MFMA 16x16x4 products inside the workgroup (each wave one 16-row
// strip of the output), the second scaled by 1/(a0 E).
// Dot products: wave sums, then the four wave totals added in a fixed order
// by every thread (deterministic).
#include "launch.h"
#include "stencil2d.h"

namespace rve {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kN = 64;           // grid size handled
constexpr int kLd = kN + 1;      // LDS row stride (odd: spreads column reads over banks)
constexpr int kRows = kN / 4;    // rows of nodes per thread (one 16-row strip per wave)

// Sum over the workgroup, the same value in every thread.
__device__ inline double wg_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// dst = (src Q)^T, optionally times einv / a0 (element [row][col] of the
// result scaled by einv[row][col]). Wave w computes rows 16w .. 16w+15 of
// src Q (four 16 x 16 tiles) and stores them transposed.
template <bool SCALE>
__device__ inline void transform(const double* src, const double* q, double* dst, const double* __restrict__ einv,
                                 double inv_a0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < kN; k0 += 4) {
    const double a = src[(16 * w + fr) * kLd + k0 + fk];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double b = q[(k0 + fk) * kLd + 16 * j + fr];
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    }
  }
  // accumulator register i of lane l: row (l/16) + 4i, column l%16 of the tile
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * w + fk + 4 * i, col = 16 * j + fr;
      double v = acc[j][i];
      if constexpr (SCALE) v *= einv[row * kN + col] * inv_a0;
      dst[col * kLd + row] = v;
    }
}

template <int SCH>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_pcg64(const double* __restrict__ a, double* __restrict__ xg, const double* __restrict__ rg,
        const double* __restrict__ qm, const double* __restrict__ einv, SysState* sys, const RealState* real,
        double tol, int maxit) {
  __shared__ double sa[kN * kLd];   // cells
  __shared__ double sq[kN * kLd];   // Hartley matrix
  __shared__ double s0[kN * kLd];   // operand / transform buffers
  __shared__ double s1[kN * kLd];
  __shared__ double red[4];
  const int s = blockIdx.x, b = s >> 1;
  SysState& S = sys[s];
  if (!S.active) return;   // uniform: f = 0 or an invalid field (x stays 0)
  const int tid = threadIdx.x, col = tid & 63, row0 = (tid >> 6) * kRows;
  const long long N2 = (long long)kN * kN;
  const double* A = a + (long long)b * N2;
  for (int e = tid; e < kN * kN; e += kBlock) {
    const int i = e / kN, j = e % kN;
    sa[i * kLd + j] = A[e];
    sq[i * kLd + j] = qm[e];
  }
  double x[kRows], r[kRows], p[kRows], z[kRows];
#pragma unroll
  for (int m = 0; m < kRows; ++m) {
    x[m] = 0.0;
    r[m] = rg[(long long)s * N2 + (row0 + m) * kN + col];
  }
  const double inv_a0 = real[b].inv_a0, fnorm = S.fnorm;

  // z = (a0 A_Delta)^+ r: r into s0, four transforms s0 -> s1 -> s0 -> s1 -> s0
  auto precond = [&]() {
    __syncthreads();   // earlier readers of s0 / s1 are done
#pragma unroll
    for (int m = 0; m < kRows; ++m) s0[(row0 + m) * kLd + col] = r[m];
    __syncthreads();
    transform<false>(s0, sq, s1, nullptr, 0.0);
    __syncthreads();
    transform<true>(s1, sq, s0, einv, inv_a0);
    __syncthreads();
    transform<false>(s0, sq, s1, nullptr, 0.0);
    __syncthreads();
    transform<false>(s1, sq, s0, nullptr, 0.0);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kRows; ++m) z[m] = s0[(row0 + m) * kLd + col];
  };
  // q = A p with p staged in s1
  auto apply = [&](double (&q)[kRows]) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kRows; ++m) s1[(row0 + m) * kLd + col] = p[m];
    __syncthreads();
    const int cm = col == 0 ? kN - 1 : col - 1, cp = col == kN - 1 ? 0 : col + 1;
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
      const int i = row0 + m, im = i == 0 ? kN - 1 : i - 1, ip = i == kN - 1 ? 0 : i + 1;
      const double um[3] = {s1[im * kLd + cm], s1[im * kLd + col], s1[im * kLd + cp]};
      const double uc[3] = {s1[i * kLd + cm], s1[i * kLd + col], s1[i * kLd + cp]};
      const double up[3] = {s1[ip * kLd + cm], s1[ip * kLd + col], s1[ip * kLd + cp]};
      const double a00 = sa[im * kLd + cm], a01 = sa[im * kLd + col], a10 = sa[i * kLd + cm],
                   a11 = sa[i * kLd + col];
      if constexpr (SCH == 1)
        q[m] = fd5_apply<double>(a00, a01, a10, a11, um, uc, up);
      else
        q[m] = q1_apply<double>(a00, a01, a10, a11, um, uc, up);
    }
  };

  precond();
  double rz = 0.0;
#pragma unroll
  for (int m = 0; m < kRows; ++m) {
    p[m] = z[m];
    rz += r[m] * z[m];
  }
  rz = wg_sum(rz, red);
  int it = 0, status = 0;
  double relres = 1.0;
  if (!(rz > 0.0) || !isfinite(rz)) status = 2;   // RVE_BREAKDOWN
  while (status == 0) {
    double q[kRows];
    apply(q);
    double pq = 0.0;
#pragma unroll
    for (int m = 0; m < kRows; ++m) pq += p[m] * q[m];
    pq = wg_sum(pq, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = 2;
      break;
    }
    const double alpha = rz / pq;
    double rr = 0.0;
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
      x[m] = fma(alpha, p[m], x[m]);
      r[m] = fma(-alpha, q[m], r[m]);
      rr += r[m] * r[m];
    }
    rr = wg_sum(rr, red);
    ++it;
    relres = sqrt(rr) / fnorm;
    if (relres <= tol) break;
    if (!isfinite(relres)) {
      status = 2;
      break;
    }
    if (it >= maxit) {
      status = 1;   // RVE_NOT_CONVERGED
      break;
    }
    precond();
    double rzn = 0.0;
#pragma unroll
    for (int m = 0; m < kRows; ++m) rzn += r[m] * z[m];
    rzn = wg_sum(rzn, red);
    if (!(rzn > 0.0) || !isfinite(rzn)) {
      status = 2;
      break;
    }
    const double beta = rzn / rz;
    rz = rzn;
#pragma unroll
    for (int m = 0; m < kRows; ++m) p[m] = fma(beta, p[m], z[m]);
  }
#pragma unroll
  for (int m = 0; m < kRows; ++m) xg[(long long)s * N2 + (row0 + m) * kN + col] = x[m];
  if (tid == 0) {
    S.iters = it;
    S.relres = relres;
    S.status = status;
    S.active = 0;
  }
}

}  // namespace

bool small_solver_fits(const Work& w) {
  return w.dim == 2 && w.n == kN && w.mixed == 0 && w.sprec == 0;
}

void launch_pcg_small(const Work& w, const double* q64, const double* einv64, double tol, int maxit,
                      hipStream_t st) {
  if (w.scheme == 1)
    hipLaunchKernelGGL(k_pcg64<1>, dim3(w.S), dim3(kBlock), 0, st, w.a, w.x, (const double*)w.r, q64, einv64,
                       w.sys, (const RealState*)w.real, tol, maxit);
  else
    hipLaunchKernelGGL(k_pcg64<0>, dim3(w.S), dim3(kBlock), 0, st, w.a, w.x, (const double*)w.r, q64, einv64,
                       w.sys, (const RealState*)w.real, tol, maxit);
}

}  // namespace rve
