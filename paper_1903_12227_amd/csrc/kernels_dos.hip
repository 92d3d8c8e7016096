// Spectral density of the stiffness matrix (Appendix, eqns. DOS and
// DOS_gauss) by Chebyshev moments with probe vectors.
//
// With c = lmax / 2 >= lambda_max / 2 and Ahat = A / c - I (spectrum in
// [-1, 1]), the moments mu_k = v^T T_k(Ahat) v / m of a probe v follow from
// w_0 = v, w_1 = Ahat v, w_{k+1} = 2 Ahat w_k - w_{k-1} and the doubling
// identities T_{2k} = 2 T_k^2 - T_0, T_{2k+1} = 2 T_{k+1} T_k - T_1:
// mu_{2k} = 2 w_k.w_k / m - mu_0, mu_{2k+1} = 2 w_{k+1}.w_k / m - mu_1, so K
// moments take about K/2 operator applies. The density is then
// phi(t) = sum_k a_k(t) mu_k with a_k(t) the Chebyshev coefficients of
// x -> g_eta(t - c (1 + x)); by a Chebyshev-Gauss rule with Q nodes theta_q,
// phi(t) = (1/Q) sum_q g_eta(t - c (1 + cos theta_q)) S_q with
// S_q = sum_k (2 - [k == 0]) mu_k cos(k theta_q), which is evaluated here in
// that order.
#include "launch.h"

namespace rve {

namespace {

// w_next = alpha (A w) + beta w + gamma w_prev (in place over w_prev), with
// per-workgroup partial sums of w.w and w_next.w for every vector.
__global__ void __launch_bounds__(kBlock) k_cheb_step(const double* __restrict__ aw, const double* __restrict__ w,
                                                       double* __restrict__ wp, long long N2, double alpha,
                                                       double beta, double gamma, double* __restrict__ part) {
  __shared__ double sh[4 * 2];
  const int s = blockIdx.y;
  const long long off = (long long)s * N2;
  const long long stride = (long long)gridDim.x * kBlock * 2;
  double acc[2] = {0.0, 0.0};
  for (long long i = ((long long)blockIdx.x * kBlock + threadIdx.x) * 2; i < N2; i += stride) {
    const double2 av = *reinterpret_cast<const double2*>(aw + off + i);
    const double2 wv = *reinterpret_cast<const double2*>(w + off + i);
    const double2 pv = *reinterpret_cast<const double2*>(wp + off + i);
    double2 nv;
    nv.x = alpha * av.x + beta * wv.x + gamma * pv.x;
    nv.y = alpha * av.y + beta * wv.y + gamma * pv.y;
    *reinterpret_cast<double2*>(wp + off + i) = nv;
    acc[0] += wv.x * wv.x + wv.y * wv.y;
    acc[1] += nv.x * wv.x + nv.y * wv.y;
  }
  block_sum<2>(acc, sh);
  if (threadIdx.x == 0) {
    part[((long long)s * gridDim.x + blockIdx.x) * 2] = acc[0];
    part[((long long)s * gridDim.x + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// The two moments of step k for every vector, from the step's partials.
// k = 0: mu_0 = w_0.w_0 / m, mu_1 = w_1.w_0 / m. k >= 1: mu_2k and mu_2k+1
// by the doubling identities. Vectors are in pair-major order (pair p,
// realization b, member i): s = (p B + b) 2 + i; its moments go to
// mu[b][2 p + i][.].
__global__ void k_cheb_moments(const double* __restrict__ part, int P, int B, int nv, int K, int k, double inv_m,
                               double* __restrict__ mu) {
  const int s = blockIdx.x, lane = threadIdx.x;
  double d0 = 0.0, d1 = 0.0;
  for (int t = lane; t < P; t += kWave) {
    d0 += part[((long long)s * P + t) * 2];
    d1 += part[((long long)s * P + t) * 2 + 1];
  }
  d0 = wave_sum(d0);
  d1 = wave_sum(d1);
  if (lane == 0) {
    const int i = s & 1, pb = s >> 1, b = pb % B, p = pb / B;
    double* M = mu + ((long long)b * nv + 2 * p + i) * K;
    if (k == 0) {
      M[0] = d0 * inv_m;
      if (K > 1) M[1] = d1 * inv_m;
    } else {
      if (2 * k < K) M[2 * k] = 2.0 * d0 * inv_m - M[0];
      if (2 * k + 1 < K) M[2 * k + 1] = 2.0 * d1 * inv_m - M[1];
    }
  }
}

__device__ inline double gauss_eta(double t, double eta) {
  const double u = t / eta;
  return exp(-0.5 * u * u) / (2.5066282746310002 * eta);   // sqrt(2 pi) eta
}

// S[b][q] = sum_k (2 - [k == 0]) mubar_k cos(k theta_q), mubar the probe mean.
__global__ void k_dos_S(const double* __restrict__ mu, int B, int nv, int K, int Q, double* __restrict__ S) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (q >= Q) return;
  const double th = 3.14159265358979323846 * ((double)q + 0.5) / (double)Q;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    double m = 0.0;
    for (int v = 0; v < nv; ++v) m += mu[((long long)b * nv + v) * K + k];
    acc += (k == 0 ? 1.0 : 2.0) * (m / nv) * cos((double)k * th);
  }
  S[(long long)b * Q + q] = acc;
}

// phi[b][i] = (1/Q) sum_q g_eta(t_i - c (1 + cos theta_q)) S[b][q].
__global__ void k_dos_phi(const double* __restrict__ S, int Q, double c, double eta, int nt,
                          const double* __restrict__ t, double* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (i >= nt) return;
  double acc = 0.0;
  for (int q = 0; q < Q; ++q) {
    const double th = 3.14159265358979323846 * ((double)q + 0.5) / (double)Q;
    acc += gauss_eta(t[i] - c * (1.0 + cos(th)), eta) * S[(long long)b * Q + q];
  }
  phi[(long long)b * nt + i] = acc / (double)Q;
}

// Per-workgroup max of the cell values and count of invalid cells (<= 0 or
// NaN) over `total` cells: part[2 blk] = max, part[2 blk + 1] = count.
__global__ void __launch_bounds__(kBlock) k_field_max(const double* __restrict__ a, long long total,
                                                       double* __restrict__ part) {
  __shared__ double sh[4 * 2];
  double mx = 0.0, bad = 0.0;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += stride) {
    const double v = a[i];
    if (v > 0.0) mx = fmax(mx, v);
    else bad += 1.0;
  }
  mx = wave_max(mx);
  bad = wave_sum(bad);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[2 * w] = mx;
    sh[2 * w + 1] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = fmax(fmax(sh[0], sh[2]), fmax(sh[4], sh[6]));
    part[2 * blockIdx.x + 1] = (sh[1] + sh[3]) + (sh[5] + sh[7]);
  }
}

__global__ void k_field_max_final(const double* __restrict__ part, int P, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double mx = 0.0, bad = 0.0;
  for (int t = lane; t < P; t += kWave) {
    mx = fmax(mx, part[2 * t]);
    bad += part[2 * t + 1];
  }
  mx = wave_max(mx);
  bad = wave_sum(bad);
  if (lane == 0) {
    out[0] = mx;
    out[1] = bad;
  }
}

}  // namespace

int field_max_blocks(long long total) {
  long long b = (total + kBlock - 1) / kBlock;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_field_max(const double* a, long long total, double* part, double* out, hipStream_t st) {
  const int P = field_max_blocks(total);
  hipLaunchKernelGGL(k_field_max, dim3(P), dim3(kBlock), 0, st, a, total, part);
  hipLaunchKernelGGL(k_field_max_final, dim3(1), dim3(kWave), 0, st, part, P, out);
}

int dos_vec_tiles(long long N2) {
  long long vb = N2 / 1024;
  if (vb > 256) vb = 256;
  if (vb < 1) vb = 1;
  return (int)vb;
}

// W, Wp, AW: [nv/2][B][2][n][n] (pair-major), W holding the probes and Wp
// zeroed (the first step reads it with weight 0); part:
// [B nv][dos_vec_tiles(n^2)][2]; mu: [B][nv][K].
void launch_dos_moments(int B, int n, int scheme, const double* a, int nv, double* W, double* Wp, double* AW,
                        double lmax, int K, double* part, double* mu, hipStream_t st) {
  const long long N2 = (long long)n * n;
  const int S = B * nv, P = dos_vec_tiles(N2);
  const double c = 0.5 * lmax, inv_m = 1.0 / (double)N2;
  const long long pair = (long long)B * 2 * N2;
  const int steps = (K + 1) / 2;   // step k yields mu_2k and mu_2k+1
  double* w = W;
  double* wp = Wp;
  for (int k = 0; k < steps; ++k) {
    for (int p = 0; p < nv / 2; ++p) launch_apply_stencil(B, n, scheme, a, w + p * pair, AW + p * pair, st);
    // k = 0: w_1 = A w_0 / c - w_0 (into wp); later w_{k+1} = 2 A w_k / c - 2 w_k - w_{k-1}
    const double al = k == 0 ? 1.0 / c : 2.0 / c, be = k == 0 ? -1.0 : -2.0, ga = k == 0 ? 0.0 : -1.0;
    hipLaunchKernelGGL(k_cheb_step, dim3(P, S), dim3(kBlock), 0, st, AW, w, wp, N2, al, be, ga, part);
    hipLaunchKernelGGL(k_cheb_moments, dim3(S), dim3(kWave), 0, st, part, P, B, nv, K, k, inv_m, mu);
    double* t = w;   // w_{k+1} now sits in wp: swap roles
    w = wp;
    wp = t;
  }
}

void launch_dos_eval(int B, int nv, int K, const double* mu, double lmax, double eta, int Q, int nt,
                     const double* t, double* S, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(k_dos_S, dim3((Q + kBlock - 1) / kBlock, B), dim3(kBlock), 0, st, mu, B, nv, K, Q, S);
  hipLaunchKernelGGL(k_dos_phi, dim3((nt + kBlock - 1) / kBlock, B), dim3(kBlock), 0, st, S, Q, 0.5 * lmax, eta,
                     nt, t, phi);
}

}  // namespace rve
