// On-device sampling of the random inclusion model (Sec. 2, covered domain
// eqn. Stoch-decomp, coefficient eqn. ahm_coef) on the node lattice: every
// lattice site is independently a square centre with probability
// occ_threshold / 2^32, decided by integer comparison of one word of
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed and
// counted by (site group, realization index); a square centred at site s
// covers cells s - side/2 + u, u = 0 .. side-1, in each direction (mod n).
// Integer arithmetic only, so the field of a given (seed, realization) is
// the same on every device and in any batch.
#include "launch.h"

namespace rve {

namespace {

constexpr unsigned kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr unsigned kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// Philox4x32 with 10 rounds: per round (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2
// (32 x 32 -> 64-bit products), c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
// the key advances by the Weyl constants between rounds.
__device__ inline uint4 philox4x32_10(uint4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const unsigned long long p0 = (unsigned long long)kPhiloxM0 * c.x;
    const unsigned long long p1 = (unsigned long long)kPhiloxM1 * c.z;
    c = make_uint4((unsigned)(p1 >> 32) ^ c.y ^ k0, (unsigned)p1, (unsigned)(p0 >> 32) ^ c.w ^ k1, (unsigned)p0);
  }
  return c;
}

constexpr int kST = 64;          // cell tile edge
constexpr int kMaxSide = 32;
constexpr int kSH = kST + kMaxSide - 1;   // site rows / columns a tile can need

// One 64 x 64 cell tile of one realization: occupancy of the sites the tile
// needs (rows and columns c - side/2 + 1 .. c + side/2 of its cells) into
// LDS, then the window OR along rows and along columns. The occupancy comes
// from one Philox word per site (lattice Poisson law), or (occ_in non-null)
// from a byte per site written by k_fixed_centres.
__global__ void __launch_bounds__(kBlock) k_sample_lattice(int n, int side, unsigned seed_lo, unsigned seed_hi,
                                                             long long first, unsigned occ_threshold, double a_in,
                                                             double a_bg, double* __restrict__ a,
                                                             const uint8_t* __restrict__ occ_in) {
  __shared__ unsigned char occ[kSH][kSH + 1];
  __shared__ unsigned char row_or[kSH][kST + 1];
  const int b = blockIdx.z;
  const long long r = first + b;
  const unsigned r_lo = (unsigned)((unsigned long long)r & 0xFFFFFFFFull);
  const unsigned r_hi = (unsigned)((unsigned long long)r >> 32);
  const int R0 = blockIdx.y * kST, C0 = blockIdx.x * kST;
  const int lo = side / 2 - 1;          // sites before a cell in its window
  const int hw = kST + side - 1;        // sites per tile edge
  for (int idx = threadIdx.x; idx < hw * hw; idx += kBlock) {
    const int ai = idx / hw, bj = idx % hw;
    int i = R0 - lo + ai, j = C0 - lo + bj;
    i = (i % n + n) % n;
    j = (j % n + n) % n;
    const unsigned s = (unsigned)i * (unsigned)n + (unsigned)j;
    if (occ_in) {
      occ[ai][bj] = occ_in[(long long)b * n * n + s];
    } else {
      const uint4 wv = philox4x32_10(make_uint4(s >> 2, r_lo, r_hi, 0u), seed_lo, seed_hi);
      const unsigned x = (s & 3u) == 0 ? wv.x : (s & 3u) == 1 ? wv.y : (s & 3u) == 2 ? wv.z : wv.w;
      occ[ai][bj] = x < occ_threshold ? 1 : 0;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < hw * kST; idx += kBlock) {
    const int ai = idx / kST, c = idx % kST;
    unsigned char v = 0;
    for (int t = 0; t < side; ++t) v |= occ[ai][c + t];
    row_or[ai][c] = v;
  }
  __syncthreads();
  const long long N2 = (long long)n * n;
  double* A = a + (long long)b * N2;
  for (int idx = threadIdx.x; idx < kST * kST; idx += kBlock) {
    const int rr = idx / kST, c = idx % kST;
    unsigned char v = 0;
    for (int t = 0; t < side; ++t) v |= row_or[rr + t][c];
    A[(long long)(R0 + rr) * n + C0 + c] = v ? a_in : a_bg;
  }
}

// The paper's fixed-count law: exactly K square centres per realization at
// uniformly drawn grid nodes (independent draws, so centres may coincide).
// Centre k of realization r: words 0 and 1 of Philox4x32-10 with counter
// (k, r mod 2^32, r div 2^32, kFixedTag) form v = w0 + 2^32 w1, and the node
// is floor(v n^2 / 2^64). One thread per (realization, centre) sets its
// node's byte in occ [B][n^2] (all writers store the same value).
constexpr unsigned kFixedTag = 0x46495843u;
__global__ void __launch_bounds__(kBlock) k_fixed_centres(int B, long long n2, int K, unsigned seed_lo,
                                                          unsigned seed_hi, long long first, uint8_t* __restrict__ occ) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)B * K) return;
  const int b = (int)(t / K), k = (int)(t % K);
  const unsigned long long r = (unsigned long long)(first + b);
  const uint4 wv = philox4x32_10(make_uint4((unsigned)k, (unsigned)(r & 0xFFFFFFFFull), (unsigned)(r >> 32), kFixedTag),
                                 seed_lo, seed_hi);
  const unsigned long long v = (unsigned long long)wv.x | ((unsigned long long)wv.y << 32);
  const unsigned long long c = __umul64hi(v, (unsigned long long)n2);
  occ[(long long)b * n2 + (long long)c] = 1;
}

__global__ void __launch_bounds__(kBlock) k_zero_bytes(uint8_t* __restrict__ p, long long count) {
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) p[i] = 0;
}

// Probe vectors with entries +-1: entry i of the [total] array takes bit
// (i mod 32) of word (i div 32) mod 4 of Philox4x32-10 with counter
// (i div 128 mod 2^32, i div 2^39, 0, kProbeTag) and key (seed mod 2^32,
// seed div 2^32); a set bit gives -1. Thread t writes entries 128 t ..
// 128 t + 127.
constexpr unsigned kProbeTag = 0x50524F42u;   // distinguishes these counters from the lattice sampler's
__global__ void __launch_bounds__(kBlock) k_probes(long long total, unsigned seed_lo, unsigned seed_hi,
                                                   double* __restrict__ v) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long i0 = t * 128;
  if (i0 >= total) return;
  const uint4 wv = philox4x32_10(make_uint4((unsigned)((unsigned long long)t & 0xFFFFFFFFull),
                                            (unsigned)((unsigned long long)t >> 32), 0u, kProbeTag),
                                 seed_lo, seed_hi);
  const unsigned words[4] = {wv.x, wv.y, wv.z, wv.w};
  for (int k = 0; k < 128 && i0 + k < total; ++k)
    v[i0 + k] = ((words[k >> 5] >> (k & 31)) & 1u) ? -1.0 : 1.0;
}

}  // namespace

void launch_probes(long long total, unsigned long long seed, double* v, hipStream_t st) {
  const long long threads = (total + 127) / 128;
  const long long blocks = (threads + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_probes, dim3((unsigned)blocks), dim3(kBlock), 0, st, total,
                     (unsigned)(seed & 0xFFFFFFFFull), (unsigned)(seed >> 32), v);
}

bool sample_side_valid(int n, int side) { return side >= 1 && side <= kMaxSide && side <= n; }

void launch_sample_lattice(int B, int n, int side, unsigned long long seed, long long first, unsigned occ_threshold,
                           double a_in, double a_bg, double* a, hipStream_t st) {
  const dim3 g(n / kST, n / kST, B);
  hipLaunchKernelGGL(k_sample_lattice, g, dim3(kBlock), 0, st, n, side, (unsigned)(seed & 0xFFFFFFFFull),
                     (unsigned)(seed >> 32), first, occ_threshold, a_in, a_bg, a, (const uint8_t*)nullptr);
}

void launch_sample_fixed(int B, int n, int side, unsigned long long seed, long long first, int K, double a_in,
                         double a_bg, uint8_t* occ, double* a, hipStream_t st) {
  const long long n2 = (long long)n * n;
  long long zb = (B * n2 + kBlock - 1) / kBlock;
  if (zb > 4096) zb = 4096;
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)zb), dim3(kBlock), 0, st, occ, B * n2);
  const long long threads = (long long)B * K;
  if (threads > 0)
    hipLaunchKernelGGL(k_fixed_centres, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, B, n2,
                       K, (unsigned)(seed & 0xFFFFFFFFull), (unsigned)(seed >> 32), first, occ);
  const dim3 g(n / kST, n / kST, B);
  hipLaunchKernelGGL(k_sample_lattice, g, dim3(kBlock), 0, st, n, side, 0u, 0u, first, 0u, a_in, a_bg, a,
                     (const uint8_t*)occ);
}

}  // namespace rve
