// Three-dimensional corrector problems (d = 3): the problem setting of Sec. 2
// is unchanged, and the Kronecker construction of Sec. 3.2 extends to
// three-factor products (eqn. As_Kron_d). Grid units (h = 1); cells and
// nodes are [n][n][n] with x3 contiguous, cell (i, j, k) spans nodes
// i..i+1, j..j+1, k..k+1 (mod n), and realization b owns the systems
// s = 3b + d (direction e_d).
//
// Trilinear element: the unit-cube stiffness is k (x) m (x) m + m (x) k (x) m
// + m (x) m (x) k with k = [[1,-1],[-1,1]] and m = [[2,1],[1,2]]/6. Its
// entries depend only on how many coordinates two corners differ in: 1/3
// (none), 0 (one), -1/12 (two or three). So the operator at node P sums, over
// the eight cells c around P with corner signs (sx, sy, sz) pointing from P
// into c,
//   (A u)(P) = sum_c a_c / 12 * (4 u(P) - u(P + (sx,sy,0)) - u(P + (sx,0,sz))
//                                - u(P + (0,sy,sz)) - u(P + (sx,sy,sz))),
// a 21-point stencil (the six axis neighbours carry weight zero).
//
// Tile kernels: 256 threads per workgroup; lane = x3 index within a 64-wide
// column block, the four waves take four consecutive x2 rows, and each wave
// slides a register window along x1 over a strip of kStrip3 planes, so a
// value is loaded from HBM about once per strip (plus a halo plane); the
// operator apply stages each plane with its x2 / x3 halo in LDS, the RHS and
// A_hom kernels take the neighbours from cache lines just fetched.
// One-dimensional grid with the XCD-contiguous remap of the 2D kernels.
// Reductions go through per-workgroup partials finished in a fixed order.
#include "launch.h"

namespace rve {

namespace {

constexpr double kTwelfth = 1.0 / 12.0;

struct Tile3 {
  int k, j, i0;   // this lane's x3 index and x2 row, first plane of the strip
  int unit;       // system (operator apply) or realization (RHS, A_hom)
  int tile;       // tile index within the unit
};

__device__ inline Tile3 tile3_of(int n) {
  const unsigned T = gridDim.x, L = blockIdx.x;
  const unsigned t = (T & 7u) ? L : (L & 7u) * (T >> 3) + (L >> 3);
  const int gk = n / kWave, gj = n / 4;
  const unsigned per = (unsigned)(gk * gj * (n / kStrip3));
  Tile3 r;
  r.unit = (int)(t / per);
  r.tile = (int)(t % per);
  const int kx = r.tile % gk, jy = (r.tile / gk) % gj, ih = r.tile / (gk * gj);
  r.k = kx * kWave + (int)(threadIdx.x & 63);
  r.j = jy * 4 + (int)(threadIdx.x >> 6);
  r.i0 = ih * kStrip3;
  return r;
}

// Galerkin right-hand sides f_d(P) = -sum_c a_c int_c d(psi_P)/dx_d: the
// x_d-derivative of a corner function integrates to +-1/4 over its cell, so
// f_d(P) = (sum of the four cells on the + side along x_d - the four on the
// - side) / 4. Also per-tile sums of f_1..f_3 and of a (each cell once, as
// the cell (i, j, k) of node (i, j, k)), min / max of a and a count of cells
// with a <= 0 or NaN.
__global__ void __launch_bounds__(kBlock) k_rhs3(const double* __restrict__ a, double* __restrict__ r, int n,
                                                  double* __restrict__ part) {
  __shared__ double sh[4 * 5];
  __shared__ double mm[8];
  const Tile3 tl = tile3_of(n);
  const int b = tl.unit, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long N3 = (long long)n * n * n, NN = (long long)n * n;
  const double* A = a + (long long)b * N3;
  double* F = r + 3LL * b * N3;
  const int k = tl.k, km = wrap_dec(k, n), j = tl.j;
  const long long row[2] = {(long long)wrap_dec(j, n) * n, (long long)j * n};
  double ac[2][2][2];   // cells [plane i-1, i][row j-1, j][col k-1, k]
  auto load_cells = [&](int ci, double (&c)[2][2]) {
    const long long pl = (long long)ci * NN;
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      c[y][0] = A[pl + row[y] + km];
      c[y][1] = A[pl + row[y] + k];
    }
  };
  load_cells(wrap_dec(tl.i0, n), ac[0]);
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double amin = 1.0e308, amax = -1.0e308;
  for (int t = 0; t < kStrip3; ++t) {
    const int i = tl.i0 + t;
    load_cells(i, ac[1]);
    double px = 0.0, mx = 0.0, py = 0.0, my = 0.0, pz = 0.0, mz = 0.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) {
          const double v = ac[x][y][z];
          if (x) px += v; else mx += v;
          if (y) py += v; else my += v;
          if (z) pz += v; else mz += v;
        }
    const double f1 = 0.25 * (px - mx), f2 = 0.25 * (py - my), f3 = 0.25 * (pz - mz);
    const long long o = (long long)i * NN + row[1] + k;
    F[o] = f1;
    F[N3 + o] = f2;
    F[2 * N3 + o] = f3;
    const double own = ac[1][1][1];
    s[0] += f1;
    s[1] += f2;
    s[2] += f3;
    s[3] += own;
    s[4] += !(own > 0.0) ? 1.0 : 0.0;   // also catches NaN
    amin = fmin(amin, own);
    amax = fmax(amax, own);
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int z = 0; z < 2; ++z) ac[0][y][z] = ac[1][y][z];
  }
  const double vmin = wave_min(amin), vmax = wave_max(amax);
  block_sum<5>(s, sh);
  if (lane == 0) {
    mm[w] = vmin;
    mm[4 + w] = vmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int P = tiles3(n);
    double* o = part + ((long long)b * P + tl.tile) * kMiscNV3;
    o[0] = s[0];
    o[1] = s[1];
    o[2] = s[2];
    o[3] = s[3];
    o[4] = fmin(fmin(mm[0], mm[1]), fmin(mm[2], mm[3]));
    o[5] = fmax(fmax(mm[4], mm[5]), fmax(mm[6], mm[7]));
    o[6] = s[4];
  }
}

// Per realization (one wave): the coefficient statistics, a0, and the means
// of the three raw right-hand sides.
__global__ void k_scalar_init3(SysState* sys, RealState* real, const double* __restrict__ part, int P, int n,
                               int scaled) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double f[3] = {0.0, 0.0, 0.0}, sa = 0.0, bad = 0.0, mn = 1.0e308, mx = -1.0e308;
  for (int t = lane; t < P; t += kWave) {
    const double* o = part + ((long long)b * P + t) * kMiscNV3;
    f[0] += o[0];
    f[1] += o[1];
    f[2] += o[2];
    sa += o[3];
    mn = fmin(mn, o[4]);
    mx = fmax(mx, o[5]);
    bad += o[6];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) f[d] = wave_sum(f[d]);
  sa = wave_sum(sa);
  bad = wave_sum(bad);
  mn = wave_min(mn);
  mx = wave_max(mx);
  if (lane == 0) {
    const double N3 = (double)n * (double)n * (double)n;
    RealState rs;
    rs.a_sum = sa;
    rs.a_min = mn;
    rs.a_max = mx;
    rs.inv_a0 = 2.0 / (mx + mn);
    rs.bad = (int)bad;
    rs.pad = 0;
    real[b] = rs;
    const int valid = (bad == 0.0) && isfinite(sa);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sys[3 * b + d].mean_f = f[d] / N3;
      sys[3 * b + d].valid = valid;
      // scaled copies: |f - mean f| <= 2 (a_max - a_min)
      if (scaled && mx > mn) sys[3 * b + d].lo_next = 0.25 / (mx - mn);
    }
  }
}

// q = A u over one system per workgroup (coefficients of realization
// unit / spr).
// FUSED: u is the new search direction p_k = z_k + beta_{k-1} p_{k-1}
// (p_0 = z_0), rounded to its storage type PT before use; p_k goes to ring
// slot k mod m (k read from *kiter), p_{k-1} comes from slot (k - 1) mod m;
// q and partial sums of p_k.q are written for active systems. probe = 1
// (timing at k = 0 only) reads p_{k-1} as a later iteration would.
// Not FUSED: u = p_in, spr = 1 (one operand per realization).
//
// Each step of the strip stages the next operand plane of the workgroup's
// region (its 4 x 64 nodes plus a one-node halo: 6 x 66, the direction
// formed once per node) and the current cell plane (5 x 65) in LDS, double
// buffered so one barrier per step suffices; each lane then reads its 3 x 3
// neighbourhood and 2 x 2 cells from LDS and keeps the two previous planes
// in registers.
template <bool FUSED, class PT>
__global__ void __launch_bounds__(kBlock) k_stencil3(const double* __restrict__ a, const PT* p_in, PT* ring,
                                                      long long slot_stride, int m, const int* kiter,
                                                      const PT* __restrict__ z, double* __restrict__ q, int n,
                                                      int spr, const SysState* sys, double* __restrict__ part,
                                                      int probe) {
  constexpr int CW = kWave + 2, PE = 6 * CW;   // staged operand plane: rows j0-1 .. j0+4, cols k0-1 .. k0+64
  constexpr int AC = kWave + 1, AE = 5 * AC;   // staged cell plane: rows j0-1 .. j0+3, cols k0-1 .. k0+63
  static_assert(PE <= 2 * kBlock && AE <= 2 * kBlock, "two staged elements per thread");
  __shared__ double su[2][PE];
  __shared__ double sa[2][AE];
  __shared__ double sh[4];
  const Tile3 tl = tile3_of(n);
  const int s = tl.unit;
  int first = 0;
  double beta = 0.0;
  const PT* p_old = p_in;
  PT* p_new = nullptr;
  if constexpr (FUSED) {
    if (!sys[s].active) return;   // uniform over the workgroup
    const int it = kiter[0];
    first = it == 0 && !probe;
    p_new = ring + (long long)(it % m) * slot_stride;
    p_old = ring + (long long)((it + m - 1) % m) * slot_stride;
    beta = first ? 0.0 : sys[s].beta;
  }
  const long long N3 = (long long)n * n * n, NN = (long long)n * n;
  const double* A = a + (long long)(s / spr) * N3;
  const PT* Po = p_old + (long long)s * N3;
  const PT* Zs = FUSED ? z + (long long)s * N3 : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k0 = tl.k - lane, j0 = tl.j - w;

  // in-plane offsets of this thread's staged elements: element tid (always
  // inside both regions) and element tid + 256 (inside for the first
  // PE - 256 / AE - 256 threads; elsewhere the offset is 0, so the load stays
  // in bounds, and the LDS write is skipped)
  int po[2], ao[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * kBlock;
    int gj = j0 - 1 + e / CW, gk = k0 - 1 + e % CW;
    gj = gj < 0 ? gj + n : gj >= n ? gj - n : gj;
    gk = gk < 0 ? gk + n : gk >= n ? gk - n : gk;
    po[u] = e < PE ? gj * n + gk : 0;
    int hj = j0 - 1 + e / AC, hk = k0 - 1 + e % AC;
    hj = hj < 0 ? hj + n : hj;
    hk = hk < 0 ? hk + n : hk;
    ao[u] = e < AE ? hj * n + hk : 0;
  }
  const bool p1 = tid + kBlock < PE, a1 = tid + kBlock < AE;
  // raw loads of one operand plane and one cell plane, kept in registers
  // (issued a step ahead of their use, so they stay in flight across the
  // barrier and the arithmetic of the current step). The previous direction
  // is loaded at k = 0 too (its slot holds earlier data) and then not used.
  struct Raw {
    PT z[2], p[2];
    double a[2];
  };
  auto load_op = [&](int pi, Raw& R) {
    const PT* pp = Po + (long long)pi * NN;
    const PT* zp = FUSED ? Zs + (long long)pi * NN : nullptr;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if constexpr (FUSED) R.z[u] = zp[po[u]];
      R.p[u] = pp[po[u]];
    }
  };
  auto load_cells = [&](int ci, Raw& R) {
    const double* ap = A + (long long)ci * NN;
#pragma unroll
    for (int u = 0; u < 2; ++u) R.a[u] = ap[ao[u]];
  };
  auto cook = [&](const Raw& R, int u) -> double {
    if constexpr (FUSED) {
      // p_k is rounded to PT before use, so q = A p_k, p_k.q and the later
      // x += alpha p_k all see the same direction
      const double pk = (double)(PT)fma(beta, (double)R.p[u], (double)R.z[u]);
      return first ? (double)R.z[u] : pk;
    } else {
      return (double)R.p[u];
    }
  };
  auto stage_op = [&](const Raw& R, int buf) {
    su[buf][tid] = cook(R, 0);
    if (p1) su[buf][tid + kBlock] = cook(R, 1);
  };
  auto stage_cells = [&](const Raw& R, int buf) {
    sa[buf][tid] = R.a[0];
    if (a1) sa[buf][tid + kBlock] = R.a[1];
  };
  auto read_plane = [&](int buf, double (&u)[3][3]) {
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int x = 0; x < 3; ++x) u[y][x] = su[buf][(w + y) * CW + lane + x];
  };
  auto read_cells = [&](int buf, double (&c)[2][2]) {
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int x = 0; x < 2; ++x) c[y][x] = sa[buf][(w + y) * AC + lane + x];
  };

  double u[3][3][3];    // operand [plane i-1, i, i+1][row j-1, j, j+1][col k-1, k, k+1]
  double ac[2][2][2];   // cells [plane i-1, i][row j-1, j][col k-1, k]
  // LDS buffer b is rewritten only after every thread has passed the barrier
  // that follows its last read of b (the barrier of the next step)
  Raw R;
  load_op(wrap_dec(tl.i0, n), R);
  load_cells(wrap_dec(tl.i0, n), R);
  stage_op(R, 0);
  stage_cells(R, 0);
  load_op(tl.i0, R);
  __syncthreads();
  read_plane(0, u[0]);
  read_cells(0, ac[0]);
  stage_op(R, 1);
  load_op(wrap_inc(tl.i0, n), R);
  load_cells(tl.i0, R);
  __syncthreads();
  read_plane(1, u[1]);
  double d = 0.0;
  for (int t = 0; t < kStrip3; ++t) {
    const int i = tl.i0 + t, buf = t & 1;
    stage_op(R, buf);   // operand plane i + 1
    stage_cells(R, buf);   // cell plane i
    if (t + 1 < kStrip3) {
      load_op(wrap_inc(i + 1, n), R);
      load_cells(i + 1, R);
    }
    __syncthreads();
    read_plane(buf, u[2]);
    read_cells(buf, ac[1]);
    const double c = u[1][1][1];
    double qv = 0.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int zz = 0; zz < 2; ++zz) {
          const int ix = 2 * x, iy = 2 * y, iz = 2 * zz;
          qv += ac[x][y][zz] * (4.0 * c - ((u[ix][iy][1] + u[ix][1][iz]) + (u[1][iy][iz] + u[ix][iy][iz])));
        }
    qv *= kTwelfth;
    const long long o = (long long)s * N3 + (long long)i * NN + (long long)tl.j * n + tl.k;
    q[o] = qv;
    if constexpr (FUSED) {
      p_new[o] = (PT)c;
      d += c * qv;
    }
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        u[0][y][x] = u[1][y][x];
        u[1][y][x] = u[2][y][x];
      }
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int x = 0; x < 2; ++x) ac[0][y][x] = ac[1][y][x];
  }
  if constexpr (FUSED) {
    double dd[1] = {d};
    block_sum<1>(dd, sh);
    if (threadIdx.x == 0) part[(long long)s * tiles3(n) + tl.tile] = dd[0];
  }
}

// Mass-weighted product of two 2 x 2 arrays of edge differences: the
// integral over the cell of the product of their bilinear interpolants,
// sum_{t,t'} A[t] B[t'] m[t0][t0'] m[t1][t1'] with m = [[2,1],[1,2]]/6.
__device__ inline double edge_dot(const double (&A)[2][2], const double (&B)[2][2]) {
  const double same = (A[0][0] * B[0][0] + A[0][1] * B[0][1]) + (A[1][0] * B[1][0] + A[1][1] * B[1][1]);
  const double one = ((A[0][0] * B[0][1] + A[0][1] * B[0][0]) + (A[1][0] * B[1][1] + A[1][1] * B[1][0])) +
                     ((A[0][0] * B[1][0] + A[1][0] * B[0][0]) + (A[0][1] * B[1][1] + A[1][1] * B[0][1]));
  const double both = (A[0][0] * B[1][1] + A[1][1] * B[0][0]) + (A[0][1] * B[1][0] + A[1][0] * B[0][1]);
  return (4.0 * same + 2.0 * one + both) * (1.0 / 36.0);
}

// Per-tile partials, per cell e = (i, j, k) with the trilinear correctors x_d:
// [0..5]  a_e int_e (e_p + grad x_p).(e_q + grad x_q), (p, q) = 11 12 13 22 23 33;
// [6..14] a_e int_e (delta_pq + d_q x_p), row-major in (p, q);
// [15..17] x_d at node (i, j, k) (the sums give the means of the iterates).
__global__ void __launch_bounds__(kBlock) k_ahom3(const double* __restrict__ a, const double* __restrict__ x,
                                                   int n, double* __restrict__ part) {
  __shared__ double sh[4 * kMiscNV3];
  const Tile3 tl = tile3_of(n);
  const int b = tl.unit;
  const long long N3 = (long long)n * n * n, NN = (long long)n * n;
  const double* A = a + (long long)b * N3;
  const double* X = x + 3LL * b * N3;
  const int k = tl.k, j = tl.j;
  const int col[2] = {k, wrap_inc(k, n)};
  const long long row[2] = {(long long)j * n, (long long)wrap_inc(j, n) * n};
  double v[3][2][2][2];   // [system][plane i, i+1][row j, j+1][col k, k+1]
  auto load_plane = [&](int pi, int slot) {
    const long long pl = (long long)pi * NN;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) v[dd][slot][y][z] = X[dd * N3 + pl + row[y] + col[z]];
  };
  load_plane(tl.i0, 0);
  double acc[kMiscNV3];
#pragma unroll
  for (int t = 0; t < kMiscNV3; ++t) acc[t] = 0.0;
  for (int t = 0; t < kStrip3; ++t) {
    const int i = tl.i0 + t;
    load_plane(wrap_inc(i, n), 1);
    const double ae = A[(long long)i * NN + row[0] + k];
    // edge differences of each corrector along each axis, indexed by the
    // two transverse corner coordinates, and the cell means of its gradient
    double e[3][3][2][2], g[3][3];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
#pragma unroll
      for (int p0 = 0; p0 < 2; ++p0)
#pragma unroll
        for (int p1 = 0; p1 < 2; ++p1) {
          e[dd][0][p0][p1] = v[dd][1][p0][p1] - v[dd][0][p0][p1];
          e[dd][1][p0][p1] = v[dd][p0][1][p1] - v[dd][p0][0][p1];
          e[dd][2][p0][p1] = v[dd][p0][p1][1] - v[dd][p0][p1][0];
        }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        g[dd][ax] = 0.25 * ((e[dd][ax][0][0] + e[dd][ax][0][1]) + (e[dd][ax][1][0] + e[dd][ax][1][1]));
    }
    int slot = 0;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int qq = p; qq < 3; ++qq) {
        const double gg = (edge_dot(e[p][0], e[qq][0]) + edge_dot(e[p][1], e[qq][1])) + edge_dot(e[p][2], e[qq][2]);
        acc[slot++] += ae * ((p == qq ? 1.0 : 0.0) + g[qq][p] + g[p][qq] + gg);
      }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int qq = 0; qq < 3; ++qq) acc[6 + 3 * p + qq] += ae * ((p == qq ? 1.0 : 0.0) + g[p][qq]);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) acc[15 + dd] += v[dd][0][0][0];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) v[dd][0][y][z] = v[dd][1][y][z];
  }
  block_sum<kMiscNV3>(acc, sh);
  if (threadIdx.x == 0) {
    double* o = part + ((long long)b * tiles3(n) + tl.tile) * kMiscNV3;
#pragma unroll
    for (int t = 0; t < kMiscNV3; ++t) o[t] = acc[t];
  }
}

__global__ void k_scalar_ahom3(SysState* sys, const double* __restrict__ part, int P, int n,
                               double* __restrict__ ahom, double* __restrict__ ahom_flux) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double v[kMiscNV3];
#pragma unroll
  for (int t = 0; t < kMiscNV3; ++t) v[t] = 0.0;
  for (int t = lane; t < P; t += kWave) {
    const double* o = part + ((long long)b * P + t) * kMiscNV3;
#pragma unroll
    for (int u = 0; u < kMiscNV3; ++u) v[u] += o[u];
  }
#pragma unroll
  for (int t = 0; t < kMiscNV3; ++t) v[t] = wave_sum(v[t]);
  if (lane == 0) {
    const double inv = 1.0 / ((double)n * (double)n * (double)n);
    double* E = ahom + 9LL * b;
    int slot = 0;
    for (int p = 0; p < 3; ++p)
      for (int qq = p; qq < 3; ++qq) {
        E[3 * p + qq] = v[slot] * inv;
        E[3 * qq + p] = v[slot] * inv;
        ++slot;
      }
    if (ahom_flux) {
      double* F = ahom_flux + 9LL * b;
      for (int t = 0; t < 9; ++t) F[t] = v[6 + t] * inv;
    }
    for (int dd = 0; dd < 3; ++dd) sys[3 * b + dd].mean_x = v[15 + dd] * inv;
  }
}

__global__ void k_finalize3(const SysState* sys, int B, int* iters, double* relres, int* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int worst = 0;
  for (int dd = 0; dd < 3; ++dd) {
    const SysState& S = sys[3 * b + dd];
    if (iters) iters[3 * b + dd] = S.iters;
    if (relres) relres[3 * b + dd] = S.relres;
    // errors (negative codes) dominate; otherwise the larger warning code
    const int c = S.status;
    worst = (worst < 0 || c < 0) ? min(worst, c) : max(worst, c);
  }
  if (status) status[b] = worst;
}

}  // namespace

void launch_rhs3(const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs3, dim3((unsigned)(tiles3(w.n) * w.B)), dim3(kBlock), 0, st, w.a, w.r, w.n, w.part_misc);
}

void launch_scalar_init3(const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_init3, dim3(w.B), dim3(kWave), 0, st, w.sys, w.real, w.part_misc, tiles3(w.n), w.n,
                     (int)(w.mixed == 3));
}

void launch_stencil3_fused(const Work& w, hipStream_t st, int probe) {
  const dim3 g((unsigned)(tiles3(w.n) * w.S)), blk(kBlock);
  const long long slot = (long long)w.S * w.N2;
  if (w.mixed == 0)
    hipLaunchKernelGGL((k_stencil3<true, double>), g, blk, 0, st, w.a, (const double*)nullptr, (double*)w.pring,
                       slot, w.m_ring, (const int*)w.kiter, (const double*)w.z, w.q, w.n, 3, w.sys, w.part_pq,
                       probe);
  else
    hipLaunchKernelGGL((k_stencil3<true, float>), g, blk, 0, st, w.a, (const float*)nullptr, (float*)w.pring, slot,
                       w.m_ring, (const int*)w.kiter, (const float*)w.z, w.q, w.n, 3, w.sys, w.part_pq, probe);
}

void launch_apply_stencil3(int B, int n, const double* a, const double* u, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_stencil3<false, double>), dim3((unsigned)(tiles3(n) * B)), dim3(kBlock), 0, st, a, u,
                     (double*)nullptr, 0LL, 1, (const int*)nullptr, (const double*)nullptr, out, n, 1,
                     (const SysState*)nullptr, (double*)nullptr, 0);
}

void launch_ahom3(const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_ahom3, dim3((unsigned)(tiles3(w.n) * w.B)), dim3(kBlock), 0, st, w.a, w.x, w.n,
                     w.part_misc);
}

void launch_scalar_ahom3(const Work& w, double* ahom, double* ahom_flux, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_ahom3, dim3(w.B), dim3(kWave), 0, st, w.sys, w.part_misc, tiles3(w.n), w.n, ahom,
                     ahom_flux);
}

void launch_finalize3(const Work& w, int* iters, double* relres, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize3, dim3((w.B + kBlock - 1) / kBlock), dim3(kBlock), 0, st, w.sys, w.B, iters,
                     relres, status);
}

}  // namespace rve
