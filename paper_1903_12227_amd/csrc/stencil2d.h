// The two-dimensional operators at one node (grid units), shared by the
// batched operator apply and the single-workgroup solver.
#pragma once

#include <hip/hip_runtime.h>

namespace rve {

constexpr double kSixth = 1.0 / 6.0;
constexpr double kThird = 1.0 / 3.0;
constexpr double kTwoThirds = 2.0 / 3.0;

// Node (p,q) touches cells (p-1,q-1)=a00, (p-1,q)=a01, (p,q-1)=a10,
// (p,q)=a11. Each cell contributes (a_e/6)(4 u_self - u_x1nbr - u_x2nbr -
// 2 u_diag): the consistent Q1 element matrix a_e (k (x) m + m (x) k) of
// the rank-2 Kronecker form (Sec. 3.2). Collected per neighbour:
//   centre (2/3)(a00+a01+a10+a11); (p+-1, q): -(a10+a11)/6, -(a00+a01)/6;
//   (p, q+-1): -(a01+a11)/6, -(a00+a10)/6; diagonals -a_e/3 of the one
//   cell they share with the node.
template <class T>
__device__ inline T q1_apply(T a00, T a01, T a10, T a11, const T (&um)[3], const T (&uc)[3], const T (&up)[3]) {
  T v = (T)kTwoThirds * ((a00 + a01) + (a10 + a11)) * uc[1];
  v -= (T)kSixth * ((a10 + a11) * up[1] + (a00 + a01) * um[1] + (a01 + a11) * uc[2] + (a00 + a10) * uc[0]);
  v -= (T)kThird * (a11 * up[2] + a01 * um[2] + a10 * up[0] + a00 * um[0]);
  return v;
}

// Lumped five-point operator (Sec. 3.2, eqns. Lapl_Kron_D and As_Kron with
// cell blocks): each edge carries the mean of the two cells beside it, so at
// node (p, q), with the same cells and rows as q1_apply,
//   (A u) = [(a10+a11)(u - u(p+1,q)) + (a00+a01)(u - u(p-1,q))
//            + (a01+a11)(u - u(p,q+1)) + (a00+a10)(u - u(p,q-1))] / 2.
template <class T>
__device__ inline T fd5_apply(T a00, T a01, T a10, T a11, const T (&um)[3], const T (&uc)[3], const T (&up)[3]) {
  const T c = uc[1];
  return (T)0.5 * ((a10 + a11) * (c - up[1]) + (a00 + a01) * (c - um[1]) + (a01 + a11) * (c - uc[2]) +
                   (a00 + a10) * (c - uc[0]));
}

}  // namespace rve
