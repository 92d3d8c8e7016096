// Host-side launchers of the librve kernels. Each kernel source file defines
// its kernels and the launchers below; the API layer calls only these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace rve {

// Device pointers and sizes of one equal-n batch of B realizations
// (S = dim B corrector systems, system s = dim b + i for direction i).
struct Work {
  int B = 0, n = 0, S = 0;
  int dim = 2;               // 2: n x n grids; 3: n x n x n grids (x3 contiguous)
  long long N2 = 0;          // nodes per system: n^dim
  const double* a = nullptr; // [B][n^dim] cells
  // two dimensions, FP64 apply: if every field of the batch takes only its
  // minimum and maximum value, one byte per cell (1 = maximum), which the
  // operator kernels read instead of a; else null
  const uint8_t* a8 = nullptr;
  double* x = nullptr;       // [S][n^dim] iterate (grid units)
  double* r = nullptr;       // residual
  // Search directions p and preconditioned residual z are FP64 when the
  // transform GEMMs are FP64 and FP32 otherwise (mixed modes); they only
  // steer the iteration, while x, r and q = A p stay FP64, so r = f - A x
  // holds to FP64 rounding in every mode.
  // The directions live in a ring of m_ring slots, [m_ring][S][n][n]: p_k is
  // written to slot k mod m_ring, and x is brought up to date only every
  // m_ring iterations, from the directions in the ring and their step
  // lengths alpha_hist[S][m_ring].
  void* pring = nullptr;
  int m_ring = 2;
  // pdirect = 1 (2D, 16-bit tile transforms, standard beta, FP64 apply): the
  // last transform forms the new direction p_{k+1} = z_{k+1} + beta_k p_k in
  // its epilogue (beta is known once the scaling transform's r.z partials are
  // summed) and writes it to ring slot k+1 mod m_ring; the operator apply then
  // reads p_k alone instead of z_k and p_{k-1}. The ring then has
  // RVE_DIRECTION_RING + 1 slots, since p_{k+1} is written one iteration
  // before the fold of the chunk that ends at k.
  int pdirect = 0;
  // pdirect with 16-bit transforms: the directions in the ring are BF16
  // instead of FP32 (the apply, the residual update and the fold read them
  // so; the last transform rounds p_{k+1} = z_{k+1} + beta_k p_k to BF16 once)
  int pdir16 = 0;
  int pdir_first = 0;   // pdirect: the apply before the first iteration (p_0 = z_0 into slot k mod m)
  double* alpha_hist = nullptr;
  double* q = nullptr;       // A p
  void* z = nullptr;
  void* rlo = nullptr;       // mixed modes: r rounded to the GEMM type, the first GEMM's input
  void* u1 = nullptr;        // transform intermediates, [S][n][n] of the GEMM type
  void* u2 = nullptr;
  int mixed = 0;             // 0: FP64 GEMMs; 1: FP32 GEMMs; 2: BF16 GEMMs; 3: FP16 GEMMs (scaled)
  // FP32 operator apply: a32 holds the coefficients in FP32, q is FP32, and
  // f (the mean-free right-hand sides) serves the periodic r = f - A x
  int sprec = 0;
  int scheme = 0;            // 0: consistent Q1 nine-point operator; 1: lumped five-point
  const float* a32 = nullptr;
  double* f = nullptr;
  int stencil = 0;           // operator-apply shape (stencil_choice_*)
  int ustencil = 0;          // shape of the recomputing residual update (qfree)
  int gemm_variant = 0;      // 0: 64 x 64 transform tiles; 1: 128 x 128 (16-bit, n % 128 == 0);
                             // 2: even/odd-folded 128 x 128 (BF16, n % 256 == 0);
                             // 3: as 1 with the operands loaded straight into LDS;
                             // 4: 256 x 128 (16-bit, n % 256 == 0); 5: 256 x 256
  SysState* sys = nullptr;   // [S]
  RealState* real = nullptr; // [B]
  double* part_pq = nullptr;   // [S][P] partial sums of p.Ap
  double* part_rr = nullptr;   // [S][P] partial sums of r.r
  double* part_rzo = nullptr;  // [S][P] partial sums of r_new.z_old (flexible beta)
  double* part_rz = nullptr;   // [S][P] partial sums of r.z
  double* part_misc = nullptr; // [B][P][kMiscNV] per-realization partials
  // Shared by all batches of one solve: the iteration counter k (advanced on
  // the device after each iteration, so a captured chunk of iterations can be
  // replayed unchanged) and the per-iteration counts of systems still
  // iterating (count[k]).
  int* kiter = nullptr;
  int* count = nullptr;
  int P_tile = 0;   // workgroups per realization of the RHS / A_hom / gradient kernels
  int P_st = 0;     // workgroups per realization of the operator apply
  int P_vec = 0;    // workgroups per system of the vector kernels
  // qfree = 1 (two dimensions, FP64 operator apply): the fused apply does not
  // store q = A p and the residual update recomputes it, in a tile shape of
  // its own (ustencil); its r.r / r.z_old partials then number
  // stencil_tiles_per_realization(n, ustencil) per system, else P_vec
  int qfree = 0;
  int P_rr = 0;
  int P_gemm = 0;   // output tiles per system of the transform GEMMs
};

constexpr int kMiscNV = 9;
constexpr int kMiscNV3 = 18;   // per-realization partials of the three-dimensional kernels

// Elementwise and stencil kernels (kernels_vec.hip).
void launch_init_state(const Work& w, hipStream_t st);
// code[b][e] = (a == max a of b); *not_two_valued |= 1 if a cell of the batch
// equals neither its realization's minimum nor its maximum (w.N2 % 4 == 0;
// after launch_scalar_init)
void launch_encode_two_valued(const Work& w, uint8_t* code, int* not_two_valued, hipStream_t st);
void launch_ctl_reset(int* kiter, int* count, int count_len, hipStream_t st);
void launch_rhs(const Work& w, hipStream_t st);
void launch_scalar_init(const Work& w, hipStream_t st);
void launch_meansub(const Work& w, hipStream_t st);
void launch_scalar_fnorm(const Work& w, hipStream_t st);
// alpha_k = r.z / p.Ap from the operator-apply partials; also kept in
// alpha_hist for the deferred x update.
void launch_scalar_alpha(const Work& w, hipStream_t st);
// stopping test of iteration k; counts the systems that go on in count[k]
void launch_scalar_conv(const Work& w, double tol, int maxit, hipStream_t st);
void launch_scalar_beta(const Work& w, int flexible, int first, hipStream_t st, int* advance = nullptr);
// the shared iteration counter += 1 (one thread)
void launch_advance(int* kiter, hipStream_t st);
void launch_round_lo(const Work& w, hipStream_t st);
// Fused direction step + operator apply of the current PCG iteration in the
// shape w.stencil (w.P_st must equal stencil_tiles_per_realization(n,
// w.stencil)). probe = 1, only at iteration 0 and only for timing, reads the
// previous direction's ring slot like a later iteration (outputs are then
// rewritten by the real iteration 0).
void launch_stencil_fused(const Work& w, hipStream_t st, int probe = 0);
// Operator-apply shapes, encoded as c = V + 8 (H / 16) + 64 (D - 1) for D in
// {1, 2} and V + 8 (H / 16) + 128 for D = 4: V in {1, 2, 4} columns per lane,
// H in {16, 32, 64} rows per wave strip, D rows of loads in flight per wave;
// valid when the 64V x 4H workgroup tile divides the n x n grid.
int stencil_choice_default(int n);
bool stencil_choice_valid(int n, int c);
inline int stencil_choice_V(int c) { return c & 7; }
inline int stencil_choice_H(int c) { return 16 * ((c >> 3) & 7); }
inline int stencil_choice_D(int c) { return (c & 128) ? 4 : 1 + ((c >> 6) & 1); }
int stencil_tiles_per_realization(int n, int c);
// probe = 1 (recomputing update only, before iteration 0, for timing): r is
// rewritten unchanged
void launch_update_r(const Work& w, int flexible, hipStream_t st, int probe = 0);
// residual replacement r = f - A x (FP64) of the FP32 operator apply
void launch_replace_r(const Work& w, hipStream_t st);
void launch_to_f32(const double* in, float* out, long long total, hipStream_t st);
// x += alpha_j p_j in increasing j (the order of the plain recurrence) over
// the directions of each system still in the ring: final = 0 at the start of
// iteration k = c m (directions k-m .. k-1), final = 1 after the last
// iteration (directions since the last multiple of m).
void launch_fold_x(const Work& w, int final, hipStream_t st);
constexpr int kRing = 8;   // direction ring length (iterations per x update)
// BF16 directions (Work::pdir16) on grids up to kDir16MaxN and for fields of
// contrast (max a / min a) up to kDir16MaxContrast: beyond either the longer
// iteration accumulates the lost conjugacy (n = 4096: a stall near 2e-7; at
// n = 512 whole solves gain 6-8 % at contrast 10, 4-6 % at 20, 1-6 % at 30
// and lose 5-12 % at 100)
constexpr int kDir16MaxN = 512;
constexpr double kDir16MaxContrast = 20.0;
void launch_widen(const float* in, double* out, long long total, hipStream_t st);
void launch_ahom(const Work& w, hipStream_t st);
void launch_scalar_ahom(const Work& w, double* ahom, double* ahom_flux, hipStream_t st);
void launch_phi_out(const Work& w, double* phi, double h, hipStream_t st);
void launch_finalize(const Work& w, int* iters, double* relres, int* status, hipStream_t st);
// Per-cell gradient; with want_in, per-tile partial sums over the inclusion
// cells (mask[e] != 0, or a_e == a_in when mask is null) into part
// [B][grad_tiles_per_realization(n)].
void launch_grad(int B, int n, int scheme, const double* a, const double* phi, double inv_h,
                 const double* G, double* grad, double a_in, const unsigned char* mask, double* part,
                 int want_in, hipStream_t st);
int grad_tiles_per_realization(int n);
// grad_in[b] = sum of realization b's partials; grad_in_sum (optional) = sum_b grad_in[b]
void launch_scalar_grad(int B, int n, const double* part, double* grad_in, double* grad_in_sum, hipStream_t st);
// a[b][e] = mask[b][e] ? a_in[b] : a_bg for B fields of N2 cells
void launch_field_from_mask(int B, long long N2, const unsigned char* mask, const double* a_in, double a_bg,
                            double* a, hipStream_t st);
void launch_stats(int N, double L, const double* ahom, double* out, hipStream_t st);
void launch_apply_stencil(int B, int n, int scheme, const double* a, const double* u, double* out,
                          hipStream_t st);

// Three-dimensional corrector problems (kernels_3d.hip). Cells and nodes
// [n][n][n], x3 contiguous; cell (i, j, k) spans nodes i..i+1, j..j+1,
// k..k+1 (mod n). The launchers of the dimension-specific steps above
// (RHS, scalar_init, fused operator apply, A_hom, finalize) forward here
// when w.dim == 3; the per-system vector kernels serve both dimensions.
constexpr int kStrip3 = 16;   // planes per wave strip of the 3D tile kernels
// workgroups per system (operator apply) or realization (RHS, A_hom) of the
// 3D tile kernels: 64 x3-columns x 4 x2-rows x kStrip3 x1-planes each
__host__ __device__ inline int tiles3(int n) { return (n / kWave) * (n / 4) * (n / kStrip3); }
void launch_rhs3(const Work& w, hipStream_t st);
void launch_scalar_init3(const Work& w, hipStream_t st);
void launch_stencil3_fused(const Work& w, hipStream_t st, int probe);
void launch_apply_stencil3(int B, int n, const double* a, const double* u, double* out, hipStream_t st);
void launch_ahom3(const Work& w, hipStream_t st);
void launch_scalar_ahom3(const Work& w, double* ahom, double* ahom_flux, hipStream_t st);
void launch_finalize3(const Work& w, int* iters, double* relres, int* status, hipStream_t st);

// Single-workgroup PCG (kernels_small.hip): the whole iteration of each
// system in one launch, for w.dim == 2, n == 64, FP64 transforms and apply.
// Expects the state the solver's set-up leaves (r = f - mean f, x = 0,
// fnorm, a0, active flags); writes x, iters, relres and status.
bool small_solver_fits(const Work& w);
void launch_pcg_small(const Work& w, const double* q64, const double* einv64, double tol, int maxit,
                      hipStream_t st);

// On-device sampling of the inclusion model (kernels_sample.hip): B fields
// [B][n][n] for realizations first .. first + B - 1.
bool sample_side_valid(int n, int side);
void launch_sample_lattice(int B, int n, int side, unsigned long long seed, long long first, unsigned occ_threshold,
                           double a_in, double a_bg, double* a, hipStream_t st);
// the fixed-count law: K centres per realization; occ is scratch of B n^2 bytes
void launch_sample_fixed(int B, int n, int side, unsigned long long seed, long long first, int K, double a_in,
                         double a_bg, uint8_t* occ, double* a, hipStream_t st);

// +-1 probe vectors from Philox4x32-10 words (kernels_sample.hip): total
// entries, at most 2^39 * 128.
void launch_probes(long long total, unsigned long long seed, double* v, hipStream_t st);

// Spectral density by Chebyshev moments (kernels_dos.hip).
int dos_vec_tiles(long long N2);
// out[0] = max of the positive cells, out[1] = count of cells <= 0 or NaN,
// over `total` cells; part holds 2 field_max_blocks(total) doubles
int field_max_blocks(long long total);
void launch_field_max(const double* a, long long total, double* part, double* out, hipStream_t st);
void launch_dos_moments(int B, int n, int scheme, const double* a, int nv, double* W, double* Wp, double* AW,
                        double lmax, int K, double* part, double* mu, hipStream_t st);
void launch_dos_eval(int B, int nv, int K, const double* mu, double lmax, double eta, int Q, int nt,
                     const double* t, double* S, double* phi, hipStream_t st);

// Transform GEMMs of the preconditioner (kernels_gemm.hip).
enum GemmPrec { kGemmF64 = 0, kGemmF32 = 1, kGemmBF16 = 2, kGemmF16 = 3 };
struct GemmTables {
  const void* q = nullptr;        // [n][n] Hartley matrix in the GEMM operand type
  const double* einv64 = nullptr; // [n][n] 1/E, (0,0) entry 0
  const float* einv32 = nullptr;
  const __bf16* ch16 = nullptr;   // [n/2][n/2] cos(2 pi k t/n)/sqrt(n), BF16 (folded transform)
  const __bf16* sh16 = nullptr;   // [n/2][n/2] sin(2 pi k t/n)/sqrt(n), BF16
  const double* einv3_64 = nullptr;  // [n][n][n] 1/E of the 3D operator (w.dim == 3), (0,0,0) entry 0
  const float* einv3_32 = nullptr;
  // FP16 transforms: the residual copy is scaled per system (SysState::lo_scale),
  // einv32 / einv3_32 hold E_min / E and the last transform unscales
  double emin = 1.0;
  // [n] sin^2(pi k / n), from which the 16-bit 2D transforms form 1/E
  // (fd = 1: the five-point symbol) instead of reading an n x n table
  const float* sin2 = nullptr;
  int fd = 0;
  // compute units: the 256 x 256 16-bit transform runs one workgroup per CU
  // that loops over tiles (0: one workgroup per tile)
  int cus = 0;
};
size_t gemm_elem_size(int prec);
// z = (a0 A_Delta)^+ r for every active system, with partial sums of r.z.
// In the mixed modes the first transform reads w.rlo, which must hold r in
// the GEMM precision; w.P_gemm must equal
// gemm_tiles_per_system(n, prec, w.gemm_variant).
// phase < 0 launches all four transforms; 0..3 only that one (in order).
// With w.dim == 3 there are six transforms (phases 0..5), in 64 x 64 tiles.
void launch_precond(const Work& w, int prec, const GemmTables& t, hipStream_t st, int phase = -1);
int precond_phases(const Work& w);
int gemm_tiles_per_system3(int n);
bool gemm_variant_valid(int n, int prec, int variant);
// the 16-bit tile variants, whose last transform can write the next search
// direction (Work::pdirect)
bool gemm_variant_writes_direction(int n, int prec, int variant);
int gemm_tiles_per_system(int n, int prec, int variant);
int gemm_tiles_per_system_max(int n);

}  // namespace rve
