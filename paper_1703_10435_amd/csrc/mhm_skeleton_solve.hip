// Skeleton solve on the device: preconditioned MINRES on the symmetric
// indefinite system of eq. (6), [[M, B^T], [B, 0]] [lambda; u_0] = [E; F].
//
// The element blocks M_e are negative definite, so the multiplier block is
// negative (semi-)definite and the u_0 block is zero: a saddle point.  The
// paper solves it with sparse direct solvers and names hybrid
// direct-iterative solvers as future work (Section 6).  Here it is solved
// iteratively with MINRES (Paige and Saunders' minimal-residual method for
// symmetric indefinite systems, the preconditioned form with an SPD
// preconditioner), preconditioned by the block diagonal
//   P = diag(|diag(M)|, diag(B |diag(M)|^-1 B^T)),
// the Jacobi scaling of the multiplier block and the diagonal of the
// approximate Schur complement for the u_0 rows.
//
// One MINRES step is three launches: the CSR product with its dot product,
// the Lanczos vector with the next dot product, and the scalar recurrences
// together with the update of the direction and the iterate.  Dot products
// are reduced in two stages through per-workgroup partials (no atomics),
// so the iteration is deterministic.  Chunks of 16 steps are captured once
// in a HIP graph and replayed; the host reads the residual estimate after
// each chunk to stop.
#include <algorithm>

#include "mhm_kernels.h"

namespace mhm {
namespace {

constexpr int SV_THREADS = 256;
constexpr int SV_MAX_BLOCKS = 1024;
constexpr int ROW_LANES = 8;   // lanes per CSR row in the products

// scalar slots
enum : int {
  SC_GAMMA = 0,    // gamma_j
  SC_GAMMA_P,      // gamma_{j-1} (0 before the first step)
  SC_C, SC_C_P,    // c_j, c_{j-1}
  SC_S, SC_S_P,    // s_j, s_{j-1}
  SC_ETA,          // eta (signed residual estimate)
  SC_ETA0,         // gamma_1
  SC_A1, SC_A2, SC_A3,   // alpha_1..3 of the current step
  SC_XCOEF,        // c_{j+1} eta_old: weight of w_{j+1} in the iterate
  SC_DONE,         // 1 once the Lanczos process has broken down (exact solution)
  SC_RES,          // |eta| / gamma_1
  SC_STEPS,        // steps taken
  SC_COUNT
};

__device__ __forceinline__ double block_reduce(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

// Sum of the first `nb` partials, identical in every workgroup that asks.
__device__ __forceinline__ double sum_partials(const double* part, int nb, double* red) {
  double v = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) v += part[k];
  return block_reduce(v, red);
}

// One CSR row by ROW_LANES lanes (consecutive lanes, coalesced entries).
__device__ __forceinline__ double row_dot(const int32_t* rp, const int32_t* ci, const double* va, const double* x,
                                          int row, int sub) {
  double v = 0.0;
  for (int k = rp[row] + sub; k < rp[row + 1]; k += ROW_LANES) v += va[k] * x[ci[k]];
#pragma unroll
  for (int o = ROW_LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// d_i = |M_ii| for multiplier rows (1 if zero); then, for the u_0 rows,
// d_t = sum_j B_tj^2 / d_j (1 if zero).  Stored as 1 / d.
__global__ void __launch_bounds__(SV_THREADS) k_prec_lambda(int n_lambda, const int32_t* rp, const int32_t* ci,
                                                            const double* va, double* dinv) {
  for (int i = blockIdx.x * SV_THREADS + threadIdx.x; i < n_lambda; i += gridDim.x * SV_THREADS) {
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d = fabs(va[k]);
    dinv[i] = d > 0.0 ? 1.0 / d : 1.0;
  }
}
__global__ void __launch_bounds__(SV_THREADS) k_prec_u0(int n, int n_lambda, const int32_t* rp, const int32_t* ci,
                                                        const double* va, double* dinv) {
  for (int i = n_lambda + blockIdx.x * SV_THREADS + threadIdx.x; i < n; i += gridDim.x * SV_THREADS) {
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = ci[k];
      if (j < n_lambda) d += va[k] * va[k] * dinv[j];
    }
    dinv[i] = d > 0.0 ? 1.0 / d : 1.0;
  }
}

// Start: v_1 = b, z_1 = P^-1 b, partials of <z_1, v_1>; x, w, w_prev, v_0 = 0.
__global__ void __launch_bounds__(SV_THREADS) k_start(int n, const double* b, const double* dinv, double* v1,
                                                      double* z1, double* v0, double* w, double* wp, double* x,
                                                      double* part) {
  __shared__ double red[SV_THREADS / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * SV_THREADS + threadIdx.x; i < n; i += gridDim.x * SV_THREADS) {
    const double bi = b[i], zi = bi * dinv[i];
    v1[i] = bi;
    z1[i] = zi;
    v0[i] = 0.0;
    w[i] = 0.0;
    wp[i] = 0.0;
    x[i] = 0.0;
    acc += zi * bi;
  }
  acc = block_reduce(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void k_init_scalars(const double* part, int nb, double* sc) {
  __shared__ double red[SV_THREADS / 64];
  const double g2 = sum_partials(part, nb, red);
  if (threadIdx.x == 0) {
    const double g = sqrt(fmax(g2, 0.0));
    for (int k = 0; k < SC_COUNT; ++k) sc[k] = 0.0;
    sc[SC_GAMMA] = g;
    sc[SC_C] = sc[SC_C_P] = 1.0;
    sc[SC_ETA] = g;
    sc[SC_ETA0] = g;
    sc[SC_RES] = g > 0.0 ? 1.0 : 0.0;
    sc[SC_DONE] = g > 0.0 ? 0.0 : 1.0;
  }
}

// y = A z (raw z); partials of <y, z>.
__global__ void __launch_bounds__(SV_THREADS) k_spmv_dot(int n, const int32_t* rp, const int32_t* ci,
                                                         const double* va, const double* z, double* y, double* part,
                                                         const double* sc) {
  __shared__ double red[SV_THREADS / 64];
  if (sc[SC_DONE] != 0.0) return;
  const int sub = threadIdx.x % ROW_LANES;
  const int rows_per_block = SV_THREADS / ROW_LANES;
  double acc = 0.0;
  for (int base = blockIdx.x * rows_per_block; base < n; base += gridDim.x * rows_per_block) {
    const int row = base + threadIdx.x / ROW_LANES;
    double v = 0.0;
    if (row < n) v = row_dot(rp, ci, va, z, row, sub);   // every lane of the row group ends with the sum
    if (row < n && sub == 0) {
      y[row] = v;
      acc += v * z[row];
    }
  }
  acc = block_reduce(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// v_{j+1} = A z_j / g - (delta/g) v_j - (g/g_prev) v_{j-1} (written over
// v_{j-1}), z_{j+1} = P^-1 v_{j+1}, partials of <z_{j+1}, v_{j+1}>, with
// g = gamma_j and delta = <A z_j, z_j> / g^2.
__global__ void __launch_bounds__(SV_THREADS) k_lanczos(int n, const double* y, const double* vj, double* vprev_next,
                                                        const double* dinv, double* znext, const double* part_in,
                                                        int nb, double* part_out, const double* sc) {
  __shared__ double red[SV_THREADS / 64];
  if (sc[SC_DONE] != 0.0) return;
  const double g = sc[SC_GAMMA], gp = sc[SC_GAMMA_P];
  const double delta = sum_partials(part_in, nb, red) / (g * g);
  const double ig = 1.0 / g, cv = delta / g, cp = gp > 0.0 ? g / gp : 0.0;
  double acc = 0.0;
  for (int i = blockIdx.x * SV_THREADS + threadIdx.x; i < n; i += gridDim.x * SV_THREADS) {
    const double vn = y[i] * ig - cv * vj[i] - cp * vprev_next[i];
    const double zn = vn * dinv[i];
    vprev_next[i] = vn;
    znext[i] = zn;
    acc += zn * vn;
  }
  acc = block_reduce(acc, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = acc;
}

// The MINRES recurrences of step j and the update of the direction and the
// iterate, in one launch.  Every workgroup reduces the same partials
// (<A z_j, z_j> and <z_{j+1}, v_{j+1}>) in the same order, so all of them
// hold identical scalars; workgroup 0 publishes them in the other scalar
// set (sc_in is read by every workgroup, so the sets alternate by step).
//   delta = <A z_j, z_j> / gamma_j^2,  gamma_{j+1} = sqrt(<z_{j+1}, v_{j+1}>)
//   Givens rotation: a0 = c_j delta - c_{j-1} s_j gamma_j,
//   a1 = sqrt(a0^2 + gamma_{j+1}^2), a2 = s_j delta + c_{j-1} c_j gamma_j,
//   a3 = s_{j-1} gamma_j, c_{j+1} = a0 / a1, s_{j+1} = gamma_{j+1} / a1
//   w_{j+1} = (z_j / gamma_j - a3 w_{j-1} - a2 w_j) / a1 (over w_{j-1})
//   x_j = x_{j-1} + c_{j+1} eta w_{j+1},  eta <- -s_{j+1} eta
// A breakdown (gamma_{j+1} = 0: the Krylov space holds the solution) marks
// the iteration done; later launches return at once.
__global__ void __launch_bounds__(SV_THREADS) k_step(int n, const double* part_d, int nbd, const double* part_g,
                                                     int nbg, const double* sc_in, double* sc_out, const double* zj,
                                                     const double* wj, double* wprev_next, double* x) {
  __shared__ double red[SV_THREADS / 64];
  if (sc_in[SC_DONE] != 0.0) {
    if (blockIdx.x == 0 && threadIdx.x < SC_COUNT) sc_out[threadIdx.x] = sc_in[threadIdx.x];
    return;
  }
  const double g = sc_in[SC_GAMMA];
  const double delta = sum_partials(part_d, nbd, red) / (g * g);
  const double gn = sqrt(fmax(sum_partials(part_g, nbg, red), 0.0));
  const double c = sc_in[SC_C], cp = sc_in[SC_C_P], s = sc_in[SC_S], sp = sc_in[SC_S_P];
  const double a0 = c * delta - cp * s * g;
  double a1 = sqrt(a0 * a0 + gn * gn);
  const double a2 = s * delta + cp * c * g;
  const double a3 = sp * g;
  const double cn = a1 > 0.0 ? a0 / a1 : 1.0, sn = a1 > 0.0 ? gn / a1 : 0.0;
  if (!(a1 > 0.0)) a1 = 1.0;
  const double eta = sc_in[SC_ETA];
  const double ig = 1.0 / g, ia1 = 1.0 / a1, xc = cn * eta;
  for (int i = blockIdx.x * SV_THREADS + threadIdx.x; i < n; i += gridDim.x * SV_THREADS) {
    const double wn = (zj[i] * ig - a3 * wprev_next[i] - a2 * wj[i]) * ia1;
    wprev_next[i] = wn;
    x[i] += xc * wn;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc_out[SC_GAMMA] = gn;
    sc_out[SC_GAMMA_P] = g;
    sc_out[SC_C] = cn;
    sc_out[SC_C_P] = c;
    sc_out[SC_S] = sn;
    sc_out[SC_S_P] = s;
    sc_out[SC_ETA] = -sn * eta;
    sc_out[SC_ETA0] = sc_in[SC_ETA0];
    sc_out[SC_A1] = a1;
    sc_out[SC_A2] = a2;
    sc_out[SC_A3] = a3;
    sc_out[SC_XCOEF] = xc;
    sc_out[SC_DONE] = gn > 0.0 ? 0.0 : 1.0;
    sc_out[SC_RES] = sc_in[SC_ETA0] > 0.0 ? fabs(sn * eta) / sc_in[SC_ETA0] : 0.0;
    sc_out[SC_STEPS] = sc_in[SC_STEPS] + 1.0;
  }
}

// Structure check of the CSR arrays before any product reads through them:
// row pointers non-decreasing from 0, column indices inside [0, n).
__global__ void __launch_bounds__(SV_THREADS) k_check_csr(int n, const int32_t* rp, const int32_t* ci, int* bad) {
  int nbad = 0;
  for (int i = blockIdx.x * SV_THREADS + threadIdx.x; i < n; i += gridDim.x * SV_THREADS) {
    const int a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || (i == 0 && a != 0)) {
      ++nbad;
      continue;
    }
    for (int k = a; k < b; ++k) nbad += (ci[k] < 0 || ci[k] >= n) ? 1 : 0;
  }
  if (nbad) atomicAdd(bad, nbad);
}

// r = b - A x; partials of <r, r> and <b, b> (for the final relative residual).
__global__ void __launch_bounds__(SV_THREADS) k_residual(int n, const int32_t* rp, const int32_t* ci,
                                                         const double* va, const double* x, const double* b,
                                                         double* part_r, double* part_b) {
  __shared__ double red[SV_THREADS / 64];
  const int sub = threadIdx.x % ROW_LANES;
  const int rows_per_block = SV_THREADS / ROW_LANES;
  double rr = 0.0, bb = 0.0;
  for (int base = blockIdx.x * rows_per_block; base < n; base += gridDim.x * rows_per_block) {
    const int row = base + threadIdx.x / ROW_LANES;
    double v = 0.0;
    if (row < n) v = row_dot(rp, ci, va, x, row, sub);
    if (row < n && sub == 0) {
      const double r = b[row] - v;
      rr += r * r;
      bb += b[row] * b[row];
    }
  }
  rr = block_reduce(rr, red);
  bb = block_reduce(bb, red);
  if (threadIdx.x == 0) {
    part_r[blockIdx.x] = rr;
    part_b[blockIdx.x] = bb;
  }
}

__global__ void k_residual_final(const double* part_r, const double* part_b, int nb, double* out) {
  __shared__ double red[SV_THREADS / 64];
  const double rr = sum_partials(part_r, nb, red);
  const double bb = sum_partials(part_b, nb, red);
  if (threadIdx.x == 0) out[0] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

}  // namespace

size_t skeleton_solve_bytes(int n) {
  // 9 vectors, two partial arrays, scalars
  return sizeof(double) * ((size_t)9 * n + 3 * SV_MAX_BLOCKS + 2 * SC_COUNT + 8);
}

hipError_t skeleton_csr_check(int n, const int32_t* rp, const int32_t* ci, void* work, int* host_bad,
                              hipStream_t st) {
  int* bad = static_cast<int*>(work);
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  const int nb = std::max(1, std::min(SV_MAX_BLOCKS, (n + SV_THREADS - 1) / SV_THREADS));
  hipLaunchKernelGGL(k_check_csr, dim3(nb), dim3(SV_THREADS), 0, st, n, rp, ci, bad);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipMemcpyAsync(host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t skeleton_solve(int n, int n_lambda, const int32_t* rp, const int32_t* ci, const double* va,
                          const double* b, double* x, double tol, int max_iters, void* work, double* host_sc,
                          int* iters, double* relres, hipStream_t st) {
  double* wk = static_cast<double*>(work);
  double* dinv = wk;
  double* vA = dinv + n;        // three Lanczos vectors
  double* vB = vA + n;
  double* zA = vB + n;          // two preconditioned vectors
  double* zB = zA + n;
  double* wA = zB + n;          // two directions
  double* wB = wA + n;
  double* y = wB + n;
  double* part1 = y + n;
  double* part2 = part1 + SV_MAX_BLOCKS;
  double* part3 = part2 + SV_MAX_BLOCKS;
  double* scA = part3 + SV_MAX_BLOCKS;   // two scalar sets, alternating by step
  double* scB = scA + SC_COUNT;
  double* res_out = scB + SC_COUNT;
  const int nb = std::max(1, std::min(SV_MAX_BLOCKS, (n + SV_THREADS - 1) / SV_THREADS));
  const int nbr = std::max(1, std::min(SV_MAX_BLOCKS, (n + SV_THREADS / ROW_LANES - 1) / (SV_THREADS / ROW_LANES)));
  hipError_t e;
#define SV_CHECK() \
  if ((e = hipGetLastError()) != hipSuccess) return e
  const int nbl = std::max(1, std::min(SV_MAX_BLOCKS, (n_lambda + SV_THREADS - 1) / SV_THREADS));
  if (n_lambda > 0) hipLaunchKernelGGL(k_prec_lambda, dim3(nbl), dim3(SV_THREADS), 0, st, n_lambda, rp, ci, va, dinv);
  SV_CHECK();
  if (n > n_lambda) hipLaunchKernelGGL(k_prec_u0, dim3(nb), dim3(SV_THREADS), 0, st, n, n_lambda, rp, ci, va, dinv);
  SV_CHECK();
  // v_j in vA, v_{j-1} in vB; z_j in zA; w_j in wA, w_{j-1} in wB
  hipLaunchKernelGGL(k_start, dim3(nb), dim3(SV_THREADS), 0, st, n, b, dinv, vA, zA, vB, wA, wB, x, part1);
  SV_CHECK();
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(SV_THREADS), 0, st, part1, nb, scA);
  SV_CHECK();
  // Step j reads the buffers in the roles below and swaps them: an even
  // number of steps returns every buffer to its role, so a chunk of an even
  // number of steps is the same launch sequence every time.
  struct Roles {
    double *vj, *vp, *zj, *zn, *wj, *wp, *si, *so;
  };
  auto enqueue_steps = [&](int count, Roles& r, hipStream_t s) -> hipError_t {
    hipError_t e2 = hipSuccess;
    for (int k = 0; k < count && e2 == hipSuccess; ++k) {
      hipLaunchKernelGGL(k_spmv_dot, dim3(nbr), dim3(SV_THREADS), 0, s, n, rp, ci, va, r.zj, y, part2, r.si);
      hipLaunchKernelGGL(k_lanczos, dim3(nb), dim3(SV_THREADS), 0, s, n, y, r.vj, r.vp, dinv, r.zn, part2, nbr,
                         part3, r.si);
      hipLaunchKernelGGL(k_step, dim3(nb), dim3(SV_THREADS), 0, s, n, part2, nbr, part3, nb, r.si, r.so, r.zj, r.wj,
                         r.wp, x);
      e2 = hipGetLastError();
      std::swap(r.vj, r.vp);   // v_{j+1} was written over v_{j-1}
      std::swap(r.zj, r.zn);
      std::swap(r.wj, r.wp);   // w_{j+1} was written over w_{j-1}
      std::swap(r.si, r.so);
    }
    return e2;
  };
  Roles roles{vA, vB, zA, zB, wA, wB, scA, scB};
  constexpr int kChunk = 16;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (max_iters >= 4 * kChunk) {
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      Roles rc = roles;
      const hipError_t e1 = enqueue_steps(kChunk, rc, cs);
      const hipError_t e2 = hipStreamEndCapture(cs, &graph);
      e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
  }
  int it = 0;
  *iters = 0;
  while (it < max_iters) {
    const int steps = std::min(kChunk, max_iters - it);
    if (exec && steps == kChunk) {
      e = hipGraphLaunch(exec, st);   // roles unchanged after an even chunk
    } else {
      e = enqueue_steps(steps, roles, st);
    }
    if (e != hipSuccess) break;
    it += steps;
    e = hipMemcpyAsync(host_sc, roles.si, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    *iters = (int)host_sc[SC_STEPS];
    if (host_sc[SC_DONE] != 0.0 || host_sc[SC_RES] <= tol) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual, dim3(nbr), dim3(SV_THREADS), 0, st, n, rp, ci, va, x, b, part1, part2);
  SV_CHECK();
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(SV_THREADS), 0, st, part1, part2, nbr, res_out);
  SV_CHECK();
  e = hipMemcpyAsync(host_sc, res_out, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  *relres = host_sc[0];
#undef SV_CHECK
  return hipSuccess;
}

}  // namespace mhm
