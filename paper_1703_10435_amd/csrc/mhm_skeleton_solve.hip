// Skeleton solve on the device: preconditioned MINRES on the symmetric
// indefinite system of eq. (6), [[M, B^T], [B, 0]] [lambda; u_0] = [E; F].
//
// The element blocks M_e are negative definite, so the multiplier block is
// negative (semi-)definite and the u_0 block is zero: a saddle point.  The
// paper solves it with sparse direct solvers and names hybrid
// direct-iterative solvers as future work (Section 6).  Here it is solved
// iteratively with MINRES (Paige and Saunders' minimal-residual method for
// symmetric indefinite systems, the preconditioned form with an SPD
// preconditioner), preconditioned by a block diagonal P = diag(D, S~):
//   - multiplier rows in groups of `lambda_block` (the DoFs of one face):
//     D = the face blocks of -M, inverted once (lambda_block = 1: |diag(M)|);
//   - u_0 rows: S = B D^-1 B^T (the Schur complement of the face-block
//     approximation), assembled once, one row per element with its up to
//     three face neighbours; S~^-1 is a fixed number of Chebyshev steps on
//     S from zero, a fixed SPD polynomial in S, run by one workgroup with
//     the search direction in LDS (up to 8192 elements; diag(S) above).
//     With lambda_block = 1, S~ = diag(S).
// The u_0 block of the saddle point is an elliptic operator on the coarse
// mesh; its diagonal alone leaves MINRES thousands of steps on C2's system,
// the Chebyshev steps a few hundred.
//
// One MINRES step is three launches (four with face blocks): the CSR product
// with its dot product, the Lanczos vector with the next dot product (with
// face blocks: the Lanczos vector, then the preconditioner with the dot
// product), and the scalar recurrences together with the update of the
// direction and the iterate.  Dot products
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
constexpr int PB_MAX = 8;      // largest face block of the preconditioner
constexpr int S_NB = 3;        // face neighbours of an element in S
constexpr int PA_THREADS = 1024;  // preconditioner launch
constexpr int PA_ROWS = 4;        // u_0 rows per thread held in registers through the sweeps
constexpr int CHEB_STEPS = 16;            // Chebyshev steps (one product with S each)
constexpr double CHEB_RATIO = 300.0;      // assumed lambda_max / lambda_min of D^-1 S

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

// Position of column `col` in row `row` (sorted columns), or -1.
__device__ __forceinline__ int find_col(const int32_t* rp, const int32_t* ci, int row, int col) {
  int lo = rp[row], hi = rp[row + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = ci[mid];
    if (c == col) return mid;
    if (c < col) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// D_f^-1 for face f: the pb x pb block of -M on rows/columns f pb .. f pb + pb - 1,
// inverted by Gauss-Jordan elimination without pivoting (the block is SPD).
// A block that is not (a non-positive pivot) falls back to 1/|diag|.
__global__ void __launch_bounds__(SV_THREADS) k_blk_inv(int nf, int pb, const int32_t* rp, const int32_t* ci,
                                                       const double* va, double* dblk) {
  for (int f = blockIdx.x * SV_THREADS + threadIdx.x; f < nf; f += gridDim.x * SV_THREADS) {
    double a[PB_MAX][PB_MAX];
    const int r0 = f * pb;
#pragma unroll
    for (int i = 0; i < PB_MAX; ++i)
#pragma unroll
      for (int j = 0; j < PB_MAX; ++j) {
        double v = 0.0;
        if (i < pb && j < pb) {
          const int k = find_col(rp, ci, r0 + i, r0 + j);
          v = k >= 0 ? -va[k] : 0.0;
        }
        a[i][j] = v;
      }
    double dg[PB_MAX];
#pragma unroll
    for (int i = 0; i < PB_MAX; ++i) dg[i] = a[i][i];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < PB_MAX; ++k) {
      if (k < pb) {
        const double piv = a[k][k];
        ok = ok && piv > 0.0;
        const double inv = piv > 0.0 ? 1.0 / piv : 0.0;
#pragma unroll
        for (int j = 0; j < PB_MAX; ++j) a[k][j] = j == k ? inv : a[k][j] * inv;
#pragma unroll
        for (int i = 0; i < PB_MAX; ++i) {
          if (i != k) {
            const double fct = a[i][k];
#pragma unroll
            for (int j = 0; j < PB_MAX; ++j) a[i][j] = j == k ? -fct * inv : a[i][j] - fct * a[k][j];
          }
        }
      }
    }
    double* o = dblk + (int64_t)f * pb * pb;
    for (int i = 0; i < pb; ++i)
      for (int j = 0; j < pb; ++j) {
        double v = 0.0;
#pragma unroll
        for (int ii = 0; ii < PB_MAX; ++ii)
#pragma unroll
          for (int jj = 0; jj < PB_MAX; ++jj)
            if (ii == i && jj == j) v = a[ii][jj];
        if (!ok) v = i == j ? (fabs(dg[i]) > 0.0 ? 1.0 / fabs(dg[i]) : 1.0) : 0.0;
        o[i * pb + j] = v;
      }
  }
}

// S = B D^-1 B^T on the u_0 rows, one element (row n_lambda + t) per thread:
// for each face f met in the row (sorted columns, so a fixed order),
// y = D_f^-1 b_t,f adds b_t,f . y to S_tt, and the face's other element t'
// (the other u_0 column of multiplier row f pb) gets S_tt' = b_t',f . y in
// the next neighbour slot.  Stores 1 / S_tt and the slots (column -1: none).
__global__ void __launch_bounds__(SV_THREADS) k_schur(int n, int n_lambda, int pb, const int32_t* rp,
                                                     const int32_t* ci, const double* va, const double* dblk,
                                                     double* sdi, int32_t* sc_col, double* sc_val) {
  const int ne = n - n_lambda;
  for (int t = blockIdx.x * SV_THREADS + threadIdx.x; t < ne; t += gridDim.x * SV_THREADS) {
    const int row = n_lambda + t;
    double stt = 0.0;
    int ns = 0;
    int32_t nc[S_NB] = {-1, -1, -1};
    double nv[S_NB] = {0.0, 0.0, 0.0};
    int k = rp[row];
    const int kend = rp[row + 1];
    while (k < kend && ci[k] < n_lambda) {
      const int f = ci[k] / pb;
      double bt[PB_MAX], y[PB_MAX];
#pragma unroll
      for (int i = 0; i < PB_MAX; ++i) bt[i] = 0.0;
      while (k < kend && ci[k] < n_lambda && ci[k] / pb == f) {
        const int i = ci[k] - f * pb;
#pragma unroll
        for (int q = 0; q < PB_MAX; ++q)
          if (q == i) bt[q] = va[k];
        ++k;
      }
      const double* Df = dblk + (int64_t)f * pb * pb;
#pragma unroll
      for (int i = 0; i < PB_MAX; ++i) {
        double v = 0.0;
        if (i < pb)
          for (int j = 0; j < pb; ++j) {
            double bj = 0.0;
#pragma unroll
            for (int q = 0; q < PB_MAX; ++q)
              if (q == j) bj = bt[q];
            v += Df[i * pb + j] * bj;
          }
        y[i] = v;
      }
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < PB_MAX; ++i) d += bt[i] * y[i];
      stt += d;
      // the other element of face f: a u_0 column of multiplier row f pb other than this row
      int other = -1;
      for (int kk = rp[f * pb]; kk < rp[f * pb + 1]; ++kk)
        if (ci[kk] >= n_lambda && ci[kk] != row) other = ci[kk];
      if (other >= 0 && ns < S_NB) {
        double o = 0.0;
#pragma unroll
        for (int i = 0; i < PB_MAX; ++i) {
          if (i < pb) {
            const int kk = find_col(rp, ci, f * pb + i, other);
            if (kk >= 0) o += va[kk] * y[i];
          }
        }
#pragma unroll
        for (int q = 0; q < S_NB; ++q)
          if (q == ns) {
            nc[q] = other - n_lambda;
            nv[q] = o;
          }
        ++ns;
      }
    }
    sdi[t] = stt > 0.0 ? 1.0 / stt : 1.0;
#pragma unroll
    for (int q = 0; q < S_NB; ++q) {
      sc_col[(int64_t)t * S_NB + q] = nc[q];
      sc_val[(int64_t)t * S_NB + q] = nv[q];
    }
  }
}

// z = P^-1 v and the partials of <z, v>.  Workgroup 0: the u_0 rows, by
// CHEB_STEPS Chebyshev steps on S from zero (cheb != 0: the shared vector
// fits in LDS), else z = v / S_tt.  The other workgroups: the face blocks.
__global__ void __launch_bounds__(PA_THREADS) k_prec_apply(int n, int n_lambda, int pb, int cheb,
                                                          const double* v, double* z, const double* dblk,
                                                          const double* sdi, const int32_t* sc_col,
                                                          const double* sc_val, double* cx, double* cr,
                                                          double* part, const double* sc) {
  __shared__ double red[PA_THREADS / 64];
  extern __shared__ double xs[];   // 2 (n - n_lambda) when cheb
  if (sc[SC_DONE] != 0.0) return;
  const int ne = n - n_lambda, nf = n_lambda / pb;
  double acc = 0.0;
  if (blockIdx.x == 0) {
    const double* vu = v + n_lambda;
    if (cheb) {
      // Chebyshev iteration on S x = v_u (Jacobi-scaled, x_0 = 0) over the
      // interval [lmax / CHEB_RATIO, lmax], lmax the Gershgorin bound of
      // D^-1 S: a fixed polynomial p(D^-1 S) D^-1, positive on (0, lmax],
      // so the preconditioner stays SPD; it reduces the error of the low
      // modes far faster than Jacobi sweeps of the same count.  The search
      // direction is shared through LDS (two buffers).  Each thread's rows
      // t = tid + k PA_THREADS (S row, 1 / S_tt, v_t, iterate, residual) stay
      // in registers when they fit (ne <= PA_ROWS PA_THREADS); otherwise the
      // rows are re-read each step and the iterate and residual live in the
      // workspace (cx, cr: each thread touches only its own rows).
      double* x0 = xs;
      double* x1 = xs + ne;
      const bool held = ne <= PA_ROWS * PA_THREADS;
      double rd[PA_ROWS], rv[PA_ROWS], rsv[PA_ROWS][S_NB], xr[PA_ROWS], rr[PA_ROWS];
      int32_t rsc[PA_ROWS][S_NB];
      double gl = 0.0;
#pragma unroll
      for (int k = 0; k < PA_ROWS; ++k) {
        const int t = threadIdx.x + k * PA_THREADS;
        const bool in = held && t < ne;
        rd[k] = in ? sdi[t] : 0.0;
        rv[k] = in ? vu[t] : 0.0;
        double g = in ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < S_NB; ++q) {
          rsc[k][q] = in ? sc_col[(int64_t)t * S_NB + q] : -1;
          rsv[k][q] = in ? sc_val[(int64_t)t * S_NB + q] : 0.0;
          g += fabs(rsv[k][q]) * rd[k];
        }
        gl = fmax(gl, g);
        xr[k] = 0.0;
        rr[k] = rv[k];
      }
      if (!held)
        for (int t = threadIdx.x; t < ne; t += PA_THREADS) {
          double g = 1.0;
#pragma unroll
          for (int q = 0; q < S_NB; ++q) g += fabs(sc_val[(int64_t)t * S_NB + q]) * sdi[t];
          gl = fmax(gl, g);
        }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) gl = fmax(gl, __shfl_xor(gl, o, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = gl;
      __syncthreads();
      double lmax = 0.0;
      for (int w = 0; w < PA_THREADS / 64; ++w) lmax = fmax(lmax, red[w]);
      lmax = lmax > 0.0 ? lmax : 1.0;
      const double lmin = lmax / CHEB_RATIO;
      const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma1 = theta / delta;
      double rho = 1.0 / sigma1;
      if (held) {
#pragma unroll
        for (int k = 0; k < PA_ROWS; ++k) {
          const int t = threadIdx.x + k * PA_THREADS;
          if (t < ne) x0[t] = rd[k] * rv[k] / theta;   // d_0
        }
      } else {
        for (int t = threadIdx.x; t < ne; t += PA_THREADS) {
          cx[t] = 0.0;
          cr[t] = vu[t];
          x0[t] = sdi[t] * vu[t] / theta;
        }
      }
      __syncthreads();
      for (int it = 0; it < CHEB_STEPS; ++it) {
        const double* dc = (it & 1) ? x1 : x0;
        double* dn = (it & 1) ? x0 : x1;
        const double rho_n = 1.0 / (2.0 * sigma1 - rho);
        const double c1 = rho_n * rho, c2 = 2.0 * rho_n / delta;
        if (held) {
#pragma unroll
          for (int k = 0; k < PA_ROWS; ++k) {
            const int t = threadIdx.x + k * PA_THREADS;
            if (t < ne) {
              const double dt = dc[t];
              double sd = dt / rd[k];
#pragma unroll
              for (int q = 0; q < S_NB; ++q)
                if (rsc[k][q] >= 0) sd += rsv[k][q] * dc[rsc[k][q]];
              xr[k] += dt;
              rr[k] -= sd;
              dn[t] = c1 * dt + c2 * rd[k] * rr[k];
            }
          }
        } else {
          for (int t = threadIdx.x; t < ne; t += PA_THREADS) {
            const double di = sdi[t], dt = dc[t];
            double sd = dt / di;
#pragma unroll
            for (int q = 0; q < S_NB; ++q) {
              const int c = sc_col[(int64_t)t * S_NB + q];
              if (c >= 0) sd += sc_val[(int64_t)t * S_NB + q] * dc[c];
            }
            cx[t] += dt;
            const double rt = cr[t] - sd;
            cr[t] = rt;
            dn[t] = c1 * dt + c2 * di * rt;
          }
        }
        rho = rho_n;
        __syncthreads();
      }
      if (held) {
#pragma unroll
        for (int k = 0; k < PA_ROWS; ++k) {
          const int t = threadIdx.x + k * PA_THREADS;
          if (t < ne) {
            z[n_lambda + t] = xr[k];
            acc += xr[k] * vu[t];
          }
        }
      } else {
        for (int t = threadIdx.x; t < ne; t += PA_THREADS) {
          z[n_lambda + t] = cx[t];
          acc += cx[t] * vu[t];
        }
      }
    } else {
      for (int t = threadIdx.x; t < ne; t += PA_THREADS) {
        const double zt = sdi[t] * vu[t];
        z[n_lambda + t] = zt;
        acc += zt * vu[t];
      }
    }
  } else {
    for (int f = (blockIdx.x - 1) * PA_THREADS + threadIdx.x; f < nf; f += (gridDim.x - 1) * PA_THREADS) {
      const double* Df = dblk + (int64_t)f * pb * pb;
      const double* vf = v + (int64_t)f * pb;
      double* zf = z + (int64_t)f * pb;
      for (int i = 0; i < pb; ++i) {
        double s = 0.0;
        for (int j = 0; j < pb; ++j) s += Df[i * pb + j] * vf[j];
        zf[i] = s;
        acc += s * vf[i];
      }
    }
  }
  acc = block_reduce(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
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
// With face blocks (dinv == nullptr) only v_{j+1} is written here;
// k_prec_apply forms z_{j+1} and its partials.
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
    vprev_next[i] = vn;
    if (dinv) {
      const double zn = vn * dinv[i];
      znext[i] = zn;
      acc += zn * vn;
    }
  }
  if (!dinv) return;
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

size_t skeleton_solve_bytes(int n, int pb) {
  // 9 vectors, three partial arrays, scalars; with face blocks the block
  // inverses (n_lambda pb <= n pb values), S per element row (1 / S_tt,
  // 3 values, 3 int32 columns: 5.5 doubles' worth) and the Chebyshev
  // iterate and residual (2 per element row): at most 8 n
  const size_t blk = pb > 1 ? (size_t)n * pb + 8 * (size_t)n + 64 : 0;
  return sizeof(double) * ((size_t)9 * n + 3 * SV_MAX_BLOCKS + 2 * SC_COUNT + 8 + blk);
}

int skeleton_block_max() { return PB_MAX; }

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

hipError_t skeleton_solve(int n, int n_lambda, int pb, const int32_t* rp, const int32_t* ci, const double* va,
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
  // face blocks (pb > 1): D^-1 per face, then S on the u_0 rows
  const bool blocked = pb > 1 && n_lambda > 0 && n_lambda % pb == 0;
  const int ne = n - n_lambda, nf = blocked ? n_lambda / pb : 0;
  double* dblk = res_out + 8;
  double* sdi = dblk + (size_t)n_lambda * (blocked ? pb : 0);
  double* sc_val = sdi + ne;
  int32_t* sc_col = reinterpret_cast<int32_t*>(sc_val + (size_t)S_NB * ne);
  double* cheb_x = sc_val + (size_t)S_NB * ne + ((size_t)S_NB * ne + 1) / 2;   // after the int32 columns
  double* cheb_r = cheb_x + ne;
  // the Chebyshev steps hold two copies of the u_0 search direction in one workgroup's LDS
  const size_t cheb_lds = sizeof(double) * 2 * (size_t)ne;
  const int cheb = blocked && ne > 0 && cheb_lds <= 128 * 1024 ? 1 : 0;
  const int nbp = 1 + std::max(1, std::min(SV_MAX_BLOCKS - 1, (nf + PA_THREADS - 1) / PA_THREADS));
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
  if (blocked) {
    if (cheb) {
      e = hipFuncSetAttribute((const void*)k_prec_apply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cheb_lds);
      if (e != hipSuccess) return e;
    }
    const int nbf = std::max(1, std::min(SV_MAX_BLOCKS, (nf + SV_THREADS - 1) / SV_THREADS));
    hipLaunchKernelGGL(k_blk_inv, dim3(nbf), dim3(SV_THREADS), 0, st, nf, pb, rp, ci, va, dblk);
    SV_CHECK();
    if (ne > 0) {
      const int nbe = std::max(1, std::min(SV_MAX_BLOCKS, (ne + SV_THREADS - 1) / SV_THREADS));
      hipLaunchKernelGGL(k_schur, dim3(nbe), dim3(SV_THREADS), 0, st, n, n_lambda, pb, rp, ci, va, dblk, sdi, sc_col,
                         sc_val);
      SV_CHECK();
    }
  }
  // z = P^-1 v with its partials, for the face-block preconditioner
  auto prec_apply = [&](const double* v, double* z, double* part, const double* sc, hipStream_t s2) {
    hipLaunchKernelGGL(k_prec_apply, dim3(nbp), dim3(PA_THREADS), cheb ? cheb_lds : 0, s2, n, n_lambda, pb, cheb,
                       v, z, dblk, sdi, sc_col, sc_val, cheb_x, cheb_r, part, sc);
  };
  // v_j in vA, v_{j-1} in vB; z_j in zA; w_j in wA, w_{j-1} in wB
  hipLaunchKernelGGL(k_start, dim3(nb), dim3(SV_THREADS), 0, st, n, b, dinv, vA, zA, vB, wA, wB, x, part1);
  SV_CHECK();
  if (blocked) {
    // scalars not set yet: a zeroed slot reads as "not done"
    e = hipMemsetAsync(scA, 0, sizeof(double) * SC_COUNT, st);
    if (e != hipSuccess) return e;
    prec_apply(vA, zA, part1, scA, st);
    SV_CHECK();
  }
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(SV_THREADS), 0, st, part1, blocked ? nbp : nb, scA);
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
      hipLaunchKernelGGL(k_lanczos, dim3(nb), dim3(SV_THREADS), 0, s, n, y, r.vj, r.vp, blocked ? nullptr : dinv,
                         r.zn, part2, nbr, part3, r.si);
      if (blocked) prec_apply(r.vp, r.zn, part3, r.si, s);   // v_{j+1} is in r.vp now
      hipLaunchKernelGGL(k_step, dim3(nb), dim3(SV_THREADS), 0, s, n, part2, nbr, part3, blocked ? nbp : nb, r.si,
                         r.so, r.zj, r.wj, r.wp, x);
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
