// Time steps on stored factors (gfx950): only the source column.
//
// With coefficients that do not change in time, the local matrix and the
// multiplier load vectors stay the same from step to step (Section 3), so
// after the first step the factor L of Ahat, the multiplier columns of X, M
// and B are all still valid.  A later step only has a new source f: its
// compatible load vector btilde = b - c (1^T b) / |K| (eq. (8)), one forward
// and one backward solve with the stored L, the zero-mean projection and the
// source-dependent contributions E = R^T eta^f and F = (1, f)_K (eq. (6)).
//
// Work per element: one pass over the factor for each sweep, 2 n^2 flops in
// total; the kernel is bound by reading the factor from HBM.  One wave
// handles one element: the sweep is a chain of 16-row tile steps, and a wave
// runs it with no workgroup barriers (quad DPP sums and lane shuffles).
// Lane (u, k) = (lane / 4, lane % 4) holds four entries of every tile: a
// row segment (row u, columns 4k..4k+3) in the forward sweep, a column
// segment (column u, rows 4k..4k+3) in the backward one.  The tiles stream
// through a ring of D register sets, D tiles ahead of the arithmetic.
//
// FP32 factors: FP64 refinement with the matrix-free residual of Ahat (the
// operator's stencil from kappa), the same stopping rule as the full solve;
// elements whose refinement does not converge report -1 and are recomputed
// in FP64 by the caller's fallback pass.
#include "mhm_common.h"
#include "mhm_kernels.h"

namespace mhm {
namespace {

constexpr int SS_WAVES = 4;   // waves (elements in flight) per workgroup

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Sum over the four lanes of a quad; every lane of the quad gets it
// (quad_perm [1,0,3,2] then [2,3,0,1]).
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// One triangular sweep of the single right-hand side y (LDS, 16 nt entries,
// zero past n) against the stored factor: forward L y <- y, backward
// L^T y <- y.  Tiles (I, J) of L are stored row by row, tile (I, J) at
// index I (I + 1) / 2 + J, the diagonal ones holding W = L_II^{-1}.
// Forward order: row I = 0..nt-1, tiles J = 0..I (the storage order).
// Backward order: column I = nt-1..0, tiles (J, I) for J = nt-1 down to I.
template <typename T, bool BACK, int D>
__device__ __forceinline__ void sweep1(const T* __restrict__ Lb, T* y, int nt, int lane) {
  const int u = lane >> 2, k4 = lane & 3;
  const int ntile = (nt * (nt + 1)) / 2;
  auto advance = [&](int& I, int& J) {
    if (BACK) {
      if (J > I) --J;
      else { --I; J = nt - 1; }
    } else {
      if (J < I) ++J;
      else { ++I; J = 0; }
    }
  };
  auto load = [&](T (&v)[4], int I, int J) {
    const T* p = BACK ? Lb + (int64_t)((J * (J + 1)) / 2 + I) * TILE : Lb + (int64_t)((I * (I + 1)) / 2 + J) * TILE;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = BACK ? p[(4 * k4 + k) * TST + u] : p[u * TST + 4 * k4 + k];
  };
  // Fetch cursor: runs D tiles ahead and stops on the last tile (the ring
  // then re-reads it from cache), so that every step issues its loads
  // unconditionally and the memory counters wait exactly D - 1 tiles back.
  T buf[D][4];
  int fi = BACK ? nt - 1 : 0, fj = BACK ? nt - 1 : 0, fleft = ntile - 1;
  auto fetch = [&](T (&v)[4]) {
    load(v, fi, fj);
    if (fleft > 0) {
      advance(fi, fj);
      --fleft;
    }
  };
#pragma unroll
  for (int q = 0; q < D; ++q) fetch(buf[q]);
  int I = BACK ? nt - 1 : 0, J = BACK ? nt - 1 : 0;   // arithmetic cursor
  T acc = T(0);
  for (int t0 = 0; t0 < ntile; t0 += D) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if (t0 + q < ntile) {
        if (I != J) {
          // forward: sum_c L_IJ[u][c] y_J[c];  backward: sum_r L_JI[r][u] y_J[r]
          const T* yj = y + 16 * J + 4 * k4;
#pragma unroll
          for (int k = 0; k < 4; ++k) acc += buf[q][k] * yj[k];
        } else {
          // z = y_I - sum (entry u, in every lane of quad u); then
          // y_I = W z (forward) or W^T z (backward): lane (u, k) needs
          // z[4k..4k+3], held by quads 4k..4k+3
          const T z = y[16 * I + u] - quad_sum(acc);
          T v = T(0);
#pragma unroll
          for (int k = 0; k < 4; ++k) v += buf[q][k] * __shfl(z, 4 * (4 * k4 + k) + k4, 64);
          v = quad_sum(v);
          if (k4 == 0) y[16 * I + u] = v;
          acc = T(0);
        }
        advance(I, J);
      }
      fetch(buf[q]);
    }
  }
}

template <typename T>
__device__ __forceinline__ void sweep_pair(const T* Lb, T* y, int nt, int lane) {
  constexpr int D = sizeof(T) == 8 ? 8 : 12;
  sweep1<T, false, D>(Lb, y, nt, lane);
  wave_sync();
  sweep1<T, true, D>(Lb, y, nt, lane);
  wave_sync();
}

template <typename T>
__global__ void __launch_bounds__(64 * SS_WAVES) k_source_step(BatchDev b, SourceArgs a) {
  __shared__ Elem Es[SS_WAVES];
  __shared__ int ok_s[SS_WAVES];
  extern __shared__ double dyn[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Elem& E = Es[wave];
  double* bt = dyn + (int64_t)wave * a.wave_words;                    // btilde (FP64), n_cap
  T* y = reinterpret_cast<T*>(bt + a.n_cap);                          // solve vector, 16 nt_cap
  const int NImax = nimax(b);
  constexpr bool fp32 = sizeof(T) == 4;

  for (int e = blockIdx.x * SS_WAVES + wave; e < b.n_elem; e += gridDim.x * SS_WAVES) {
    wave_sync();
    if (lane == 0) {
      int st = INFO_OK;
      if (!load_elem(b, e, E) || E.rhs0 < 0) st = INFO_BAD_DESC;
      else if (E.n > a.n_cap) st = INFO_TOO_LARGE;
      else if (a.fac_state[e] != 1 || a.fac_off[e] < 0) st = INFO_NO_FACTOR;
      a.info[e] = st;
      if (a.ir_iters) a.ir_iters[e] = 0;
      ok_s[wave] = st == INFO_OK;
    }
    wave_sync();
    if (!ok_s[wave]) continue;

    const int s = E.s, n = E.n, nt = E.nt, NI = E.NI;
    const double* fp = b.f + E.tri0;
    const double* kapg = b.kappa + E.tri0;
    auto kap = [&](int t) -> double { return kapg[t]; };
    const T* Lb = reinterpret_cast<const T*>(static_cast<const char*>(a.fac) + a.fac_off[e]);
    double* xg = a.X + E.rhs0 + (int64_t)NI * n;   // the source column of X

    // FP64 factors: one refinement step with a double-double residual where
    // a plain FP64 solve is not accurate enough (refine64_needed, per wave)
    bool ref = fp32;
    if (!fp32) {
      if (a.refine64 != 0) {
        ref = a.refine64 > 0;
      } else {
        double kmax = 0.0, kinv = 0.0;
        for (int t = lane; t < s * s; t += 64) {
          kmax = fmax(kmax, kapg[t]);
          kinv = fmax(kinv, 1.0 / kapg[t]);
        }
        ref = !(wave_max(kmax) * wave_max(kinv) * ((double)s * s) <= REFINE64_SCALE);
      }
    }

    // ------------------------------------------------ load vector, eq. (8)
    double fs = 0.0, tr = 0.0, cc2 = 0.0;
    for (int p = lane; p < n; p += 64) {
      int i, j;
      node_ij(p, s, i, j);
      const double bp = E.cunit * node_tri_sum(i, j, s, [&](int t) { return fp[t]; });
      bt[p] = bp;
      fs += bp;
      if (ref) {   // gamma = tr(A) / (n c^T c) of the factored Ahat
        const double cp = node_tri_count(i, j, s) * E.cunit;
        cc2 += cp * cp;
        tr += stencil(i, j, s, E.G, kap).d;
      }
    }
    fs = wave_sum(fs);
    double g = 0.0;
    if (ref) {
      tr = wave_sum(tr);
      cc2 = wave_sum(cc2);
      g = tr / (n * cc2);
    }
    double bm = 0.0;
    for (int p = lane; p < 16 * nt; p += 64) {
      double v = 0.0;
      if (p < n) {
        int i, j;
        node_ij(p, s, i, j);
        v = bt[p] - node_tri_count(i, j, s) * E.cunit * fs * E.inv_area;
        bt[p] = v;
        bm = fmax(bm, fabs(v));
      }
      y[p] = (T)v;
    }
    wave_sync();

    // ------------------------------------------------------------ solves
    sweep_pair<T>(Lb, y, nt, lane);

    double shift;   // (c^T x) / |K| of the final iterate
    if (!ref) {
      double cx = 0.0;
      for (int p = lane; p < n; p += 64) {
        int i, j;
        node_ij(p, s, i, j);
        cx += node_tri_count(i, j, s) * E.cunit * (double)y[p];
      }
      shift = wave_sum(cx) * E.inv_area;
      for (int p = lane; p < n; p += 64) xg[p] = (double)y[p] - shift;
    } else {
      // --------------------------------------------------- FP64 refinement
      // FP32 L: FP64 residuals until the backward error target; FP64 L: one
      // step with a double-double residual.
      // ||Ahat||_inf: stencil row sums plus gamma c_p |K| of the rank-one term
      double anorm;
      {
        double an = 0.0;
        for (int p = lane; p < n; p += 64) {
          int i, j;
          node_ij(p, s, i, j);
          const Stencil st = stencil(i, j, s, E.G, kap);
          const double cp = node_tri_count(i, j, s) * E.cunit;
          an = fmax(an, fabs(st.d) + fabs(st.e) + fabs(st.w) + fabs(st.n) + fabs(st.so) + fabs(st.nw) +
                            fabs(st.se) + g * cp * E.area);
        }
        anorm = wave_max(an);
      }
      const double bmax = wave_max(bm);
      double cx = 0.0, xm = 0.0;
      for (int p = lane; p < n; p += 64) {
        int i, j;
        node_ij(p, s, i, j);
        const double xv = (double)y[p];
        xg[p] = xv;
        cx += node_tri_count(i, j, s) * E.cunit * xv;
        xm = fmax(xm, fabs(xv));
      }
      cx = wave_sum(cx);
      xm = wave_max(xm);
      wave_sync();
      double prev = 0.0;
      int it = 0, conv = 0;
      for (;; ++it) {
        if (!fp32 && it >= 1) {
          conv = 1;
          break;
        }
        // r = btilde - Ahat x (FP64, matrix-free; double-double for FP64 L), into y
        double rm = 0.0;
        for (int p = lane; p < n; p += 64) {
          int i, j;
          node_ij(p, s, i, j);
          const Stencil st = stencil(i, j, s, E.G, kap);
          const double cp = node_tri_count(i, j, s) * E.cunit;
          const bool hasE = i + j <= s - 1, hasW = i >= 1, hasS = j >= 1;
          double r;
          if (fp32) {
            double ax = st.d * xg[p] + cp * (g * cx);
            if (hasE) ax += st.e * xg[p + 1] + st.n * xg[p + (s + 1 - j)];
            if (hasW) ax += st.w * xg[p - 1] + st.nw * xg[p + (s - j)];
            if (hasS) ax += st.so * xg[p - (s + 2 - j)] + st.se * xg[p - (s + 1 - j)];
            r = bt[p] - ax;
          } else {
            double hi = 0.0, lo = 0.0;
            dd_add_prod(hi, lo, st.d, xg[p]);
            dd_add_prod(hi, lo, cp, g * cx);
            if (hasE) {
              dd_add_prod(hi, lo, st.e, xg[p + 1]);
              dd_add_prod(hi, lo, st.n, xg[p + (s + 1 - j)]);
            }
            if (hasW) {
              dd_add_prod(hi, lo, st.w, xg[p - 1]);
              dd_add_prod(hi, lo, st.nw, xg[p + (s - j)]);
            }
            if (hasS) {
              dd_add_prod(hi, lo, st.so, xg[p - (s + 2 - j)]);
              dd_add_prod(hi, lo, st.se, xg[p - (s + 1 - j)]);
            }
            r = dd_sub_from(bt[p], hi, lo);
          }
          y[p] = (T)r;
          rm = fmax(rm, fabs(r));
        }
        rm = wave_max(rm);
        if (fp32) {
          const double be = ir_backward_error(&rm, &xm, &bmax, 1, anorm);
          conv = ir_decide(be, prev, it, a.max_iters, a.ir_tol);
          prev = be;
          if (conv != 0) break;
        }
        wave_sync();
        sweep_pair<T>(Lb, y, nt, lane);
        cx = 0.0;
        xm = 0.0;
        for (int p = lane; p < n; p += 64) {
          int i, j;
          node_ij(p, s, i, j);
          const double xv = xg[p] + (double)y[p];
          xg[p] = xv;
          cx += node_tri_count(i, j, s) * E.cunit * xv;
          xm = fmax(xm, fabs(xv));
        }
        cx = wave_sum(cx);
        xm = wave_max(xm);
        wave_sync();
      }
      if (lane == 0) {
        if (a.ir_iters) a.ir_iters[e] = it;
        if (conv < 0) a.info[e] = INFO_IR_FALLBACK;
      }
      if (conv < 0) continue;
      shift = cx * E.inv_area;
      for (int p = lane; p < n; p += 64) xg[p] -= shift;
    }
    wave_sync();

    // ------------------------------- contributions E = R^T eta^f, F, eq. (6)
    if (lane < NImax) {
      double v = 0.0;
      if (lane < NI) {
        const int ef = lane / E.P;
        for (int k = 0; k <= s; ++k) v += face_load(E, lane, k) * xg[face_node(ef, k, s)];
      }
      a.E[(int64_t)e * NImax + lane] = v;
    }
    if (lane == 0) a.F[e] = fs;
  }
}

}  // namespace

size_t source_step_lds(bool fp32, int n_cap, int& wave_words) {
  const int nt_cap = (n_cap + 15) / 16;
  const size_t y_bytes = (size_t)16 * nt_cap * (fp32 ? sizeof(float) : sizeof(double));
  wave_words = n_cap + (int)((y_bytes + 7) / 8);
  return (size_t)SS_WAVES * wave_words * sizeof(double);
}

int source_step_waves() { return SS_WAVES; }

hipError_t launch_source_step(bool fp32, const mhm_batch* bt, const SourceArgs& a, size_t lds, int grid,
                              hipStream_t st) {
  const BatchDev d = to_dev(bt);
  const void* kern = fp32 ? (const void*)k_source_step<float> : (const void*)k_source_step<double>;
  hipError_t err = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  if (fp32) hipLaunchKernelGGL(k_source_step<float>, dim3(grid), dim3(64 * SS_WAVES), lds, st, d, a);
  else hipLaunchKernelGGL(k_source_step<double>, dim3(grid), dim3(64 * SS_WAVES), lds, st, d, a);
  return hipGetLastError();
}

}  // namespace mhm
