// Left-looking blocked local-problem kernel for large elements (gfx950).
//
// Same steps and results as k_local (a2-a6, FP64 or FP32 + FP64 refinement),
// for elements whose tiles do not fit on chip (n up to 16 * 79 nodes).  One
// workgroup of 8 waves handles one element at a time; the factor L (and the
// right-hand-side row) lives in a per-workgroup slot of a device workspace.
//
// Block columns of PW tiles are built one after another:
//   (a) the panel's tiles are initialised in registers straight from the
//       operator (Ahat = A + gamma c c^T is never stored) and the right-hand
//       sides, rows of 16 distributed over the waves (wave w owns rows
//       j0 + w + 8 ri);
//   (b) every earlier tile column m is applied, C_ij -= L_im L_jm^T, with the
//       B operands (the PW tiles L_jm) staged in LDS and the A operands L_im
//       loaded from the workspace (L2 / Infinity Cache resident);
//   (c) the panel is factored in place (diagonal tile by one wave in LDS,
//       panel solve and in-panel updates in registers) and written once.
// Each tile of L is therefore written once and read once per later block
// column, about n^3/(6*16*PW) tile reads per element instead of the
// n^3/(3*16) read-modify-writes of a right-looking sweep.
#include "mhm_common.h"
#include "mhm_kernels.h"

namespace mhm {

namespace ll {
constexpr int NW = 8;
constexpr int NTHREADS = 64 * NW;

// acc[idx / PW][idx % PW] = v for a run-time idx (a chain of compares over
// fixed register slots)
template <int K, int N, int PW, class A, class V>
__device__ __forceinline__ void set_slot(A& acc, int idx, const V& v) {
  if constexpr (K < N) {
    if (idx == K) acc[K / PW][K % PW] = v;
    else set_slot<K + 1, N, PW>(acc, idx, v);
  }
}
}  // namespace ll

template <typename T, bool FUSED, int PW, int RPW>
__global__ void __launch_bounds__(ll::NTHREADS) k_local_ll(BatchDev b, LocalArgs args) {
  using namespace ll;
  typedef typename Mfma<T>::v4 V4;
  __shared__ Elem E;
  __shared__ int ok, bad, conv;
  __shared__ double red[48];
  __shared__ double colsum[16];
  __shared__ double cx[16];
  __shared__ double gam;
  __shared__ double wred[NW][3][16];
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NImax = 3 * (b.l_max + 1);
  const bool fp32 = sizeof(T) == 4;

  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();
    if (tid == 0) {
      int st = INFO_OK;
      if (args.only_fallback && args.info[e] != INFO_IR_FALLBACK) {
        ok = 0;
      } else {
        const bool good = load_elem(b, e, E) && E.rhs0 >= 0 && (FUSED || E.mat0 >= 0);
        if (!good) st = INFO_BAD_DESC;
        else if ((E.nt * (E.nt + 1)) / 2 + E.nt > args.tile_cap || E.n > args.n_cap || E.nt + 1 > NW * RPW ||
                 (FUSED && E.NI * (E.s + 1) > args.f_cap))
          st = INFO_TOO_LARGE;
        ok = st == INFO_OK;
        if (!ok || !args.only_fallback) args.info[e] = st;
        if (args.ir_iters && !args.only_fallback) args.ir_iters[e] = 0;
      }
      bad = -1;
      conv = 0;
    }
    __syncthreads();
    if (!ok) continue;

    const int s = E.s, n = E.n, r = E.r, nt = E.nt;
    double* c = dyn;
    double* bf = c + args.n_cap;
    double* ft = bf + args.n_cap;
    T* stage = reinterpret_cast<T*>(ft + args.f_cap);  // 2 x PW tiles
    T* Wt = stage + 2 * PW * TILE;                       // current diagonal inverse
    T* pub = Wt + TILE;                                  // PW published panel tiles
    T* scr = pub + PW * TILE + wave * TILE;              // this wave's scratch tile
    T* ws = reinterpret_cast<T*>(args.ws) + (int64_t)blockIdx.x * args.ws_slot;
    auto tl = [&](int I, int J) -> T* { return ws + (int64_t)((I * (I + 1)) / 2 + J) * TILE; };
    const double* kapg = b.kappa + E.tri0;
    auto kap = [&](int t) -> double { return kapg[t]; };

    // ------------------------------------------------------------- set-up
    if (FUSED) face_table(E, ft);
    __syncthreads();
    {
      double tr = 0.0, cc2 = 0.0, fs = 0.0;
      const double* fp = b.f + E.tri0;
      for (int p = tid; p < n; p += NTHREADS) {
        int i, j;
        node_ij(p, s, i, j);
        const double cp = node_tri_count(i, j, s) * E.cunit;
        c[p] = cp;
        cc2 += cp * cp;
        if (FUSED || fp32) tr += stencil(i, j, s, E.G, kap).d;
        if (FUSED) {
          const double bp = E.cunit * node_tri_sum(i, j, s, [&](int t) { return fp[t]; });
          bf[p] = bp;
          fs += bp;
        }
      }
      block_sum3(tr, cc2, fs, red);
      if (tid == 0) {
        gam = tr / (n * cc2);
        colsum[E.NI] = fs;
      }
      if (FUSED) face_colsums(E, ft, colsum);
    }
    __syncthreads();
    const double g = gam;
    T* Lo = nullptr;
    if (!FUSED && args.Lout && E.mat0 >= 0) Lo = reinterpret_cast<T*>(args.Lout + E.mat0);

    // Initial value of tile (I, J) in the MFMA result layout: Ahat for I < nt,
    // the transposed right-hand sides Btilde^T for I == nt.
    auto init_tile = [&](int I, int J) -> V4 {
      V4 v4;
      const int cl = lane & 15, grp = lane >> 4;
      const int q = 16 * J + cl;
      if (I == nt) {
        int qi = 0, qj = 0;
        if (FUSED && q < n) node_ij(q, s, qi, qj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = Mfma<T>::row(grp, v);
          double x = 0.0;
          if (a < r && q < n) x = FUSED ? btilde_tab(E, ft, bf, c, colsum, a, q, qi, qj)
                                        : args.Btil[E.rhs0 + (int64_t)a * n + q];
          v4[v] = (T)x;
        }
        return v4;
      }
      if (FUSED) {
        const bool band = 16 * (I - J) <= s + 17;
        Stencil st = {0, 0, 0, 0, 0, 0, 0, 0};
        int qj = 0;
        if (band && q < n) {
          int qi;
          node_ij(q, s, qi, qj);
          st = stencil(qi, qj, s, E.G, kap);
        }
        const int pE = q + 1, pW = q - 1, pN = q + (s + 1 - qj), pS = q - (s + 2 - qj), pNW = q + (s - qj),
                  pSE = q - (s + 1 - qj);
        const double gcq = q < n ? g * c[q] : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = 16 * I + Mfma<T>::row(grp, v);
          double x;
          if (p < n && q < n) {
            x = gcq * c[p];
            if (band) {
              x += (p == q) ? st.d : 0.0;
              x += (p == pE) ? st.e : 0.0;
              x += (p == pW) ? st.w : 0.0;
              x += (p == pN) ? st.n : 0.0;
              x += (p == pS) ? st.so : 0.0;
              x += (p == pNW) ? st.nw : 0.0;
              x += (p == pSE) ? st.se : 0.0;
            }
          } else {
            x = (p == q) ? 1.0 : 0.0;
          }
          v4[v] = (T)x;
        }
      } else {
        const double* A = args.Ahat + E.mat0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = 16 * I + Mfma<T>::row(grp, v);
          v4[v] = (T)((p < n && q < n) ? A[(int64_t)q * n + p] : (p == q ? 1.0 : 0.0));
        }
      }
      return v4;
    };

    // ------------------------------------------------------ factorisation
    for (int j0 = 0; j0 < nt; j0 += PW) {
      const int pw = nt - j0 < PW ? nt - j0 : PW;
      V4 acc[RPW][PW];
      // (a) initial panel (one copy of the tile code; each result goes to its
      // fixed register slot through a compile-time dispatch chain)
#pragma unroll 1
      for (int t = 0; t < RPW * PW; ++t) {
        const int ri = t / PW, jj = t - ri * PW;
        const int i = j0 + wave + NW * ri;
        V4 v = {0, 0, 0, 0};
        if (i <= nt && jj < pw && (i == nt || i >= j0 + jj)) v = init_tile(i, j0 + jj);
        ll::set_slot<0, RPW * PW, PW>(acc, t, v);
      }
      // (b) earlier tile columns
      for (int m = 0; m < j0; ++m) {
        T* st = stage + (m & 1) * PW * TILE;
        for (int idx = tid; idx < pw * TILE; idx += NTHREADS) st[idx] = tl(j0 + idx / TILE, m)[idx % TILE];
        __syncthreads();
#pragma unroll
        for (int ri = 0; ri < RPW; ++ri) {
          const int i = j0 + wave + NW * ri;
          if (i <= nt) {
            const T* L = tl(i, m);
            T a[4];
#pragma unroll
            for (int cch = 0; cch < 4; ++cch) a[cch] = -ld_rowcol(L, cch, lane);
#pragma unroll
            for (int jj = 0; jj < PW; ++jj) {
              if (jj < pw && (i == nt || i >= j0 + jj)) {
                V4 x = acc[ri][jj];
#pragma unroll
                for (int cch = 0; cch < 4; ++cch) x = Mfma<T>::op(a[cch], ld_rowcol(st + jj * TILE, cch, lane), x);
                acc[ri][jj] = x;
              }
            }
          }
        }
      }
      // (c) factor the panel
#pragma unroll
      for (int jj = 0; jj < PW; ++jj) {
        if (jj < pw) {
          const int col = j0 + jj;
          // diagonal tile (row col is local row jj: wave jj, slot 0)
          if (wave == jj) {
            st_acc<T>(Wt, acc[0][jj], lane);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            const int bj = potrf_tile<T>(Wt, Lo, n, col, lane);
            if (lane == 0 && bj >= 0 && bad < 0) bad = 16 * col + bj;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            T* dst = tl(col, col);
            for (int idx = lane; idx < TILE; idx += 64) dst[idx] = Wt[idx];
          }
          __syncthreads();
          // panel solve L_i,col = C_i,col W^T for the rows below
#pragma unroll
          for (int ri = 0; ri < RPW; ++ri) {
            const int i = j0 + wave + NW * ri;
            if (i > col && i <= nt) {
              st_acc<T>(scr, acc[ri][jj], lane);
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              V4 x = {0, 0, 0, 0};
#pragma unroll
              for (int cch = 0; cch < 4; ++cch) x = Mfma<T>::op(ld_rowcol(scr, cch, lane), ld_rowcol(Wt, cch, lane), x);
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              acc[ri][jj] = x;
              st_acc<T>(tl(i, col), x, lane);
              if (Lo && i < nt) store_L<T>(Lo, n, i, col, x, lane);
              if (i < j0 + pw) st_acc<T>(pub + (i - j0) * TILE, x, lane);
            }
          }
          __syncthreads();
          // in-panel update C_i,j -= L_i,col L_j,col^T for the later panel columns
#pragma unroll
          for (int ri = 0; ri < RPW; ++ri) {
            const int i = j0 + wave + NW * ri;
            if (i > col && i <= nt && jj + 1 < pw) {
              st_acc<T>(scr, acc[ri][jj], lane);
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              T a[4];
#pragma unroll
              for (int cch = 0; cch < 4; ++cch) a[cch] = -ld_rowcol(scr, cch, lane);
#pragma unroll
              for (int j2 = jj + 1; j2 < PW; ++j2) {
                if (j2 < pw && (i == nt || i >= j0 + j2)) {
                  V4 x = acc[ri][j2];
#pragma unroll
                  for (int cch = 0; cch < 4; ++cch) x = Mfma<T>::op(a[cch], ld_rowcol(pub + j2 * TILE, cch, lane), x);
                  acc[ri][j2] = x;
                }
              }
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
    }

    // ------------------------------------------------ solves on the RHS row
    auto backward = [&]() {
      for (int j = nt - 1; j >= 0; --j) {   // X = L^{-T} Y
        if (wave == j % NW) {
          V4 x = {0, 0, 0, 0};
          mma_add_nn<T>(x, tl(nt, j), tl(j, j), lane);   // X_j^T = Z_j^T W_j
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          st_acc<T>(tl(nt, j), x, lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
        for (int i = wave; i < j; i += NW) {
          V4 z = ld_acc<T>(tl(nt, i), lane);
          mma_sub_nn<T>(z, tl(nt, j), tl(j, i), lane);   // Z_i^T -= X_j^T L_ji
          st_acc<T>(tl(nt, i), z, lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
      }
    };
    auto forward = [&]() {
      for (int j = 0; j < nt; ++j) {        // Y = L^{-1} Z
        if (wave == j % NW) {
          V4 x = {0, 0, 0, 0};
          mma_add_nt<T>(x, tl(nt, j), tl(j, j), lane);   // Y_j^T = Z_j^T W_j^T
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          st_acc<T>(tl(nt, j), x, lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
        for (int i = j + 1 + wave; i < nt; i += NW) {
          V4 z = ld_acc<T>(tl(nt, i), lane);
          mma_sub_nt<T>(z, tl(nt, j), tl(i, j), lane);   // Z_i^T -= Y_j^T L_ij^T
          st_acc<T>(tl(nt, i), z, lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
      }
    };
    backward();
    const bool failed = bad >= 0;
    double* X = args.X + E.rhs0;
    const int ca = tid >> 4, cl16 = tid & 15;   // 32 groups of 16 lanes; groups 0..15 do column sums

    if (fp32 && !failed) {
      // --------------------------------------- FP64 refinement (FP32 path)
      for (int idx = tid; idx < n * r; idx += NTHREADS) {
        const int a = idx / n, p = idx - a * n;
        X[idx] = (double)tl(nt, p >> 4)[a * TST + (p & 15)];
      }
      __syncthreads();
      const double* Btg = FUSED ? nullptr : args.Btil + E.rhs0;
      int it = 0;
      for (;; ++it) {
        {
          double v = 0.0;
          if (ca < r)
            for (int p = cl16; p < n; p += 16) v += c[p] * X[(int64_t)ca * n + p];
          v = group16_sum(v);
          if (cl16 == 0 && ca < 16) cx[ca] = v;
        }
        __syncthreads();
        const double anorm = ir_residual<T, FUSED>(E, kap, X, c, cx, g, ft, bf, colsum, Btg,
                                                   [&](int J) -> T* { return tl(nt, J); }, &wred[0][0][0], red);
        if (tid == 0) conv = ir_converged(&wred[0][0][0], NW, r, anorm, args.ir_tol);
        __syncthreads();
        if (conv || it >= args.max_iters) break;
        forward();
        backward();
        for (int idx = tid; idx < n * r; idx += NTHREADS) {
          const int a = idx / n, p = idx - a * n;
          X[idx] += (double)tl(nt, p >> 4)[a * TST + (p & 15)];
        }
        __syncthreads();
      }
      const bool cvd = conv;
      if (tid == 0) {
        if (args.ir_iters) args.ir_iters[e] = it;
        if (!cvd) args.info[e] = INFO_IR_FALLBACK;
      }
      if (!cvd) continue;
      {
        double v = 0.0;
        if (ca < r)
          for (int p = cl16; p < n; p += 16) v += c[p] * X[(int64_t)ca * n + p];
        v = group16_sum(v);
        if (cl16 == 0 && ca < 16) cx[ca] = v * E.inv_area;
      }
      __syncthreads();
      for (int idx = tid; idx < n * r; idx += NTHREADS) X[idx] -= cx[idx / n];
      __syncthreads();
    } else if (fp32) {
      if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
      continue;
    } else if (failed) {
      for (int idx = tid; idx < n * r; idx += NTHREADS) X[idx] = __builtin_nan("");
      if (tid == 0) args.info[e] = bad + 1;
      if (FUSED && args.M) {
        for (int idx = tid; idx < NImax * NImax; idx += NTHREADS)
          args.M[(int64_t)e * NImax * NImax + idx] = __builtin_nan("");
        if (tid < NImax) {
          args.E[(int64_t)e * NImax + tid] = __builtin_nan("");
          args.B[(int64_t)e * NImax + tid] = __builtin_nan("");
        }
        if (tid == 0) args.F[e] = __builtin_nan("");
      }
      continue;
    } else {
      {
        double v = 0.0;
        if (ca < r)
          for (int p = cl16; p < n; p += 16) v += c[p] * (double)tl(nt, p >> 4)[ca * TST + (p & 15)];
        v = group16_sum(v);
        if (cl16 == 0 && ca < 16) cx[ca] = v * E.inv_area;
      }
      __syncthreads();
      for (int idx = tid; idx < n * r; idx += NTHREADS) {
        const int a = idx / n, p = idx - a * n;
        X[idx] = (double)tl(nt, p >> 4)[a * TST + (p & 15)] - cx[a];
      }
      __syncthreads();
    }
    if (FUSED && args.M) contrib_element(E, X, ft, colsum[E.NI], NImax, args.M, args.E, args.B, args.F, e);
  }
}

// ------------------------------------------------------------------ launch
int local_ll_rows_per_wave(int nt) {
  const int rows = nt + 1;
  if (rows <= 2 * ll::NW) return 2;
  if (rows <= 3 * ll::NW) return 3;
  if (rows <= 5 * ll::NW) return 5;
  if (rows <= 10 * ll::NW) return 10;
  return -1;
}
int local_ll_panel(bool fp32) { return fp32 ? 4 : 2; }

size_t local_ll_lds_bytes(bool fp32, int n_cap, int f_cap) {
  const int pw = local_ll_panel(fp32);
  return sizeof(double) * (2 * (size_t)n_cap + (size_t)f_cap) +
         (size_t)(2 * pw + 1 + pw + ll::NW) * TILE * (fp32 ? sizeof(float) : sizeof(double));
}

template <typename T, bool FUSED, int PW, int RPW>
static hipError_t launch_ll_t(const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  auto kern = k_local_ll<T, FUSED, PW, RPW>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(ll::NTHREADS), lds, st, d, a);
  return hipGetLastError();
}

template <typename T, bool FUSED, int PW>
static hipError_t launch_ll_rpw(int rpw, const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  switch (rpw) {
    case 2: return launch_ll_t<T, FUSED, PW, 2>(d, a, lds, grid, st);
    case 3: return launch_ll_t<T, FUSED, PW, 3>(d, a, lds, grid, st);
    case 5: return launch_ll_t<T, FUSED, PW, 5>(d, a, lds, grid, st);
    case 10: return launch_ll_t<T, FUSED, PW, 10>(d, a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_local_ll(bool fp32, bool fused, int nt_max, const mhm_batch* bt, LocalArgs a, size_t lds, int grid,
                           hipStream_t st) {
  const int rpw = local_ll_rows_per_wave(nt_max);
  const BatchDev d = to_dev(bt);
  if (fp32) return fused ? launch_ll_rpw<float, true, 4>(rpw, d, a, lds, grid, st)
                         : launch_ll_rpw<float, false, 4>(rpw, d, a, lds, grid, st);
  return fused ? launch_ll_rpw<double, true, 2>(rpw, d, a, lds, grid, st)
               : launch_ll_rpw<double, false, 2>(rpw, d, a, lds, grid, st);
}

}  // namespace mhm
