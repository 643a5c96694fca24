// Block-level helpers shared by the LDS/workspace tile kernels and the
// left-looking kernel: reductions, broadcasts, per-element tables, the
// diagonal-tile factorisation and the contribution of eq. (6).
#pragma once

#include "mhm_device.h"

namespace mhm {


// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// sum over the 16 lanes of a lane group (lanes 16g .. 16g+15)
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// max over the 16 lanes of a lane group
__device__ __forceinline__ double group16_max(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// Block-wide sums of three values; every thread gets the results.
// `red` holds 48 doubles (up to 16 waves).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[16 + w] = b;
    red[32 + w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
  for (int k = 0; k < nw; ++k) {
    a += red[k];
    b += red[16 + k];
    c += red[32 + k];
  }
}
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int k = 1; k < nw; ++k) t = fmax(t, red[k]);
  return t;
}

__device__ __forceinline__ double readlane(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
// 1/sqrt(x): hardware estimate refined by Newton steps y <- y (3 - x y^2) / 2
__device__ __forceinline__ double rsqrt_t(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
__device__ __forceinline__ float rsqrt_t(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  y = y * (1.5f - 0.5f * x * y * y);
  return y;
}

// Sum of fn(t) over the sub-triangles t around node (i,j).
template <class FN>
__device__ __forceinline__ double node_tri_sum(int i, int j, int s, FN fn) {
  const int ij = i + j;
  double a = 0.0;
  if (ij <= s - 1) a += fn(tri_up(i, j, s));
  if (i >= 1 && ij <= s) a += fn(tri_up(i - 1, j, s));
  if (j >= 1 && ij <= s) a += fn(tri_up(i, j - 1, s));
  if (i >= 1 && j >= 1 && ij <= s) a += fn(tri_dn(i - 1, j - 1, s));
  if (i >= 1 && ij <= s - 1) a += fn(tri_dn(i - 1, j, s));
  if (j >= 1 && ij <= s - 1) a += fn(tri_dn(i, j - 1, s));
  return a;
}

// -------------------------------------------------------- per-element tables
// ft[a*(s+1) + k] = R[face node k of face e(a)][a]   (face load table)
// colsum[a] = 1^T B[:, a]  (face columns from ft, source column from bf)
__device__ __forceinline__ void face_table(const Elem& E, double* ft) {
  const int sp1 = E.s + 1;
  for (int idx = threadIdx.x; idx < E.NI * sp1; idx += blockDim.x) {
    const int a = idx / sp1, k = idx - a * sp1;
    ft[idx] = face_load(E, a, k);
  }
}
__device__ __forceinline__ void face_colsums(const Elem& E, const double* ft, double* colsum) {
  const int sp1 = E.s + 1;
  if ((int)threadIdx.x < E.NI) {
    double v = 0.0;
    for (int k = 0; k < sp1; ++k) v += ft[threadIdx.x * sp1 + k];
    colsum[threadIdx.x] = v;
  }
}

// Btilde[p][a] from the tables.
__device__ __forceinline__ double btilde_tab(const Elem& E, const double* ft, const double* bf, const double* c,
                                             const double* colsum, int a, int p, int i, int j) {
  double v = 0.0;
  if (a < E.NI) {
    const int e = a / E.P;
    const int k = face_pos(e, i, j, E.s);
    if (k >= 0) v = ft[a * (E.s + 1) + k];
  } else {
    v = bf[p];
  }
  return v - c[p] * colsum[a] * E.inv_area;
}

// ============================================================ contribution
// M[a][b] = -sum_k R(a,k) X[node(a,k)][b], E[a] = sum_k R(a,k) X[node(a,k)][NI],
// B[a] = -sum_k R(a,k), F = integral of f (= colsum of the source column).
// X column-major n x r (already projected); ft the face table.
__device__ __forceinline__ void contrib_element(const Elem& E, const double* X, const double* ft, double Fval, int NImax,
                                double* M, double* Ev, double* Bv, double* F, int e) {
  const int tid = threadIdx.x;
  const int NI = E.NI, n = E.n, s = E.s, sp1 = s + 1;
  double* Me = M + (int64_t)e * NImax * NImax;
  for (int idx = tid; idx < NImax * NImax; idx += blockDim.x) {
    const int a = idx % NImax, bb = idx / NImax;
    if (a >= NI || bb >= NI) Me[idx] = 0.0;
  }
  for (int idx = tid; idx < NI * E.r; idx += blockDim.x) {
    const int a = idx % NI, bb = idx / NI;
    const int ef = a / E.P;
    const double* fa = ft + a * sp1;
    const double* xb = X + (int64_t)bb * n;
    double v = 0.0;
    for (int k = 0; k < sp1; ++k) v += fa[k] * xb[face_node(ef, k, s)];
    if (bb < NI) Me[(int64_t)bb * NImax + a] = -v;
    else Ev[(int64_t)e * NImax + a] = v;
  }
  for (int a = tid; a < NImax; a += blockDim.x) {
    double v = 0.0;
    if (a < NI) {
      for (int k = 0; k < sp1; ++k) v -= ft[a * sp1 + k];
    } else {
      Ev[(int64_t)e * NImax + a] = 0.0;
    }
    Bv[(int64_t)e * NImax + a] = v;
  }
  if (tid == 0) F[e] = Fval;
}

// ================================================================== k_local
// Diagonal tile: Cholesky factor L and its inverse W = L^{-1}, by one wave.
// Lane c (and its copies c+16, c+32, c+48) keeps column c of the symmetric
// tile in registers.  Step j broadcasts column j from lane j with readlane
// (scalar registers feed the FMAs directly), so a step needs no LDS traffic:
//   a[r][c] -= a[r][j] a[j][c] / a[j][j]             (r, c > j)
//   W[j][c] = V[j][c] / sqrt(a[j][j]),  V[r][c] -= L[r][j] W[j][c]   (r > j)
// Column c is final after step c and is scaled by 1/sqrt(a[c][c]) at the end.
// The tile's slot receives W; L goes to `Lo` (column-major n x n, may be
// null).  Returns the first failing column or -1.
template <typename T>
__device__ __forceinline__ int potrf_tile(T* t, T* Lo, int n, int k, int lane) {
  const int c = lane & 15;
  T col[16], w[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    col[r] = r >= c ? t[r * TST + c] : t[c * TST + r];
    w[r] = r == c ? T(1) : T(0);
  }
  int bad = -1;
  T myrs = T(1);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    T ajj = readlane(col[j], j);
    if (!(ajj > T(0))) {
      if (bad < 0) bad = j;
      ajj = T(1);
    }
    const T rs = rsqrt_t(ajj);
    if (c == j) myrs = rs;
    const T tj = col[j] * (rs * rs);      // a[j][c] / a[j][j]
    const T wj = w[j] * rs;               // W[j][c]
    const T wjr = wj * rs;
    w[j] = wj;
#pragma unroll
    for (int r = j + 1; r < 16; ++r) {
      const T arj = readlane(col[r], j);  // a[r][j]
      w[r] -= arj * wjr;
      if (c > j) col[r] -= arj * tj;
    }
  }
  if (lane < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) t[r * TST + c] = w[r];
    if (Lo) {
      const int q = 16 * k + c;
      if (q < n) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int p = 16 * k + r;
          if (r >= c && p < n) Lo[(int64_t)q * n + p] = col[r] * myrs;
        }
      }
    }
  }
  return bad;
}

// Broadcast lane `src` of each 16-lane row to the whole row (DPP row_newbcast).
__device__ __forceinline__ int row_bcast_i(int x, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_mov_dpp(x, 0x150, 0xF, 0xF, true);
    case 1: return __builtin_amdgcn_mov_dpp(x, 0x151, 0xF, 0xF, true);
    case 2: return __builtin_amdgcn_mov_dpp(x, 0x152, 0xF, 0xF, true);
    case 3: return __builtin_amdgcn_mov_dpp(x, 0x153, 0xF, 0xF, true);
    case 4: return __builtin_amdgcn_mov_dpp(x, 0x154, 0xF, 0xF, true);
    case 5: return __builtin_amdgcn_mov_dpp(x, 0x155, 0xF, 0xF, true);
    case 6: return __builtin_amdgcn_mov_dpp(x, 0x156, 0xF, 0xF, true);
    case 7: return __builtin_amdgcn_mov_dpp(x, 0x157, 0xF, 0xF, true);
    case 8: return __builtin_amdgcn_mov_dpp(x, 0x158, 0xF, 0xF, true);
    case 9: return __builtin_amdgcn_mov_dpp(x, 0x159, 0xF, 0xF, true);
    case 10: return __builtin_amdgcn_mov_dpp(x, 0x15A, 0xF, 0xF, true);
    case 11: return __builtin_amdgcn_mov_dpp(x, 0x15B, 0xF, 0xF, true);
    case 12: return __builtin_amdgcn_mov_dpp(x, 0x15C, 0xF, 0xF, true);
    case 13: return __builtin_amdgcn_mov_dpp(x, 0x15D, 0xF, 0xF, true);
    case 14: return __builtin_amdgcn_mov_dpp(x, 0x15E, 0xF, 0xF, true);
    default: return __builtin_amdgcn_mov_dpp(x, 0x15F, 0xF, 0xF, true);
  }
}
__device__ __forceinline__ double row_bcast(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = row_bcast_i((int)b, src);
  const int hi = row_bcast_i((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float row_bcast(float x, int src) {
  return __int_as_float(row_bcast_i(__float_as_int(x), src));
}

// Cholesky factor and inverse of one 16x16 tile stored (lower triangle) at
// `t`, by one wave, holding only 4 + 4 values per lane.  Lanes are split
// 4 x 16: lane (c, g) = c + 16 g holds rows g + 4v (v = 0..3) of column c.
// Step j takes the pivot from its lane, the pivot row across the 16-lane rows
// (lane shuffle) and the pivot column inside each row (DPP broadcast).
// Writes W = L^{-1} back to `t` (full tile, zero above the diagonal) and the
// lower triangle of L to Lo (column-major n x n, may be null) and L itself
// as a stored tile to Ld (may be null); returns the first non-positive pivot
// (or -1).
template <typename T>
__device__ __forceinline__ int potrf_c(T* t, T* Lo, int n, int k, int lane, T* Ld = nullptr) {
  const int c = lane & 15, g = lane >> 4;
  T a[4], w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = g + 4 * v;
    a[v] = r >= c ? t[r * TST + c] : t[c * TST + r];
    w[v] = r == c ? T(1) : T(0);
  }
  int bad = -1;
  T myrs = T(1);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gj = j & 3, vj = j >> 2;          // lane group / item holding row j
    const T ajc = __shfl(a[vj], c + 16 * gj, 64);    // a[j][c]
    const T wv = __shfl(w[vj], c + 16 * gj, 64);     // V[j][c]
    T ajj = readlane(a[vj], j + 16 * gj);           // a[j][j]
    if (!(ajj > T(0))) {
      if (bad < 0) bad = j;
      ajj = T(1);
    }
    const T rs = rsqrt_t(ajj);
    if (c == j) myrs = rs;
    const T wjc = wv * rs;                           // W[j][c]
    const T f = ajc * (rs * rs);
    const bool cgt = c > j;
    // items whose four rows are all above row j are final (static test);
    // the rest are updated by selects
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (4 * v + 3 < j) continue;
      const int r = g + 4 * v;
      const T arj = row_bcast(a[v], j);      // a[r][j]
      const T wu = w[v] - arj * rs * wjc;
      const T au = a[v] - arj * f;
      w[v] = r > j ? wu : (r == j ? wjc : w[v]);
      a[v] = (r > j && cgt) ? au : a[v];
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = g + 4 * v;
    t[r * TST + c] = w[v];
  }
  if (Lo) {
    const int q = 16 * k + c;
    if (q < n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = g + 4 * v, p = 16 * k + r;
        if (r >= c && p < n) Lo[(int64_t)q * n + p] = a[v] * myrs;
      }
    }
  }
  if (Ld) {   // L_kk as a stored tile (lower triangle, zero above)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = g + 4 * v;
      Ld[r * TST + c] = r >= c ? a[v] * myrs : T(0);
    }
  }
  return bad;
}

// Store the result tile (rows 16I.., cols 16J..) of L into a column-major
// n x n matrix (lower triangle only).
template <typename T>
__device__ __forceinline__ void store_L(T* Lo, int n, int I, int J, const typename Mfma<T>::v4& acc, int lane) {
  const int q = 16 * J + (lane & 15);
  if (q >= n) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int p = 16 * I + Mfma<T>::row(lane >> 4, v);
    if (p < n && p >= q) Lo[(int64_t)q * n + p] = acc[v];
  }
}

// Trailing tile t of step k -> (i, j): columns j = k+1 .. nt-1, rows i = j .. nt
// (row nt is the right-hand-side row).
__device__ __forceinline__ void trail_ij(int t, int k, int nt, int& i, int& j) {
  const int m = nt - 1 - k;
  int jj = 0, rem = t;
  while (rem >= m - jj + 1) {
    rem -= m - jj + 1;
    ++jj;
  }
  j = k + 1 + jj;
  i = j + rem;
}

}  // namespace mhm

namespace mhm {

// FP64 residual of the refinement, R = Btilde - (A X + gamma c (c^T X)),
// matrix-free from kappa (the 7-point stencil of each node), written as T
// into the right-hand-side tiles (tile J holds rows 16J.. of R^T; cx holds
// c^T X per column).  Returns the row-sum norm of Ahat (all threads).
// Btilde comes from the tables (fused) or from Btg (column-major n x r).
// DD: the products and their sum in double-double, rounded once (the FP64
// path's refinement, which must see the residual of an FP64 iterate).  An
// error in c^T X only moves the residual along c, whose correction is a
// constant that the zero-mean projection removes.
template <typename T, bool FUSED, bool DD = false>
__device__ __forceinline__ double ir_residual_body(const Elem& E, const double* kapp, const double* X,
                                                   const double* c, const double* cx, double g, const double* ft,
                                                   const double* bf, const double* colsum, const double* Btg,
                                                   T* rhs_row, double* red) {
  auto kap = [=](int t) -> double { return kapp[t]; };
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int s = E.s, n = E.n, r = E.rc, c0 = E.c0, nt = E.nt;   // the columns of the current chunk
  for (int p = tid; p < 16 * nt; p += nthr) {   // padding rows and columns of the tiles
    T* rt = rhs_row + (int64_t)(p >> 4) * TILE + (p & 15);
    for (int a = (p >= n ? 0 : r); a < 16; ++a) rt[a * TST] = T(0);
  }
  // node-outer: one stencil per node, then its right-hand sides
  double anorm = 0.0;
  for (int p = tid; p < n; p += nthr) {
    int i, j;
    node_ij(p, s, i, j);
    const Stencil st = stencil(i, j, s, E.G, kap);
    const double cp = c[p];
    anorm = fmax(anorm, fabs(st.d) + fabs(st.e) + fabs(st.w) + fabs(st.n) + fabs(st.so) + fabs(st.nw) +
                            fabs(st.se) + g * cp * E.area);
    const bool hasE = i + j <= s - 1, hasW = i >= 1, hasS = j >= 1;
    const int pE = p + 1, pN = p + (s + 1 - j), pW = p - 1, pNW = p + (s - j), pS = p - (s + 2 - j),
              pSE = p - (s + 1 - j);
    T* rt = rhs_row + (int64_t)(p >> 4) * TILE + (p & 15);
#pragma unroll 4
    for (int a = 0; a < r; ++a) {
      const double* xa = X + (int64_t)(c0 + a) * n;
      const double b = FUSED ? btilde_tab(E, ft, bf, c, colsum, c0 + a, p, i, j) : Btg[(int64_t)(c0 + a) * n + p];
      if constexpr (DD) {
        double hi = 0.0, lo = 0.0;
        dd_add_prod(hi, lo, st.d, xa[p]);
        dd_add_prod(hi, lo, cp, g * cx[a]);
        if (hasE) {
          dd_add_prod(hi, lo, st.e, xa[pE]);
          dd_add_prod(hi, lo, st.n, xa[pN]);
        }
        if (hasW) {
          dd_add_prod(hi, lo, st.w, xa[pW]);
          dd_add_prod(hi, lo, st.nw, xa[pNW]);
        }
        if (hasS) {
          dd_add_prod(hi, lo, st.so, xa[pS]);
          dd_add_prod(hi, lo, st.se, xa[pSE]);
        }
        rt[a * TST] = (T)dd_sub_from(b, hi, lo);
      } else {
        double ax = st.d * xa[p] + cp * (g * cx[a]);
        if (hasE) ax += st.e * xa[pE] + st.n * xa[pN];
        if (hasW) ax += st.w * xa[pW] + st.nw * xa[pNW];
        if (hasS) ax += st.so * xa[pS] + st.se * xa[pSE];
        rt[a * TST] = (T)(b - ax);
      }
    }
  }
  return block_max(anorm, red);   // its barriers also publish the residual tiles
}

// Per-column maxima, column a by 16-lane groups: of |residual| from the
// right-hand-side tiles (b == null), or of |Btilde| (first refinement step).
template <typename T, bool FUSED>
__device__ __forceinline__ void ir_colmax_body(const Elem& E, const T* rhs_row, const double* ft, const double* bf,
                                               const double* c, const double* colsum, const double* Btg, bool of_b,
                                               double* out, double* part) {
  const int tid = threadIdx.x, grp = tid >> 4, cl = tid & 15;
  const int gpc = blockDim.x >> 8;
  const int a = grp & 15, k = grp >> 4;
  const int n = E.n, r = E.rc, c0 = E.c0, s = E.s;
  double v = 0.0;
  if (a < r) {
    const int step = 16 * gpc;
    for (int p = 16 * k + cl; p < n; p += step) {
      double x;
      if (of_b) {
        int i, j;
        node_ij(p, s, i, j);
        x = FUSED ? btilde_tab(E, ft, bf, c, colsum, c0 + a, p, i, j) : Btg[(int64_t)(c0 + a) * n + p];
      } else {
        x = (double)rhs_row[(int64_t)(p >> 4) * TILE + a * TST + (p & 15)];
      }
      v = fmax(v, fabs(x));
    }
  }
  v = group16_max(v);
  if (cl == 0) part[k * 16 + a] = v;
  __syncthreads();
  if (tid < r) {
    double m = 0.0;
    for (int q = 0; q < gpc; ++q) m = fmax(m, part[q * 16 + tid]);
    out[tid] = m;
  }
  __syncthreads();
}

// X (n x r, FP64, column-major) = tiles (init) or X + tiles, from the
// solved right-hand-side row (tile J holds rows 16J.. of X^T), and at the
// same time cx[a] = c^T X[:, a] and xmax[a] = max |X[:, a]|.  Column a is
// handled by 16-lane groups (blockDim/256 of them, on interleaved nodes),
// four nodes in flight per lane; part[] (LDS, 32 * blockDim/256 doubles)
// combines the groups.
template <typename T>
__device__ __forceinline__ void ir_accumulate_body(double* X, const T* rhs_row, const double* c, int n, int r,
                                                   bool init, double* cx, double* xmax, double* part) {
  const int tid = threadIdx.x, grp = tid >> 4, cl = tid & 15;
  const int gpc = blockDim.x >> 8;          // groups per column
  const int a = grp & 15, k = grp >> 4;
  double v = 0.0, xm = 0.0;
  if (a < r) {
    double* xa = X + (int64_t)a * n;
    const int step = 16 * gpc;
    for (int p0 = 16 * k + cl; p0 < n; p0 += 4 * step) {
      double t[4], x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * step;
        t[u] = 0.0;
        x[u] = 0.0;
        if (p < n) {
          t[u] = (double)rhs_row[(int64_t)(p >> 4) * TILE + a * TST + (p & 15)];
          if (!init) x[u] = xa[p];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * step;
        if (p < n) {
          const double xn = x[u] + t[u];
          xa[p] = xn;
          v += c[p] * xn;
          xm = fmax(xm, fabs(xn));
        }
      }
    }
  }
  v = group16_sum(v);
  xm = group16_max(xm);
  if (cl == 0) {
    part[k * 16 + a] = v;
    part[(gpc + k) * 16 + a] = xm;
  }
  __syncthreads();
  if (tid < r) {
    double sum = 0.0, m = 0.0;
    for (int q = 0; q < gpc; ++q) {
      sum += part[q * 16 + tid];
      m = fmax(m, part[(gpc + q) * 16 + tid]);
    }
    cx[tid] = sum;
    xmax[tid] = m;
  }
  __syncthreads();
}

// The three refinement passes as separate functions, for kernels whose
// registers are already taken by their tiles (pointers may be to LDS or
// global memory); kernels with tiles in LDS inline the bodies instead.
template <typename T, bool FUSED, bool DD = false>
__device__ __noinline__ double ir_residual(const Elem& E, const double* kapp, const double* X, const double* c,
                                           const double* cx, double g, const double* ft, const double* bf,
                                           const double* colsum, const double* Btg, T* rhs_row, double* red) {
  return ir_residual_body<T, FUSED, DD>(E, kapp, X, c, cx, g, ft, bf, colsum, Btg, rhs_row, red);
}
template <typename T, bool FUSED>
__device__ __noinline__ void ir_colmax(const Elem& E, const T* rhs_row, const double* ft, const double* bf,
                                       const double* c, const double* colsum, const double* Btg, bool of_b,
                                       double* out, double* part) {
  ir_colmax_body<T, FUSED>(E, rhs_row, ft, bf, c, colsum, Btg, of_b, out, part);
}
template <typename T>
__device__ __noinline__ void ir_accumulate(double* X, const T* rhs_row, const double* c, int n, int r, bool init,
                                           double* cx, double* xmax, double* part) {
  ir_accumulate_body<T>(X, rhs_row, c, n, r, init, cx, xmax, part);
}

// Normwise backward error of the current iterate, max over the columns:
// max_p |r_pa| / (||Ahat||_inf max_p |x_pa| + max_p |b_pa|)  (0 for a zero
// residual, inf for NaN).
__device__ __forceinline__ double ir_backward_error(const double* rmax, const double* xmax, const double* bmax, int r,
                                                    double anorm) {
  double be = 0.0;
  for (int a = 0; a < r; ++a) {
    // a zero residual is converged (a zero right-hand side has zero solution)
    const double e = rmax[a] == 0.0 ? 0.0 : rmax[a] / (anorm * xmax[a] + bmax[a]);
    be = e == e ? fmax(be, e) : __builtin_inf();
  }
  return be;
}

// Refinement decision after step `it` (0 = the first solve): 1 converged,
// 0 continue, -1 give up.  Refinement contracts the error by a roughly
// constant factor per step; when the backward error grows, or from the
// second correction on the observed factor (against the previous step's
// backward error `prev`) says the tolerance cannot be reached within the
// step budget, stop now and leave the element to the FP64 pass.
__device__ __forceinline__ int ir_decide(double be, double prev, int it, int max_iters, double tol) {
  if (be <= tol) return 1;
  if (it >= max_iters) return -1;
  if (it >= 1) {
    const double rho = be / prev;
    if (!(rho < 1.0)) return -1;   // no contraction at all
    if (it >= 2) {                 // the first step's contraction can be atypical
      const double need = log(tol / be) / log(rho);
      if (need > (double)(max_iters - it)) return -1;
    }
  }
  return 0;
}

}  // namespace mhm
