// MHM local-problem kernels for gfx950 (CDNA4).
//
// k_assemble   steps a2-a3: Ahat = A + gamma c c^T (dense, column-major),
//              Btilde = B - c (1^T B)/|K|, c, |K|               (HBM-write bound)
// k_local      steps a2-a6 on 16x16 tiles: (assemble or load) -> Cholesky
//              (MFMA f64 or f32) with the forward solve of the r right-hand
//              sides carried along as an extra tile row -> backward solve
//              (MFMA) -> FP64 matrix-free refinement (FP32 path) -> zero-mean
//              projection -> optional contribution.  Tiles live in LDS when
//              the element fits, else in a per-workgroup workspace slot.
// k_contrib    step a6: the element's blocks of the skeleton system.
//
// One workgroup of 256 threads (4 waves of 64) handles one element at a time.
#include "mhm_device.h"
#include "mhm_kernels.h"

namespace mhm {

constexpr int NTHREADS = 256;
constexpr int NWAVES = NTHREADS / 64;

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
// Block-wide sums of three values; every thread gets the results.
// `red` holds 3*NWAVES doubles.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[NWAVES + w] = b;
    red[2 * NWAVES + w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int k = 0; k < NWAVES; ++k) {
    a += red[k];
    b += red[NWAVES + k];
    c += red[2 * NWAVES + k];
  }
}
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int k = 1; k < NWAVES; ++k) t = fmax(t, red[k]);
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
  const int sp1 = E.s + 1, lp1 = E.l + 1;
  for (int idx = threadIdx.x; idx < E.NI * sp1; idx += NTHREADS) {
    const int a = idx / sp1, k = idx - a * sp1;
    const int e = a / lp1, q = a - e * lp1;
    ft[idx] = face_load(E, e, q, k);
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
    const int e = a / (E.l + 1);
    const int k = face_pos(e, i, j, E.s);
    if (k >= 0) v = ft[a * (E.s + 1) + k];
  } else {
    v = bf[p];
  }
  return v - c[p] * colsum[a] * E.inv_area;
}

// =============================================================== k_assemble
__global__ void __launch_bounds__(NTHREADS) k_assemble(BatchDev b, double* Ahat, double* Btil, double* cout,
                                                        double* area, int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double red[3 * NWAVES];
  __shared__ double colsum[16];
  __shared__ double gam;
  extern __shared__ double dyn[];   // kappa[s^2] | c[n] | bf[n] | ft[NI(s+1)]
  const int tid = threadIdx.x;
  const int smax = b.s_max, nmax = (smax + 1) * (smax + 2) / 2;
  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();
    if (tid == 0) {
      ok = load_elem(b, e, E) && E.mat0 >= 0 && E.rhs0 >= 0 && E.node0 >= 0;
      if (info) info[e] = ok ? INFO_OK : INFO_BAD_DESC;
    }
    __syncthreads();
    if (!ok) continue;
    const int s = E.s, n = E.n, r = E.r, T = s * s;
    double* kap = dyn;
    double* c = kap + smax * smax;
    double* bf = c + nmax;
    double* ft = bf + nmax;
    for (int t = tid; t < T; t += NTHREADS) kap[t] = b.kappa[E.tri0 + t];
    face_table(E, ft);
    __syncthreads();
    double tr = 0.0, cc2 = 0.0, fs = 0.0;
    const double* fp = b.f + E.tri0;
    for (int p = tid; p < n; p += NTHREADS) {
      int i, j;
      node_ij(p, s, i, j);
      const Stencil st = stencil(i, j, s, E.G, [&](int t) { return kap[t]; });
      const double cp = st.cnt * E.cunit;
      const double bp = E.cunit * node_tri_sum(i, j, s, [&](int t) { return fp[t]; });
      c[p] = cp;
      bf[p] = bp;
      tr += st.d;
      cc2 += cp * cp;
      fs += bp;
    }
    block_sum3(tr, cc2, fs, red);
    if (tid == 0) {
      gam = tr / (n * cc2);
      colsum[E.NI] = fs;
    }
    face_colsums(E, ft, colsum);
    __syncthreads();
    const double g = gam;
    // Ahat: wave w writes columns q = w, w+4, ...; lanes sweep rows.
    const int w = tid >> 6, lane = tid & 63;
    double* A = Ahat + E.mat0;
    for (int q = w; q < n; q += NWAVES) {
      int i, j;
      node_ij(q, s, i, j);
      const Stencil st = stencil(i, j, s, E.G, [&](int t) { return kap[t]; });
      const int pE = q + 1, pW = q - 1, pN = q + (s + 1 - j), pS = q - (s + 2 - j), pNW = q + (s - j),
                pSE = q - (s + 1 - j);
      const double gcq = g * c[q];
      for (int p = lane; p < n; p += 64) {
        double v = gcq * c[p];
        v += (p == q) ? st.d : 0.0;
        v += (p == pE) ? st.e : 0.0;
        v += (p == pW) ? st.w : 0.0;
        v += (p == pN) ? st.n : 0.0;
        v += (p == pS) ? st.so : 0.0;
        v += (p == pNW) ? st.nw : 0.0;
        v += (p == pSE) ? st.se : 0.0;
        A[(int64_t)q * n + p] = v;
      }
    }
    double* Bt = Btil + E.rhs0;
    for (int idx = tid; idx < n * r; idx += NTHREADS) {
      const int a = idx / n, p = idx - a * n;
      int i, j;
      node_ij(p, s, i, j);
      Bt[idx] = btilde_tab(E, ft, bf, c, colsum, a, p, i, j);
    }
    for (int p = tid; p < n; p += NTHREADS) cout[E.node0 + p] = c[p];
    if (tid == 0 && area) area[e] = E.area;
  }
}

// ============================================================ contribution
// M[a][b] = -sum_k R(a,k) X[node(a,k)][b], E[a] = sum_k R(a,k) X[node(a,k)][NI],
// B[a] = -sum_k R(a,k), F = integral of f (= colsum of the source column).
// X column-major n x r (already projected); ft the face table.
__device__ __forceinline__ void contrib_element(const Elem& E, const double* X, const double* ft, double Fval, int NImax,
                                double* M, double* Ev, double* Bv, double* F, int e) {
  const int tid = threadIdx.x;
  const int NI = E.NI, n = E.n, lp1 = E.l + 1, s = E.s, sp1 = s + 1;
  double* Me = M + (int64_t)e * NImax * NImax;
  for (int idx = tid; idx < NImax * NImax; idx += NTHREADS) {
    const int a = idx % NImax, bb = idx / NImax;
    if (a >= NI || bb >= NI) Me[idx] = 0.0;
  }
  if (tid < NI * E.r) {
    const int a = tid % NI, bb = tid / NI;
    const int ef = a / lp1;
    const double* fa = ft + a * sp1;
    const double* xb = X + (int64_t)bb * n;
    double v = 0.0;
    for (int k = 0; k < sp1; ++k) v += fa[k] * xb[face_node(ef, k, s)];
    if (bb < NI) Me[(int64_t)bb * NImax + a] = -v;
    else Ev[(int64_t)e * NImax + a] = v;
  } else if (tid >= 240 && tid < 240 + NImax) {
    const int a = tid - 240;
    double v = 0.0;
    if (a < NI) {
      for (int k = 0; k < sp1; ++k) v -= ft[a * sp1 + k];
    } else {
      Ev[(int64_t)e * NImax + a] = 0.0;
    }
    Bv[(int64_t)e * NImax + a] = v;
  }
  if (tid == 255) F[e] = Fval;
}

__global__ void __launch_bounds__(NTHREADS) k_contrib(BatchDev b, const double* X, double* M, double* Ev,
                                                       double* Bv, double* F, const int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double red[3 * NWAVES];
  __shared__ double fsum;
  extern __shared__ double ft[];   // NI(s+1)
  const int NImax = 3 * (b.l_max + 1);
  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();
    if (threadIdx.x == 0) ok = (info == nullptr || info[e] == 0 || info[e] == INFO_IR_FALLBACK) &&
                               load_elem(b, e, E) && E.rhs0 >= 0;
    __syncthreads();
    if (!ok) continue;
    face_table(E, ft);
    double fs = 0.0, z1 = 0.0, z2 = 0.0;
    for (int t = threadIdx.x; t < E.s * E.s; t += NTHREADS) fs += b.f[E.tri0 + t];
    block_sum3(fs, z1, z2, red);   // barriers: ft visible afterwards
    if (threadIdx.x == 0) fsum = fs * (E.area / ((double)E.s * E.s));
    __syncthreads();
    contrib_element(E, X + E.rhs0, ft, fsum, NImax, M, Ev, Bv, F, e);
  }
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

template <typename T, bool IN_LDS, bool FUSED>
__global__ void __launch_bounds__(NTHREADS) k_local(BatchDev b, LocalArgs args) {
  typedef typename Mfma<T>::v4 V4;
  __shared__ Elem E;
  __shared__ int ok, bad, conv;
  __shared__ double red[3 * NWAVES];
  __shared__ double colsum[16];
  __shared__ double cx[16];          // (c^T X) per column
  __shared__ double gam;
  __shared__ double wred[NWAVES][3][16];
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NImax = 3 * (b.l_max + 1);
  const bool fp32 = sizeof(T) == 4;

  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();   // every thread is done with the previous element's shared flags
    if (tid == 0) {
      int st = INFO_OK;
      if (args.only_fallback && args.info[e] != INFO_IR_FALLBACK) {
        ok = 0;
      } else {
        const bool good = load_elem(b, e, E) && E.rhs0 >= 0 && (FUSED || E.mat0 >= 0);
        if (!good) st = INFO_BAD_DESC;
        else if ((E.nt * (E.nt + 1)) / 2 + E.nt > args.tile_cap || E.n > args.n_cap ||
                 (FUSED && E.NI * (E.s + 1) > args.f_cap) || (FUSED && IN_LDS && E.s * E.s > args.k_cap))
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

    const int s = E.s, n = E.n, r = E.r, nt = E.nt, T2 = s * s;
    // dynamic LDS: c[n_cap] | bf[n_cap] | ft[f_cap] | kap[k_cap] | tiles (IN_LDS)
    double* c = dyn;
    double* bf = c + args.n_cap;
    double* ft = bf + args.n_cap;
    double* kapl = ft + args.f_cap;
    const bool kap_lds = FUSED && IN_LDS;
    T* tiles = IN_LDS ? reinterpret_cast<T*>(kapl + args.k_cap)
                      : reinterpret_cast<T*>(args.ws) + (int64_t)blockIdx.x * args.ws_slot;
    // tile (I,J), J <= I <= nt; row nt holds the right-hand sides (transposed)
    auto tl = [&](int I, int J) -> T* { return tiles + (int64_t)((I * (I + 1)) / 2 + J) * TILE; };
    const double* kapg = b.kappa + E.tri0;
    auto kap = [&](int t) -> double { return kap_lds ? kapl[t] : kapg[t]; };

    // ------------------------------------------------------------- set-up
    if (kap_lds)
      for (int t = tid; t < T2; t += NTHREADS) kapl[t] = kapg[t];
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

    // ---------------------------------------------------------- fill tiles
    if (FUSED) {
      const double g = gam;
      const int rr = tid >> 4, cl = tid & 15;
      for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
          const int p = 16 * I + rr, q = 16 * J + cl;
          const double v = (p < n && q < n) ? g * c[p] * c[q] : (p == q ? 1.0 : 0.0);
          tl(I, J)[rr * TST + cl] = (T)v;
        }
      __syncthreads();
      for (int q = tid; q < n; q += NTHREADS) {
        int i, j;
        node_ij(q, s, i, j);
        const Stencil st = stencil(i, j, s, E.G, kap);
        auto add = [&](int p, double v) {
          T* t = tl(p >> 4, q >> 4);
          t[(p & 15) * TST + (q & 15)] += (T)v;
        };
        add(q, st.d);
        if (i + j <= s - 1) {
          add(q + 1, st.e);
          add(q + (s + 1 - j), st.n);
        }
        if (i >= 1) add(q + (s - j), st.nw);
      }
      for (int J = 0; J < nt; ++J) {
        const int a = rr, p = 16 * J + cl;
        double v = 0.0;
        if (a < r && p < n) {
          int i, j;
          node_ij(p, s, i, j);
          v = btilde_tab(E, ft, bf, c, colsum, a, p, i, j);
        }
        tl(nt, J)[a * TST + cl] = (T)v;
      }
    } else {
      const double* A = args.Ahat + E.mat0;
      const int rr = tid & 15, cl = tid >> 4;
      for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
          const int p = 16 * I + rr, q = 16 * J + cl;
          const double v = (p < n && q < n) ? A[(int64_t)q * n + p] : (p == q ? 1.0 : 0.0);
          tl(I, J)[rr * TST + cl] = (T)v;
        }
      const double* Bt = args.Btil + E.rhs0;
      for (int J = 0; J < nt; ++J) {
        const int a = tid >> 4, p = 16 * J + (tid & 15);
        const double v = (a < r && p < n) ? Bt[(int64_t)a * n + p] : 0.0;
        tl(nt, J)[a * TST + (tid & 15)] = (T)v;
      }
    }
    __syncthreads();

    // ------------------------------------------------------- factorisation
    // Right-looking over tile columns k; the right-hand-side row nt is
    // eliminated with the matrix, so it ends holding Y^T = (L^{-1} Btilde)^T.
    // Look-ahead: wave 0 updates tile (k+1,k+1) first and factors it while
    // the other waves finish the trailing update of step k.
    T* Lo = nullptr;
    if (args.Lout && E.mat0 >= 0) Lo = reinterpret_cast<T*>(args.Lout + E.mat0);
    // Step k = -1 only factors the first diagonal tile.
    for (int k = -1; k < nt; ++k) {
      if (k >= 0) {
        // panel: L_ik = A_ik W_kk^T, i = k+1 .. nt
        for (int i = k + 1 + wave; i <= nt; i += 2 * NWAVES) {
          const int i2 = i + NWAVES;
          const bool two = i2 <= nt;
          V4 a1 = {0, 0, 0, 0}, a2 = {0, 0, 0, 0};
          const T* W = tl(k, k);
          const T* A1 = tl(i, k);
          const T* A2 = tl(two ? i2 : i, k);
#pragma unroll
          for (int cch = 0; cch < 4; ++cch) {
            const T wv = ld_rowcol(W, cch, lane);
            a1 = Mfma<T>::op(ld_rowcol(A1, cch, lane), wv, a1);
            a2 = Mfma<T>::op(ld_rowcol(A2, cch, lane), wv, a2);
          }
          st_acc<T>(tl(i, k), a1, lane);
          if (Lo && i < nt) store_L<T>(Lo, n, i, k, a1, lane);
          if (two) {
            st_acc<T>(tl(i2, k), a2, lane);
            if (Lo && i2 < nt) store_L<T>(Lo, n, i2, k, a2, lane);
          }
        }
        __syncthreads();
      }
      // trailing update C_ij -= L_ik L_jk^T (k < j <= i <= nt); wave 0 takes
      // tile (k+1, k+1) (trailing tile 0) and factors it
      const int m = nt - 1 - k;
      if (wave == 0) {
        if (m > 0) {
          if (k >= 0) {
            V4 acc = ld_acc<T>(tl(k + 1, k + 1), lane);
            mma_sub_nt<T>(acc, tl(k + 1, k), tl(k + 1, k), lane);
            st_acc<T>(tl(k + 1, k + 1), acc, lane);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // the stores above before the reads below
          }
          const int bj = potrf_tile<T>(tl(k + 1, k + 1), Lo, n, k + 1, lane);
          if (lane == 0 && bj >= 0 && bad < 0) bad = 16 * (k + 1) + bj;
        }
      } else if (k >= 0 && m > 0) {
        const int ntr = m * (m + 3) / 2;
        const int nw = NWAVES - 1;
        for (int t = wave; t < ntr; t += 2 * nw) {
          const int t2 = t + nw;
          const bool two = t2 < ntr;
          int i1, j1, i2, j2;
          trail_ij(t, k, nt, i1, j1);
          if (two) {
            trail_ij(t2, k, nt, i2, j2);
          } else {
            i2 = i1;
            j2 = j1;
          }
          V4 c1 = ld_acc<T>(tl(i1, j1), lane);
          V4 c2 = ld_acc<T>(tl(i2, j2), lane);
          const T* Li1 = tl(i1, k);
          const T* Lj1 = tl(j1, k);
          const T* Li2 = tl(i2, k);
          const T* Lj2 = tl(j2, k);
#pragma unroll
          for (int cch = 0; cch < 4; ++cch) {
            c1 = Mfma<T>::op(-ld_rowcol(Li1, cch, lane), ld_rowcol(Lj1, cch, lane), c1);
            c2 = Mfma<T>::op(-ld_rowcol(Li2, cch, lane), ld_rowcol(Lj2, cch, lane), c2);
          }
          st_acc<T>(tl(i1, j1), c1, lane);
          if (two) st_acc<T>(tl(i2, j2), c2, lane);
        }
      }
      __syncthreads();
    }

    // ---------------------------------------------- solves on the RHS row
    // Stored RHS tile J holds Z_J^T (rows: right-hand sides, cols: nodes).
    auto backward = [&]() {
      for (int j = nt - 1; j >= 0; --j) {  // X = L^{-T} Y
        if (wave == (j & (NWAVES - 1))) {
          V4 acc = {0, 0, 0, 0};
          mma_add_nn<T>(acc, tl(nt, j), tl(j, j), lane);   // X_j^T = Z_j^T W_j
          st_acc<T>(tl(nt, j), acc, lane);
        }
        __syncthreads();
        for (int i = wave; i < j; i += NWAVES) {
          V4 acc = ld_acc<T>(tl(nt, i), lane);
          mma_sub_nn<T>(acc, tl(nt, j), tl(j, i), lane);  // Z_i^T -= X_j^T L_ji
          st_acc<T>(tl(nt, i), acc, lane);
        }
        __syncthreads();
      }
    };
    auto forward = [&]() {
      for (int j = 0; j < nt; ++j) {       // Y = L^{-1} Z
        if (wave == (j & (NWAVES - 1))) {
          V4 acc = {0, 0, 0, 0};
          mma_add_nt<T>(acc, tl(nt, j), tl(j, j), lane);   // Y_j^T = Z_j^T W_j^T
          st_acc<T>(tl(nt, j), acc, lane);
        }
        __syncthreads();
        for (int i = j + 1 + wave; i < nt; i += NWAVES) {
          V4 acc = ld_acc<T>(tl(nt, i), lane);
          mma_sub_nt<T>(acc, tl(nt, j), tl(i, j), lane);  // Z_i^T -= Y_j^T L_ij^T
          st_acc<T>(tl(nt, i), acc, lane);
        }
        __syncthreads();
      }
    };
    backward();
    const bool failed = bad >= 0;

    double* X = args.X + E.rhs0;
    const int ca = tid >> 4, cl16 = tid & 15;   // 16 columns x 16 lanes for column sums

    if (fp32 && !failed) {
      // --------------------------------------- FP64 refinement (FP32 path)
      for (int idx = tid; idx < n * r; idx += NTHREADS) {
        const int a = idx / n, p = idx - a * n;
        X[idx] = (double)tl(nt, p >> 4)[a * TST + (p & 15)];
      }
      __syncthreads();
      const double* Btg = FUSED ? nullptr : args.Btil + E.rhs0;
      const double g = gam;
      int it = 0;
      for (;; ++it) {
        {  // c^T X per column
          double v = 0.0;
          if (ca < r)
            for (int p = cl16; p < n; p += 16) v += c[p] * X[(int64_t)ca * n + p];
          v = group16_sum(v);
          if (cl16 == 0) cx[ca] = v;
        }
        __syncthreads();
        // residual R = Btilde - (A X + gamma c (c^T X)) into the RHS tiles (FP32)
        double rmax[16], xmax[16], bmax[16];
        double anorm = 0.0;
#pragma unroll
        for (int a = 0; a < 16; ++a) rmax[a] = xmax[a] = bmax[a] = 0.0;
        for (int p = tid; p < 16 * nt; p += NTHREADS) {
          if (p >= n) {
            for (int a = 0; a < 16; ++a) tl(nt, p >> 4)[a * TST + (p & 15)] = T(0);
            continue;
          }
          int i, j;
          node_ij(p, s, i, j);
          const Stencil st = stencil(i, j, s, E.G, kap);
          const double cp = c[p];
          anorm = fmax(anorm, fabs(st.d) + fabs(st.e) + fabs(st.w) + fabs(st.n) + fabs(st.so) + fabs(st.nw) +
                                   fabs(st.se) + g * cp * E.area);
          const int pE = p + 1, pW = p - 1, pN = p + (s + 1 - j), pS = p - (s + 2 - j), pNW = p + (s - j),
                    pSE = p - (s + 1 - j);
          const bool hE = i + j <= s - 1, hW = i >= 1, hN = i + j <= s - 1, hS = j >= 1, hNW = i >= 1, hSE = j >= 1;
#pragma unroll
          for (int a = 0; a < 16; ++a) {
            double rv = 0.0;
            if (a < r) {
              const double* xa = X + (int64_t)a * n;
              double ax = st.d * xa[p] + g * cp * cx[a];
              if (hE) ax += st.e * xa[pE];
              if (hW) ax += st.w * xa[pW];
              if (hN) ax += st.n * xa[pN];
              if (hS) ax += st.so * xa[pS];
              if (hNW) ax += st.nw * xa[pNW];
              if (hSE) ax += st.se * xa[pSE];
              const double bv = FUSED ? btilde_tab(E, ft, bf, c, colsum, a, p, i, j) : Btg[(int64_t)a * n + p];
              rv = bv - ax;
              rmax[a] = fmax(rmax[a], fabs(rv));
              xmax[a] = fmax(xmax[a], fabs(xa[p]));
              bmax[a] = fmax(bmax[a], fabs(bv));
            }
            tl(nt, p >> 4)[a * TST + (p & 15)] = (T)rv;
          }
        }
        anorm = block_max(anorm, red);
#pragma unroll
        for (int a = 0; a < 16; ++a) {
          rmax[a] = wave_max(rmax[a]);
          xmax[a] = wave_max(xmax[a]);
          bmax[a] = wave_max(bmax[a]);
        }
        if (lane == 0)
          for (int a = 0; a < 16; ++a) {
            wred[wave][0][a] = rmax[a];
            wred[wave][1][a] = xmax[a];
            wred[wave][2][a] = bmax[a];
          }
        __syncthreads();
        if (tid == 0) {
          bool cv = true;
          for (int a = 0; a < r; ++a) {
            double rm = 0, xm = 0, bm = 0;
            for (int w2 = 0; w2 < NWAVES; ++w2) {
              rm = fmax(rm, wred[w2][0][a]);
              xm = fmax(xm, wred[w2][1][a]);
              bm = fmax(bm, wred[w2][2][a]);
            }
            if (!(rm <= args.ir_tol * (anorm * xm + bm))) cv = false;
          }
          conv = cv;
        }
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
      if (!cvd) continue;   // recomputed by the FP64 fallback pass
      {  // zero-mean projection of the FP64 iterate
        double v = 0.0;
        if (ca < r)
          for (int p = cl16; p < n; p += 16) v += c[p] * X[(int64_t)ca * n + p];
        v = group16_sum(v);
        if (cl16 == 0) cx[ca] = v * E.inv_area;
      }
      __syncthreads();
      for (int idx = tid; idx < n * r; idx += NTHREADS) X[idx] -= cx[idx / n];
      __syncthreads();
    } else if (fp32) {
      // FP32 pivot failure: recomputed by the FP64 fallback pass
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
      {  // zero-mean projection in FP64, straight from the solved tiles
        double v = 0.0;
        if (ca < r)
          for (int p = cl16; p < n; p += 16) v += c[p] * (double)tl(nt, p >> 4)[ca * TST + (p & 15)];
        v = group16_sum(v);
        if (cl16 == 0) cx[ca] = v * E.inv_area;
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

// ------------------------------------------------------------- host launchers
int local_face_cap(const mhm_batch* bt) { return 3 * (bt->l_max + 1) * (bt->s_max + 1); }

hipError_t launch_assemble(const mhm_batch* bt, double* Ahat, double* Btil, double* c, double* area, int32_t* info,
                           int grid, hipStream_t st) {
  const int smax = bt->s_max;
  const int nmax = (smax + 1) * (smax + 2) / 2;
  const size_t lds = sizeof(double) * ((size_t)smax * smax + 2 * (size_t)nmax + local_face_cap(bt));
  hipError_t err = hipFuncSetAttribute((const void*)k_assemble, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_assemble, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), Ahat, Btil, c, area, info);
  return hipGetLastError();
}

hipError_t launch_contrib(const mhm_batch* bt, const double* X, double* M, double* E, double* B, double* F,
                          const int32_t* info, int grid, hipStream_t st) {
  const size_t lds = sizeof(double) * local_face_cap(bt);
  hipError_t err = hipFuncSetAttribute((const void*)k_contrib, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_contrib, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), X, M, E, B, F, info);
  return hipGetLastError();
}

template <typename T, bool IN_LDS, bool FUSED>
static hipError_t launch_local_t(const mhm_batch* bt, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  auto kern = k_local<T, IN_LDS, FUSED>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), a);
  return hipGetLastError();
}

size_t local_lds_bytes(bool fp32, bool in_lds, int n_cap, int f_cap, int k_cap, int tile_cap) {
  size_t bytes = sizeof(double) * (2 * (size_t)n_cap + (size_t)f_cap + (size_t)k_cap);
  if (in_lds) bytes += (size_t)tile_cap * TILE * (fp32 ? sizeof(float) : sizeof(double));
  return bytes;
}

hipError_t launch_local(bool fp32, bool in_lds, bool fused, const mhm_batch* bt, LocalArgs a, size_t lds, int grid,
                        hipStream_t st) {
  if (fp32) {
    if (in_lds) return fused ? launch_local_t<float, true, true>(bt, a, lds, grid, st)
                             : launch_local_t<float, true, false>(bt, a, lds, grid, st);
    return fused ? launch_local_t<float, false, true>(bt, a, lds, grid, st)
                 : launch_local_t<float, false, false>(bt, a, lds, grid, st);
  }
  if (in_lds) return fused ? launch_local_t<double, true, true>(bt, a, lds, grid, st)
                           : launch_local_t<double, true, false>(bt, a, lds, grid, st);
  return fused ? launch_local_t<double, false, true>(bt, a, lds, grid, st)
               : launch_local_t<double, false, false>(bt, a, lds, grid, st);
}

}  // namespace mhm
