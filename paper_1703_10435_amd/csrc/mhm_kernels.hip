// MHM local-problem kernels for gfx950 (CDNA4).
//
// k_assemble   steps a2-a3: Ahat = A + gamma c c^T (dense, column-major),
//              Btilde = B - c (1^T B)/|K|, c, |K|               (HBM-write bound)
// k_local      steps a2-a6 on 16x16 tiles: (assemble or load) -> Cholesky
//              (MFMA f64 or f32) -> forward/backward solves of the r
//              right-hand sides (MFMA) -> FP64 matrix-free refinement (FP32
//              path) -> zero-mean projection -> optional contribution.
//              Tiles live in LDS when the element fits, else in a
//              per-workgroup slot of a device workspace.
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
// Block-wide sum; every thread gets the result.  `red` holds NWAVES doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NWAVES; ++k) t += red[k];
  return t;
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
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return 1.0f / sqrtf(x); }

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

// R[p][a] for node (i,j) and face column a (0 if the node is not on that face).
__device__ __forceinline__ double face_load_node(const Elem& E, int a, int i, int j) {
  const int e = a / (E.l + 1), q = a - e * (E.l + 1);
  const int k = face_pos(e, i, j, E.s);
  return k < 0 ? 0.0 : face_load(E, e, q, k);
}

// Column sums 1^T B: face columns from the face nodes, the source column from
// the sub-triangles (1^T b_f = integral of f).  Result in colsum[0..r-1].
__device__ void rhs_column_sums(const Elem& E, const BatchDev& b, double* colsum, double* red) {
  const int tid = threadIdx.x;
  const int lp1 = E.l + 1;
  // face columns: one wave per column, lanes over the s+1 face nodes
  const int w = tid >> 6, lane = tid & 63;
  for (int a = w; a < E.NI; a += NWAVES) {
    const int e = a / lp1, q = a - e * lp1;
    double v = 0.0;
    for (int k = lane; k <= E.s; k += 64) v += face_load(E, e, q, k);
    v = wave_sum(v);
    if (lane == 0) colsum[a] = v;
  }
  double fs = 0.0;
  const int T = E.s * E.s;
  for (int t = tid; t < T; t += NTHREADS) fs += b.f[E.tri0 + t];
  fs = block_sum(fs, red);   // contains barriers
  if (tid == 0) colsum[E.NI] = fs * (E.area / ((double)E.s * E.s));
  __syncthreads();
}

// Btilde[p][a] for node p = (i,j).
__device__ __forceinline__ double btilde_entry(const Elem& E, const BatchDev& b, const double* colsum,
                                               int a, int i, int j, double cp) {
  double v;
  if (a < E.NI) {
    v = face_load_node(E, a, i, j);
  } else {
    const double* fp = b.f + E.tri0;
    v = E.cunit * node_tri_sum(i, j, E.s, [&](int t) { return fp[t]; });
  }
  return v - cp * colsum[a] / E.area;
}

// =============================================================== k_assemble
__global__ void __launch_bounds__(NTHREADS) k_assemble(BatchDev b, double* Ahat, double* Btil, double* cout,
                                                        double* area, int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double red[NWAVES];
  __shared__ double colsum[16];
  __shared__ double gam;
  extern __shared__ double dyn[];   // kappa[s*s], c[n]
  const int tid = threadIdx.x;
  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();
    if (tid == 0) {
      ok = load_elem(b, e, E) && E.mat0 >= 0 && E.rhs0 >= 0 && E.node0 >= 0;
      if (info) info[e] = ok ? INFO_OK : INFO_BAD_DESC;
    }
    __syncthreads();
    if (!ok) { __syncthreads(); continue; }
    const int s = E.s, n = E.n, r = E.r, T = s * s;
    double* kap = dyn;
    double* c = dyn + T;
    for (int t = tid; t < T; t += NTHREADS) kap[t] = b.kappa[E.tri0 + t];
    __syncthreads();
    double tr = 0.0, cc2 = 0.0;
    for (int p = tid; p < n; p += NTHREADS) {
      int i, j;
      node_ij(p, s, i, j);
      const Stencil st = stencil(i, j, s, E.G, [&](int t) { return kap[t]; });
      const double cp = st.cnt * E.cunit;
      c[p] = cp;
      tr += st.d;
      cc2 += cp * cp;
    }
    tr = block_sum(tr, red);
    cc2 = block_sum(cc2, red);
    if (tid == 0) gam = tr / (n * cc2);
    rhs_column_sums(E, b, colsum, red);   // ends with a barrier; c[] visible
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
    // Btilde, column-major n x r
    double* Bt = Btil + E.rhs0;
    for (int idx = tid; idx < n * r; idx += NTHREADS) {
      const int a = idx / n, p = idx - a * n;
      int i, j;
      node_ij(p, s, i, j);
      Bt[idx] = btilde_entry(E, b, colsum, a, i, j, c[p]);
    }
    for (int p = tid; p < n; p += NTHREADS) cout[E.node0 + p] = c[p];
    if (tid == 0 && area) area[e] = E.area;
    __syncthreads();
  }
}

// ============================================================ contribution
// M[a][b] = -sum_k R(a,k) X[node(a,k)][b], E[a] = sum_k R(a,k) X[node(a,k)][NI],
// B[a] = -sum_k R(a,k), F = integral of f.  X column-major n x r.
__device__ void contrib_element(const Elem& E, const BatchDev& b, const double* X, int NImax, double* M,
                                double* Ev, double* Bv, double* F, int e, double* red) {
  const int tid = threadIdx.x;
  const int NI = E.NI, n = E.n, lp1 = E.l + 1, s = E.s;
  double* Me = M + (int64_t)e * NImax * NImax;
  for (int idx = tid; idx < NImax * NImax; idx += NTHREADS) {
    const int a = idx % NImax, bb = idx / NImax;
    if (a >= NI || bb >= NI) Me[idx] = 0.0;
  }
  if (tid < NI * E.r) {
    const int a = tid % NI, bb = tid / NI;
    const int ef = a / lp1, q = a - ef * lp1;
    double v = 0.0;
    for (int k = 0; k <= s; ++k) v += face_load(E, ef, q, k) * X[(int64_t)bb * n + face_node(ef, k, s)];
    if (bb < NI) Me[(int64_t)bb * NImax + a] = -v;
    else Ev[(int64_t)e * NImax + a] = v;
  } else if (tid >= 240 && tid < 240 + NImax) {
    const int a = tid - 240;
    double v = 0.0;
    if (a < NI) {
      const int ef = a / lp1, q = a - ef * lp1;
      for (int k = 0; k <= s; ++k) v -= face_load(E, ef, q, k);
    } else {
      Ev[(int64_t)e * NImax + a] = 0.0;
    }
    Bv[(int64_t)e * NImax + a] = v;
  }
  double fs = 0.0;
  for (int t = tid; t < s * s; t += NTHREADS) fs += b.f[E.tri0 + t];
  fs = block_sum(fs, red);
  if (tid == 0) F[e] = fs * (E.area / ((double)s * s));
}

__global__ void __launch_bounds__(NTHREADS) k_contrib(BatchDev b, const double* X, double* M, double* Ev,
                                                       double* Bv, double* F, const int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double red[NWAVES];
  const int NImax = 3 * (b.l_max + 1);
  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    if (threadIdx.x == 0) ok = (info == nullptr || info[e] == 0 || info[e] == INFO_IR_FALLBACK) &&
                               load_elem(b, e, E) && E.rhs0 >= 0;
    __syncthreads();
    if (ok) contrib_element(E, b, X + E.rhs0, NImax, M, Ev, Bv, F, e, red);
    __syncthreads();
  }
}

// ================================================================== k_local
// Diagonal tile: Cholesky factor L and its inverse W = L^{-1}, by one wave, in
// registers (MFMA result layout of T), right-looking over the 16 columns.
// Reads the lower triangle of `t`; returns the first failing column or -1.
template <typename T>
__device__ int potrf_inv_tile(const T* t, typename Mfma<T>::v4& lv, typename Mfma<T>::v4& wv, int lane) {
  typedef Mfma<T> MF;
  const int cc = lane & 15, g = lane >> 4;
  T a[4], w[4], l[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = MF::row(g, v);
    a[v] = r >= cc ? t[r * TST + cc] : t[cc * TST + r];
    w[v] = r == cc ? T(1) : T(0);
    l[v] = T(0);
  }
  int bad = -1;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gj = MF::grp(j), vj = MF::item(j);    // lane group and item holding row j
    T ajj = readlane(a[vj], j + 16 * gj);
    if (!(ajj > T(0))) {
      if (bad < 0) bad = j;
      ajj = T(1);
    }
    const T rs = rsqrt_t(ajj);
    T colv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) colv[v] = shfl(a[v], j + 16 * g);          // a[row(g,v)][j]
    const T rowv = shfl(a[vj], cc + 16 * gj);                               // a[j][cc]
    const T wrow = shfl(w[vj], cc + 16 * gj) * rs;                          // W[j][cc]
    const T inv = rs * rs;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = MF::row(g, v);
      const T lc = r >= j ? colv[v] * rs : T(0);                             // L[r][j]
      if (cc == j) l[v] = lc;
      a[v] -= colv[v] * rowv * inv;
      if (r > j) w[v] -= lc * wrow;
      else if (r == j) w[v] = wrow;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    lv[v] = l[v];
    wv[v] = w[v];
  }
  return bad;
}

// Store the accumulator tile (rows 16I.., cols 16J..) of L into a column-major
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

template <typename T, bool IN_LDS, bool FUSED>
__global__ void __launch_bounds__(NTHREADS) k_local(BatchDev b, LocalArgs args) {
  __shared__ Elem E;
  __shared__ int ok, bad, conv;
  __shared__ double red[NWAVES];
  __shared__ double colsum[16];
  __shared__ double cx[16];          // c^T X per column
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
        else if ((E.nt * (E.nt + 1)) / 2 + E.nt > args.tile_cap || E.n > args.n_cap) st = INFO_TOO_LARGE;
        ok = st == INFO_OK;
        if (!ok || !args.only_fallback) args.info[e] = st;
        if (args.ir_iters && !args.only_fallback) args.ir_iters[e] = 0;
      }
      bad = -1;
      conv = 0;
    }
    __syncthreads();
    if (!ok) { __syncthreads(); continue; }

    const int s = E.s, n = E.n, r = E.r, nt = E.nt, T2 = s * s;
    // dynamic LDS: c[n_cap] | kap[k_cap] (fused, in LDS) | tiles (IN_LDS)
    double* c = dyn;
    double* kapl = dyn + args.n_cap;
    const bool kap_lds = FUSED && IN_LDS;
    T* tiles = IN_LDS ? reinterpret_cast<T*>(dyn + args.n_cap + args.k_cap)
                      : reinterpret_cast<T*>(args.ws) + (int64_t)blockIdx.x * args.ws_slot;
    auto tl = [&](int I, int J) -> T* { return tiles + (int64_t)((I * (I + 1)) / 2 + J) * TILE; };
    auto tr_ = [&](int J) -> T* { return tiles + (int64_t)((nt * (nt + 1)) / 2 + J) * TILE; };
    const double* kapg = b.kappa + E.tri0;
    auto kap = [&](int t) -> double { return kap_lds ? kapl[t] : kapg[t]; };

    if (kap_lds)
      for (int t = tid; t < T2; t += NTHREADS) kapl[t] = kapg[t];
    __syncthreads();
    // c (closed form), gamma
    double tr = 0.0, cc2 = 0.0;
    for (int p = tid; p < n; p += NTHREADS) {
      int i, j;
      node_ij(p, s, i, j);
      const double cp = node_tri_count(i, j, s) * E.cunit;
      c[p] = cp;
      cc2 += cp * cp;
      if (FUSED) tr += stencil(i, j, s, E.G, kap).d;
    }
    cc2 = block_sum(cc2, red);
    if (FUSED) {
      tr = block_sum(tr, red);
      if (tid == 0) gam = tr / (n * cc2);
      rhs_column_sums(E, b, colsum, red);
    }
    __syncthreads();

    // ---------------------------------------------------------- fill tiles
    if (FUSED) {
      const double g = gam;
      for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
          const int rr = tid >> 4, cl = tid & 15;   // tid < 256 covers the tile
          const int p = 16 * I + rr, q = 16 * J + cl;
          double v = (p < n && q < n) ? g * c[p] * c[q] : (p == q ? 1.0 : 0.0);
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
        const int a = tid >> 4, cl = tid & 15, p = 16 * J + cl;
        double v = 0.0;
        if (a < r && p < n) {
          int i, j;
          node_ij(p, s, i, j);
          v = btilde_entry(E, b, colsum, a, i, j, c[p]);
        }
        tr_(J)[a * TST + cl] = (T)v;
      }
    } else {
      const double* A = args.Ahat + E.mat0;
      for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
          const int rr = tid & 15, cl = tid >> 4;
          const int p = 16 * I + rr, q = 16 * J + cl;
          const double v = (p < n && q < n) ? A[(int64_t)q * n + p] : (p == q ? 1.0 : 0.0);
          tl(I, J)[rr * TST + cl] = (T)v;
        }
      const double* Bt = args.Btil + E.rhs0;
      for (int J = 0; J < nt; ++J) {
        const int a = tid >> 4, cl = tid & 15, p = 16 * J + cl;
        const double v = (a < r && p < n) ? Bt[(int64_t)a * n + p] : 0.0;
        tr_(J)[a * TST + cl] = (T)v;
      }
    }
    __syncthreads();

    // ------------------------------------------------------- factorisation
    T* Lo = nullptr;
    if (args.Lout && E.mat0 >= 0) Lo = reinterpret_cast<T*>(args.Lout + E.mat0);
    for (int k = 0; k < nt; ++k) {
      if (wave == 0) {
        typename Mfma<T>::v4 lv, wv;
        const int bj = potrf_inv_tile<T>(tl(k, k), lv, wv, lane);
        if (Lo) store_L<T>(Lo, n, k, k, lv, lane);
        st_acc<T>(tl(k, k), wv, lane);
        if (lane == 0 && bj >= 0 && bad < 0) bad = 16 * k + bj;
      }
      __syncthreads();
      // panel: L_ik = A_ik W_kk^T
      for (int i = k + 1 + wave; i < nt; i += NWAVES) {
        typename Mfma<T>::v4 acc = {0, 0, 0, 0};
        mma_add_nt<T>(acc, tl(i, k), tl(k, k), lane);
        st_acc<T>(tl(i, k), acc, lane);
        if (Lo) store_L<T>(Lo, n, i, k, acc, lane);
      }
      __syncthreads();
      // trailing update: C_ij -= L_ik L_jk^T, k < j <= i
      const int m = nt - 1 - k;
      const int ntr = m * (m + 1) / 2;
      for (int t = wave; t < ntr; t += NWAVES) {
        // t -> (i, j) over the trailing lower triangle, column by column
        int jj = 0, rem = t;
        while (rem >= m - jj) { rem -= m - jj; ++jj; }
        const int j = k + 1 + jj, i = j + rem;
        typename Mfma<T>::v4 acc = ld_acc<T>(tl(i, j), lane);
        mma_sub_nt<T>(acc, tl(i, k), tl(j, k), lane);
        st_acc<T>(tl(i, j), acc, lane);
      }
      __syncthreads();
    }

    // ---------------------------------------------- solves on the RHS row
    // Stored RHS tile J holds Z_J^T (rows: right-hand sides, cols: nodes).
    auto solve_rhs = [&]() {
      for (int j = 0; j < nt; ++j) {       // forward: Y = L^{-1} Z
        if (wave == (j & (NWAVES - 1))) {
          typename Mfma<T>::v4 acc = {0, 0, 0, 0};
          mma_add_nt<T>(acc, tr_(j), tl(j, j), lane);   // Y_j^T = Z_j^T W_j^T
          st_acc<T>(tr_(j), acc, lane);
        }
        __syncthreads();
        for (int i = j + 1 + wave; i < nt; i += NWAVES) {
          typename Mfma<T>::v4 acc = ld_acc<T>(tr_(i), lane);
          mma_sub_nt<T>(acc, tr_(j), tl(i, j), lane);  // Z_i^T -= Y_j^T L_ij^T
          st_acc<T>(tr_(i), acc, lane);
        }
        __syncthreads();
      }
      for (int j = nt - 1; j >= 0; --j) {  // backward: X = L^{-T} Y
        if (wave == (j & (NWAVES - 1))) {
          typename Mfma<T>::v4 acc = {0, 0, 0, 0};
          mma_add_nn<T>(acc, tr_(j), tl(j, j), lane);   // X_j^T = Z_j^T W_j
          st_acc<T>(tr_(j), acc, lane);
        }
        __syncthreads();
        for (int i = wave; i < j; i += NWAVES) {
          typename Mfma<T>::v4 acc = ld_acc<T>(tr_(i), lane);
          mma_sub_nn<T>(acc, tr_(j), tl(j, i), lane);  // Z_i^T -= X_j^T L_ji
          st_acc<T>(tr_(i), acc, lane);
        }
        __syncthreads();
      }
    };
    solve_rhs();

    double* X = args.X + E.rhs0;
    const bool failed = bad >= 0;
    if (!failed) {
      // X (FP64) from the solved tiles
      for (int idx = tid; idx < n * r; idx += NTHREADS) {
        const int a = idx / n, p = idx - a * n;
        X[idx] = (double)tr_(p >> 4)[a * TST + (p & 15)];
      }
      __syncthreads();
    }

    // --------------------------------------- FP64 refinement (FP32 path)
    if (fp32 && !failed) {
      const double* Btg = FUSED ? nullptr : args.Btil + E.rhs0;
      double g = gam;
      if (!FUSED) {
        // gamma = trace(A) / (n c^T c), the same reduction order as k_assemble
        double t = 0.0;
        for (int p = tid; p < n; p += NTHREADS) {
          int i, j;
          node_ij(p, s, i, j);
          t += stencil(i, j, s, E.G, kap).d;
        }
        t = block_sum(t, red);
        g = t / (n * cc2);
      }
      int it = 0;
      for (;; ++it) {
        // c^T X per column
        for (int a = 0; a < r; ++a) {
          double v = 0.0;
          for (int p = tid; p < n; p += NTHREADS) v += c[p] * X[(int64_t)a * n + p];
          v = block_sum(v, red);
          if (tid == 0) cx[a] = v;
        }
        __syncthreads();
        // residual R = Btilde - (A X + gamma c (c^T X)), into the RHS tiles (FP32)
        double rmax[16], xmax[16], bmax[16];
        double anorm = 0.0;
#pragma unroll
        for (int a = 0; a < 16; ++a) rmax[a] = xmax[a] = bmax[a] = 0.0;
        for (int p = tid; p < 16 * nt; p += NTHREADS) {
          if (p >= n) {
            for (int a = 0; a < 16; ++a) tr_(p >> 4)[a * TST + (p & 15)] = T(0);
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
              const double bv = FUSED ? btilde_entry(E, b, colsum, a, i, j, cp) : Btg[(int64_t)a * n + p];
              rv = bv - ax;
              rmax[a] = fmax(rmax[a], fabs(rv));
              xmax[a] = fmax(xmax[a], fabs(xa[p]));
              bmax[a] = fmax(bmax[a], fabs(bv));
            }
            tr_(p >> 4)[a * TST + (p & 15)] = (T)rv;
          }
        }
        // per-column maxima across the block
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
        solve_rhs();
        for (int idx = tid; idx < n * r; idx += NTHREADS) {
          const int a = idx / n, p = idx - a * n;
          X[idx] += (double)tr_(p >> 4)[a * TST + (p & 15)];
        }
        __syncthreads();
      }
      if (tid == 0) {
        if (args.ir_iters) args.ir_iters[e] = it;
        if (!conv) args.info[e] = INFO_IR_FALLBACK;
      }
      __syncthreads();
      if (!conv) continue;   // recomputed by the FP64 fallback pass
    }
    if (fp32 && failed) {
      if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
      __syncthreads();
      continue;
    }
    if (failed) {
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
      __syncthreads();
      continue;
    }

    // ------------------------------------------- zero-mean projection (FP64)
    for (int a = 0; a < r; ++a) {
      double v = 0.0;
      for (int p = tid; p < n; p += NTHREADS) v += c[p] * X[(int64_t)a * n + p];
      v = block_sum(v, red);
      if (tid == 0) cx[a] = v / E.area;
    }
    __syncthreads();
    for (int idx = tid; idx < n * r; idx += NTHREADS) {
      const int a = idx / n;
      X[idx] -= cx[a];
    }
    __syncthreads();

    if (FUSED && args.M) contrib_element(E, b, X, NImax, args.M, args.E, args.B, args.F, e, red);
    __syncthreads();
  }
}

// ------------------------------------------------------------- host launchers
static BatchDev to_dev(const mhm_batch* p) {
  BatchDev d;
  d.n_elem = p->n_elem;
  d.s_max = p->s_max;
  d.l_max = p->l_max;
  d.s = p->s;
  d.l = p->l;
  d.vert = p->vert;
  d.sigma = p->sigma;
  d.flip = p->flip;
  d.kappa = p->kappa;
  d.f = p->f;
  d.tri_off = p->tri_off;
  d.mat_off = p->mat_off;
  d.rhs_off = p->rhs_off;
  d.node_off = p->node_off;
  d.tri_total = p->tri_total;
  d.mat_total = p->mat_total;
  d.rhs_total = p->rhs_total;
  d.node_total = p->node_total;
  return d;
}

hipError_t launch_assemble(const mhm_batch* bt, double* Ahat, double* Btil, double* c, double* area, int32_t* info,
                           int grid, hipStream_t st) {
  const int smax = bt->s_max;
  const int nmax = (smax + 1) * (smax + 2) / 2;
  const size_t lds = sizeof(double) * ((size_t)smax * smax + nmax);
  hipError_t err = hipFuncSetAttribute((const void*)k_assemble, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_assemble, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), Ahat, Btil, c, area, info);
  return hipGetLastError();
}

hipError_t launch_contrib(const mhm_batch* bt, const double* X, double* M, double* E, double* B, double* F,
                          const int32_t* info, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_contrib, dim3(grid), dim3(NTHREADS), 0, st, to_dev(bt), X, M, E, B, F, info);
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

size_t local_lds_bytes(bool fp32, bool in_lds, bool fused, int n_cap, int k_cap, int tile_cap) {
  size_t bytes = sizeof(double) * ((size_t)n_cap + (size_t)k_cap);
  if (in_lds) bytes += (size_t)tile_cap * TILE * (fp32 ? sizeof(float) : sizeof(double));
  (void)fused;
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
