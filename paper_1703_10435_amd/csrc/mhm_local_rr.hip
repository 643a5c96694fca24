// Register-resident FP64 local-problem kernel (gfx950), for elements with
// n <= 16*RR_NT nodes.
//
// Same steps and results as k_local<double, ...> (a2-a6), organised so that
// two or three elements fit on one CU at a time (built for either, with 256
// or 168 registers per lane):
//  * the 16x16 tiles of the lower triangle of Ahat live in the MFMA
//    accumulators of the four waves (tile number t of the column-major
//    triangle is owned by wave t%4, slot t/4); the right-hand-side row
//    (transposed, one tile per 16 nodes) stays in LDS and is eliminated
//    with the matrix;
//  * a trailing update C_ij -= L_ik L_jk^T reads its two operands from the
//    published panel column in LDS and accumulates in registers;
//  * for f64 the MFMA result layout (lane l holds rows (l/16)+4v of column
//    l%16) coincides with the B-operand layout (chunk v: rows 4v+(l/16)), so
//    an L tile held in registers feeds the backward solve directly;
//  * LDS holds the current panel column, the inverses W_j of the diagonal
//    tiles, the right-hand-side row and the per-element tables (about 72 KB
//    at n = 153).  Built for three workgroups per CU, the diagonal tile's
//    register slot keeps W_j once that tile is factored (its own value is
//    dead from then on) for the backward solve, LDS keeps only the current
//    W_k, and the kappa and stencil tables share the panel column's space
//    (dead once the tiles are filled): about 50 KB.
#include "mhm_device.h"
#include "mhm_kernels.h"

namespace mhm {

namespace rr {

constexpr int NTHREADS = 256;
constexpr int NWAVES = 4;
constexpr int NT = 10;                              // tiles per matrix edge (n <= 160)
constexpr int NTILES = NT * (NT + 1) / 2;           // lower triangle
constexpr int S = (NTILES + NWAVES - 1) / NWAVES;   // register slots per wave
typedef Mfma<double>::v4 V4;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
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
// Value of lane `src` of this lane's 16-lane row (DPP row_newbcast; `src`
// must fold to a constant).
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
__device__ __forceinline__ double bcast16(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = row_bcast_i((int)b, src);
  const int hi = row_bcast_i((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

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

// Cholesky factor and inverse of one 16x16 tile stored (lower triangle) at
// `t`, by one wave.  Lanes are split 4 x 16: lane (c, g) = c + 16 g holds
// rows g + 4v (v = 0..3) of column c, the MFMA result layout; the pivot
// column is broadcast inside each 16-lane row and the pivot row across rows.
// Writes W = L^{-1} back to `t` (full tile, zero above the diagonal) and the
// lower triangle of L to Lo (column-major n x n, may be null).
__device__ __forceinline__ int potrf_inv(double* t, double* Lo, int n, int k, int lane) {
  const int c = lane & 15, g = lane >> 4;
  double a[4], w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = g + 4 * v;
    a[v] = r >= c ? t[r * TST + c] : t[c * TST + r];
    w[v] = r == c ? 1.0 : 0.0;
  }
  int bad = -1;
  double myrs = 1.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gj = j & 3, vj = j >> 2;          // lane group / item holding row j
    // row j of the current matrix, seen from column c: a[j][c] (lane (c, gj), item vj)
    const double ajc = __shfl(a[vj], c + 16 * gj, 64);
    // V row j (before scaling): lane (c, gj), item vj
    const double wv = __shfl(w[vj], c + 16 * gj, 64);
    double ajj = readlane_d(a[vj], j + 16 * gj);   // pivot a[j][j]
    if (!(ajj > 0.0)) {
      if (bad < 0) bad = j;
      ajj = 1.0;
    }
    const double rs = rsqrt_nr(ajj);
    if (c == j) myrs = rs;
    const double wjc = wv * rs;                    // W[j][c]
    const double f = ajc * (rs * rs);
    const bool cgt = c > j;
    // items whose four rows are all above row j are final: skipped (a
    // static test, so the step shrinks as j grows); the rest by selects
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (4 * v + 3 < j) continue;
      const int r = g + 4 * v;
      const double arj = bcast16(a[v], j);      // a[r][j]
      const double wu = w[v] - arj * rs * wjc;
      const double au = a[v] - arj * f;
      w[v] = r > j ? wu : (r == j ? wjc : w[v]);
      a[v] = (r > j && cgt) ? au : a[v];
    }
  }
  // column c of L is a[.][c] * myrs for rows >= c (entries above stay as read)
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
  return bad;
}


__device__ __forceinline__ void store_L(double* Lo, int n, int I, int J, const V4& acc, int lane) {
  const int q = 16 * J + (lane & 15);
  if (q >= n) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int p = 16 * I + Mfma<double>::row(lane >> 4, v);
    if (p < n && p >= q) Lo[(int64_t)q * n + p] = acc[v];
  }
}

}  // namespace rr

// OCC: resident workgroups per CU the registers are budgeted for (2: 256
// per lane, no spills; 3: 168, with spills in the factorisation loop).
template <bool FUSED, int OCC>
__global__ void __launch_bounds__(rr::NTHREADS, OCC) k_local_rr(BatchDev b, LocalArgs args) {
  using namespace rr;
  __shared__ Elem E;
  __shared__ int ok, bad;
  __shared__ double red[3 * NWAVES];
  __shared__ double colsum[R_CHUNK];   // one chunk only (r <= 16): two workgroups per CU need every byte
  __shared__ double cx[16];
  __shared__ double gam;
  extern __shared__ double dyn[];      // c | bf | ft | P[NT] (kap | stencil[8][n] until the fill ends) | W | R[NT]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NImax = nimax(b);

  double* c = dyn;
  double* bf = c + args.n_cap;
  double* ft = bf + args.n_cap;
  // Three workgroups per CU (WREG): the inverse W_j of a factored diagonal
  // tile moves into that tile's register slot and LDS keeps only the current
  // one; kappa and the node tables share the panel column's space (they are
  // dead once the tiles are filled).  Two per CU: every W_j in LDS.
  constexpr bool WREG = OCC == 3;
  double *kapl, *stt, *P, *Wb, *Rb;    // node tables: entry k of node p at k n_cap + p (fused), the
                                       // stencil d e w n s nw se, then 256 j + i
  if constexpr (WREG) {
    P = ft + args.f_cap;
    kapl = P;
    stt = kapl + args.k_cap;
    const int p_len = NT * TILE > args.k_cap + 8 * args.n_cap ? NT * TILE : args.k_cap + 8 * args.n_cap;
    Wb = P + p_len;
    Rb = Wb + TILE;
  } else {
    kapl = ft + args.f_cap;
    stt = kapl + args.k_cap;
    P = stt + 8 * args.n_cap;
    Wb = P + NT * TILE;
    Rb = Wb + NT * TILE;
  }
  auto Pt = [&](int I) -> double* { return P + I * TILE; };          // panel column L_ik
  auto Wt = [&](int J) -> double* { return WREG ? Wb : Wb + J * TILE; };  // diagonal inverses
  auto Rt = [&](int J) -> double* { return Rb + J * TILE; };         // RHS row: tile J holds Z_J^T

  V4 acc[S];

  const int n_launch = launch_count(args, b.n_elem);
  for (int k_el = blockIdx.x; k_el < n_launch; k_el += gridDim.x) {
    const int e = launch_elem(args, k_el);
    __syncthreads();
    if (tid == 0) {
      int st = INFO_OK;
      const bool good = load_elem(b, e, E) && E.rhs0 >= 0 && (FUSED || E.mat0 >= 0);
      if (!good) st = INFO_BAD_DESC;
      else if (E.nt > NT || E.n > args.n_cap || E.r > R_CHUNK || (FUSED && (E.NI * (E.s + 1) > args.f_cap || E.s * E.s > args.k_cap)))
        st = INFO_TOO_LARGE;
      ok = st == INFO_OK;
      args.info[e] = st;
      if (args.ir_iters) args.ir_iters[e] = 0;
      bad = -1;
    }
    __syncthreads();
    if (!ok) continue;
    const int s = E.s, n = E.n, r = E.r, nt = E.nt, T2 = s * s;
    const int ntiles = nt * (nt + 1) / 2;
    // Tile coordinates of this wave's slots (tile 4 sl + wave of the
    // column-major lower triangle, whose column J starts at tile
    // J nt - J (J - 1) / 2; -1 past its end), wave-uniform registers: the
    // slot tests of every step need no table reads.
    int sI[S], sJ[S];
    {
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      const float b2 = 2.0f * nt + 1.0f;
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        const int t = NWAVES * sl + wv;
        int J = (int)((b2 - sqrtf(b2 * b2 - 8.0f * t)) * 0.5f);
        J = J < 0 ? 0 : (J > nt - 1 ? nt - 1 : J);
        while (J > 0 && J * nt - (J * (J - 1)) / 2 > t) --J;
        while (J < nt - 1 && (J + 1) * nt - ((J + 1) * J) / 2 <= t) ++J;
        const bool in = t < ntiles;
        sI[sl] = in ? J + t - (J * nt - (J * (J - 1)) / 2) : -1;
        sJ[sl] = in ? J : -1;
      }
    }
    const double* kapg = b.kappa + E.tri0;
    auto kap = [&](int t) -> double { return FUSED ? kapl[t] : kapg[t]; };

    // ------------------------------------------------------------- set-up
    if (FUSED) {
      for (int t = tid; t < T2; t += NTHREADS) kapl[t] = kapg[t];
      const int sp1 = s + 1;
      for (int idx = tid; idx < E.NI * sp1; idx += NTHREADS) {
        const int a = idx / sp1, k = idx - a * sp1;
        ft[idx] = face_load(E, a, k);
      }
    }
    __syncthreads();
    // An element whose plain FP64 solve would not be accurate enough is left
    // to the FP64 pass that follows this kernel (a kernel with the refinement
    // step); info -1 marks it for that pass.  Fused launches only: the
    // three-call form keeps the plain FP64 solve on these elements (the
    // deferral from it was switched off after a GPU memory fault whose cause
    // was not found).
    if (FUSED && refine64_needed(args.refine64, kapl, s, red)) {
      if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
      continue;
    }
    {
      double tr = 0.0, cc2 = 0.0, fs = 0.0;
      const double* fp = b.f + E.tri0;
      for (int p = tid; p < n; p += NTHREADS) {
        int i, j;
        node_ij(p, s, i, j);
        const double cp = node_tri_count(i, j, s) * E.cunit;
        c[p] = cp;
        cc2 += cp * cp;
        if (FUSED) {
          const Stencil st = stencil(i, j, s, E.G, kap);
          const int NC = args.n_cap;
          double* sp = stt + p;
          sp[0] = st.d; sp[NC] = st.e; sp[2 * NC] = st.w; sp[3 * NC] = st.n;
          sp[4 * NC] = st.so; sp[5 * NC] = st.nw; sp[6 * NC] = st.se; sp[7 * NC] = (double)(256 * j + i);
          tr += st.d;
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
      if (FUSED && tid < E.NI) {
        double v = 0.0;
        for (int k = 0; k <= s; ++k) v += ft[tid * (s + 1) + k];
        colsum[tid] = v;
      }
    }
    __syncthreads();

    // ------------------------------------------------------------ fill
    // Register tiles: lane l of the owner holds rows 16I + (l/16) + 4v of
    // column 16J + l%16.  RHS row in LDS: R_J[a][l] = Btilde[16J + l][a].
    {
      const double g = gam;
      const int cl = lane & 15, grp = lane >> 4;
      const double* A = FUSED ? nullptr : args.Ahat + E.mat0;
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        V4 v4 = {0, 0, 0, 0};
        if (sI[sl] >= 0) {
          const int I = sI[sl], J = sJ[sl];
          const int q = 16 * J + cl;
          if (FUSED) {
            // stencil couplings reach |p - q| <= s + 2: only tiles near the diagonal
            const bool band = 16 * (I - J) <= s + 17;
            double sd = 0, se_ = 0, sw = 0, sn = 0, ss = 0, snw = 0, sse = 0;
            int qj = 0;
            if (band && q < n) {
              const int NC = args.n_cap;
              const double* sp = stt + q;
              sd = sp[0]; se_ = sp[NC]; sw = sp[2 * NC]; sn = sp[3 * NC]; ss = sp[4 * NC]; snw = sp[5 * NC];
              sse = sp[6 * NC];
              qj = (int)sp[7 * NC] >> 8;
            }
            const int pE = q + 1, pW = q - 1, pN = q + (s + 1 - qj), pS = q - (s + 2 - qj), pNW = q + (s - qj),
                      pSE = q - (s + 1 - qj);
            const double gcq = q < n ? g * c[q] : 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int p = 16 * I + grp + 4 * v;
              double x;
              if (p < n && q < n) {
                x = gcq * c[p];
                if (band) {
                  x += (p == q) ? sd : 0.0;
                  x += (p == pE) ? se_ : 0.0;
                  x += (p == pW) ? sw : 0.0;
                  x += (p == pN) ? sn : 0.0;
                  x += (p == pS) ? ss : 0.0;
                  x += (p == pNW) ? snw : 0.0;
                  x += (p == pSE) ? sse : 0.0;
                }
              } else {
                x = (p == q) ? 1.0 : 0.0;
              }
              v4[v] = x;
            }
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int p = 16 * I + grp + 4 * v;
              v4[v] = (p < n && q < n) ? A[(int64_t)q * n + p] : (p == q ? 1.0 : 0.0);
            }
          }
        }
        acc[sl] = v4;
      }
      // right-hand-side row
      const double* Bt = FUSED ? nullptr : args.Btil + E.rhs0;
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        if (J >= nt) break;
        const int a = tid >> 4, cq = tid & 15, q = 16 * J + cq;
        double x = 0.0;
        if (a < r && q < n) {
          if (FUSED) {
            const int code = (int)stt[7 * args.n_cap + q];
            const int qi = code & 255, qj = code >> 8;
            double base = 0.0;
            if (a < E.NI) {
              const int ef = a / E.P;
              const int kk = face_pos(ef, qi, qj, s);
              if (kk >= 0) base = ft[a * (s + 1) + kk];
            } else {
              base = bf[q];
            }
            x = base - c[q] * colsum[a] * E.inv_area;
          } else {
            x = Bt[(int64_t)a * n + q];
          }
        }
        Rt(J)[a * TST + cq] = x;
      }
    }
    double* Lo = (!FUSED && args.Lout && E.mat0 >= 0) ? args.Lout + E.mat0 : nullptr;
    __syncthreads();

    // ------------------------------------------------------- factorisation
    // Step k = -1 only hands tile (0, 0) to the factor.  The RHS row is
    // eliminated with the matrix and ends holding Y^T = (L^{-1} Btilde)^T.
    for (int k = -1; k < nt; ++k) {
      if (k >= 0) {
        // panel: L_ik = A_ik W_k^T by the owners of tiles (i, k), i > k,
        // published to P[i]; Y_k^T = Z_k^T W_k^T by wave k%4
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
          if (sJ[sl] == k && sI[sl] > k) {
            const int I = sI[sl];
            st_acc<double>(Pt(I), acc[sl], lane);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            V4 x = {0, 0, 0, 0};
#pragma unroll
            for (int cch = 0; cch < 4; ++cch)
              x = Mfma<double>::op(ld_rowcol(Pt(I), cch, lane), ld_rowcol(Wt(k), cch, lane), x);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            acc[sl] = x;
            st_acc<double>(Pt(I), x, lane);
            if (!FUSED && Lo) rr::store_L(Lo, n, I, k, x, lane);
          }
        }
        if (wave == (k & 3)) {
          V4 x = {0, 0, 0, 0};
#pragma unroll
          for (int cch = 0; cch < 4; ++cch)
            x = Mfma<double>::op(ld_rowcol(Rt(k), cch, lane), ld_rowcol(Wt(k), cch, lane), x);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          st_acc<double>(Rt(k), x, lane);
        }
        __syncthreads();
      }
      // trailing update: C_ij -= L_ik L_jk^T for k < j <= i < nt.  The owner
      // of tile (k+1, k+1) updates it first, hands it to the W buffer and
      // factors it; then every wave updates its other tiles, two at a time
      // (the tiles of a step are a suffix of each wave's slots).
      bool mine = false;
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        if (sI[sl] == k + 1 && sJ[sl] == k + 1) {
          V4 x = acc[sl];
          if (k >= 0) {
#pragma unroll
            for (int cch = 0; cch < 4; ++cch)
              x = Mfma<double>::op(-ld_rowcol(Pt(k + 1), cch, lane), ld_rowcol(Pt(k + 1), cch, lane), x);
            acc[sl] = x;
          }
          st_acc<double>(Wt(k + 1), x, lane);
          mine = true;
        }
      }
      if (mine) {
        // the diagonal factorisation is the critical path of the step: the
        // wave runs it at raised issue priority over the other workgroup's
        // waves on its SIMD
        __builtin_amdgcn_s_setprio(3);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int bj = rr::potrf_inv(Wt(k + 1), Lo, n, k + 1, lane);
        if (lane == 0 && bj >= 0 && bad < 0) bad = 16 * (k + 1) + bj;
        __builtin_amdgcn_s_setprio(0);
        if constexpr (WREG) {
          // the tile's own register slot is free from here on: it keeps
          // W_k+1 for the backward solve (the result layout is its B-operand
          // layout)
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
          for (int sl = 0; sl < S; ++sl)
            if (sI[sl] == k + 1 && sJ[sl] == k + 1) acc[sl] = ld_acc<double>(Wt(k + 1), lane);
        }
      }
      if (k >= 0) {
#pragma unroll
        for (int sl = 0; sl < S; sl += 2) {
          const int I0 = sI[sl], J0 = sJ[sl];
          const int I1 = sl + 1 < S ? sI[sl + 1] : -1, J1 = sl + 1 < S ? sJ[sl + 1] : -1;
          const bool a0 = J0 > k && !(I0 == k + 1 && J0 == k + 1);
          const bool a1 = J1 > k && !(I1 == k + 1 && J1 == k + 1);
          if (a0 || a1) {
            const int i0 = a0 ? I0 : I1, j0 = a0 ? J0 : J1;
            const int i1 = a1 ? I1 : i0, j1 = a1 ? J1 : j0;
            V4 x0 = acc[sl];
            V4 x1 = sl + 1 < S ? acc[sl + 1] : acc[sl];
#pragma unroll
            for (int cch = 0; cch < 4; ++cch) {
              x0 = Mfma<double>::op(-ld_rowcol(Pt(i0), cch, lane), ld_rowcol(Pt(j0), cch, lane), x0);
              x1 = Mfma<double>::op(-ld_rowcol(Pt(i1), cch, lane), ld_rowcol(Pt(j1), cch, lane), x1);
            }
            if (a0) acc[sl] = x0;
            if (sl + 1 < S && a1) acc[sl + 1] = x1;
          }
        }
      }
      // RHS row: Z_j^T -= Y_k^T L_jk^T, j > k
      if (k >= 0)
        for (int j = k + 1 + wave; j < nt; j += NWAVES) {
          V4 z = ld_acc<double>(Rt(j), lane);
#pragma unroll
          for (int cch = 0; cch < 4; ++cch)
            z = Mfma<double>::op(-ld_rowcol(Rt(k), cch, lane), ld_rowcol(Pt(j), cch, lane), z);
          st_acc<double>(Rt(j), z, lane);
        }
      __syncthreads();
    }

    // --------------------------------------------- backward solve X = L^{-T} Y
    for (int j = nt - 1; j >= 0; --j) {
      // X_j^T = Z_j^T W_j: by the owner of tile (j, j), which holds W_j, or
      // with W_j from LDS
      if constexpr (WREG) {
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
          if (sI[sl] == j && sJ[sl] == j) {
            V4 x = {0, 0, 0, 0};
#pragma unroll
            for (int cch = 0; cch < 4; ++cch) x = Mfma<double>::op(ld_rowcol(Rt(j), cch, lane), acc[sl][cch], x);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            st_acc<double>(Rt(j), x, lane);
          }
        }
      } else if (wave == (j & 3)) {
        V4 x = {0, 0, 0, 0};
#pragma unroll
        for (int cch = 0; cch < 4; ++cch)
          x = Mfma<double>::op(ld_rowcol(Rt(j), cch, lane), ld_colrow(Wt(j), cch, lane), x);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        st_acc<double>(Rt(j), x, lane);
      }
      __syncthreads();
      // Z_i^T -= X_j^T L_ji (i < j) by the owner of tile (j, i): its registers
      // are the B operand
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        if (sI[sl] == j && sJ[sl] >= 0 && sJ[sl] < j) {
          const int I = sJ[sl];
          V4 z = ld_acc<double>(Rt(I), lane);
#pragma unroll
          for (int cch = 0; cch < 4; ++cch) z = Mfma<double>::op(-ld_rowcol(Rt(j), cch, lane), acc[sl][cch], z);
          st_acc<double>(Rt(I), z, lane);
        }
      }
      __syncthreads();
    }

    double* X = args.X + E.rhs0;
    if (bad >= 0) {
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
    }
    // zero-mean projection (FP64) and output
    {
      const int ca = tid >> 4, cl16 = tid & 15;
      double v = 0.0;
      if (ca < r)
        for (int p = cl16; p < n; p += 16) v += c[p] * Rt(p >> 4)[ca * TST + (p & 15)];
      v = group16_sum(v);
      if (cl16 == 0) cx[ca] = v * E.inv_area;
    }
    __syncthreads();
    for (int idx = tid; idx < n * r; idx += NTHREADS) {
      const int a = idx / n, p = idx - a * n;
      X[idx] = Rt(p >> 4)[a * TST + (p & 15)] - cx[a];
    }
    __syncthreads();
    if (FUSED && args.M) {
      // contribution blocks of eq. (6): M = -R^T X_I, E = R^T x_f, B, F
      const int NI = E.NI, sp1 = s + 1;
      double* Me = args.M + (int64_t)e * NImax * NImax;
      for (int idx = tid; idx < NImax * NImax; idx += NTHREADS) {
        const int a = idx % NImax, bb = idx / NImax;
        if (a >= NI || bb >= NI) Me[idx] = 0.0;
      }
      if (tid < NI * r) {
        const int a = tid % NI, bb = tid / NI;
        const int ef = a / E.P;
        const double* fa = ft + a * sp1;
        const double* xb = X + (int64_t)bb * n;
        double v = 0.0;
        for (int k = 0; k < sp1; ++k) v += fa[k] * xb[face_node(ef, k, s)];
        if (bb < NI) Me[(int64_t)bb * NImax + a] = -v;
        else args.E[(int64_t)e * NImax + a] = v;
      } else if (tid >= 240 && tid < 240 + NImax) {
        const int a = tid - 240;
        double v = 0.0;
        if (a < NI) {
          for (int k = 0; k < sp1; ++k) v -= ft[a * sp1 + k];
        } else {
          args.E[(int64_t)e * NImax + a] = 0.0;
        }
        args.B[(int64_t)e * NImax + a] = v;
      }
      if (tid == 255) args.F[e] = colsum[E.NI];
    }
  }
}

// ------------------------------------------------------------------ launch
size_t local_rr_lds_bytes(int n_cap, int f_cap, int k_cap, int occ) {
  if (occ != 3)
    return sizeof(double) * (10 * (size_t)n_cap + (size_t)f_cap + (size_t)k_cap + (size_t)(3 * rr::NT) * TILE);
  const size_t p_len = std::max((size_t)rr::NT * TILE, (size_t)k_cap + 8 * (size_t)n_cap);
  return sizeof(double) * (2 * (size_t)n_cap + (size_t)f_cap + p_len + TILE + (size_t)rr::NT * TILE);
}
int local_rr_max_nt() { return rr::NT; }

template <bool FUSED, int OCC>
static hipError_t launch_rr_t(const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  auto kern = k_local_rr<FUSED, OCC>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(rr::NTHREADS), lds, st, d, a);
  return hipGetLastError();
}

hipError_t launch_local_rr(bool fused, int occ, const mhm_batch* bt, LocalArgs a, size_t lds, int grid,
                           hipStream_t st) {
  if (occ != 2 && occ != 3) return hipErrorInvalidValue;
  const BatchDev d = to_dev(bt);
  if (fused) return occ == 3 ? launch_rr_t<true, 3>(d, a, lds, grid, st) : launch_rr_t<true, 2>(d, a, lds, grid, st);
  return occ == 3 ? launch_rr_t<false, 3>(d, a, lds, grid, st) : launch_rr_t<false, 2>(d, a, lds, grid, st);
}

}  // namespace mhm
