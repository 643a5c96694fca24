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
//   (b) every earlier tile column m is applied, C_ij -= L_im L_jm^T, each
//       wave streaming its A operands L_im and the panel's B tiles L_jm from
//       the workspace into registers, with no barrier between columns;
//   (c) the panel is factored in place (diagonal tile by one wave in LDS,
//       panel solve and in-panel updates in registers) and written once.
// Each tile of L is therefore written once and read once per later block
// column, about n^3/(6*16*PW) tile reads per element instead of the
// n^3/(3*16) read-modify-writes of a right-looking sweep.  Where a wave's
// rows of a wide panel would not fit in registers, (a)-(c) run over the
// rows in passes (the constant RS of the kernel).
#pragma once
#include "mhm_common.h"
#include "mhm_kernels.h"

namespace mhm {

namespace ll {

// Operand chunks of a stored tile for the earlier-column updates, with the
// contraction index of chunk c in lane group g taken as k = 4 g + c (the
// same for both operands, so the product is unchanged): the four values of
// a lane are adjacent in memory and come in one vector load (4-byte
// aligned; the tile rows are 17 wide).
template <typename T> struct Vec4U;
template <> struct Vec4U<float> { typedef float t __attribute__((ext_vector_type(4), aligned(4))); };
template <> struct Vec4U<double> { typedef double t __attribute__((ext_vector_type(4), aligned(8))); };
template <typename T>
__device__ __forceinline__ typename Mfma<T>::v4 ld_row4v(const T* t, int lane) {
  const typename Vec4U<T>::t v = *reinterpret_cast<const typename Vec4U<T>::t*>(t + (lane & 15) * TST + 4 * (lane >> 4));
  return typename Mfma<T>::v4{v[0], v[1], v[2], v[3]};
}
template <typename T>
__device__ __forceinline__ void ld_row4(const T* t, int lane, T (&o)[4]) {
  const typename Vec4U<T>::t v = *reinterpret_cast<const typename Vec4U<T>::t*>(t + (lane & 15) * TST + 4 * (lane >> 4));
  o[0] = v[0];
  o[1] = v[1];
  o[2] = v[2];
  o[3] = v[3];
}

// One block triangular sweep over the right-hand-side tile row of the factor
// (tiles tl(nt, i) hold Z_i^T, 16 right-hand sides by 16 nodes; the diagonal
// tiles tl(j, j) hold W_j = L_jj^{-1}):
//   backward (BACK):  X_j^T = Z_j^T W_j,    Z_i^T -= X_j^T L_ji     (i < j)
//   forward:          Y_j^T = Z_j^T W_j^T,  Z_i^T -= Y_j^T L_ij^T   (i > j)
// Wave w keeps tiles i = w + NW ri in registers.  In the step for block
// column j, after one barrier, every wave applies the published solution
// tile of column j to its own tiles; the owner of the next column solves that
// tile right after its last update and publishes it (LDS double buffer xb).
// The L operands of a step are loaded one or two steps ahead, so their
// global-memory latency overlaps the chain of column solves.  Every register
// slot is addressed statically.
template <typename T, int RPW, bool BACK, int OCC, int NW>
__device__ __forceinline__ void sweep_body(T* Lb, T* rhs_row, int nt, T* xb, T* scr, int wave, int lane) {
  typedef typename Mfma<T>::v4 V4;
  auto tl = [=](int I, int J) -> T* {
    return I == nt ? rhs_row + (int64_t)J * TILE : Lb + (int64_t)((I * (I + 1)) / 2 + J) * TILE;
  };
  // operand buffers (prefetch depth): FP32 sweeps run in their own function
  // with registers to spare; FP64 ones are inlined in the kernel
  // (two workgroups per CU or 16 waves: half the registers, one buffer)
  constexpr int NB = (OCC == 2 || NW == 16) ? 1 : sizeof(T) == 4 ? (RPW <= 5 ? 3 : 2) : (RPW <= 5 ? 2 : 1);
  V4 z[RPW];
#pragma unroll
  for (int ri = 0; ri < RPW; ++ri) {
    const int i = wave + NW * ri;
    if (i < nt) z[ri] = ld_acc<T>(tl(nt, i), lane);
    else z[ri] = V4{0, 0, 0, 0};
  }
  auto colj = [&](int st) { return BACK ? nt - 1 - st : st; };
  auto upd = [&](int i, int j) { return BACK ? i < j : (i > j && i < nt); };
  auto ld_w = [&](int j, T (&w)[4]) {
    const T* W = tl(j, j);
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = BACK ? ld_colrow(W, c, lane) : ld_rowcol(W, c, lane);
  };
  // operands of step st: L tiles applied to the own tiles, and W of the
  // column solved during that step (owner only)
  auto fetch = [&](int st, T (&b)[RPW][4], T (&w)[4]) {
    if (st >= nt) return;
    const int j = colj(st);
#pragma unroll
    for (int ri = 0; ri < RPW; ++ri) {
      const int i = wave + NW * ri;
      if (upd(i, j)) {
        // forward: rows of L_ij, one vector load per lane (contraction index
        // 4 (l / 16) + c, matched in the A operand below); backward: columns
        // of L_ji, element loads
        if (BACK) {
          const T* L = tl(j, i);
#pragma unroll
          for (int c = 0; c < 4; ++c) b[ri][c] = ld_colrow(L, c, lane);
        } else {
          ld_row4(tl(i, j), lane, b[ri]);
        }
      }
    }
    if (st + 1 < nt && wave == colj(st + 1) % NW) ld_w(colj(st + 1), w);
  };
  auto solve_tile = [&](V4& zr, const T (&w)[4], T* dst) {
    st_acc<T>(scr, zr, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    V4 x = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) x = Mfma<T>::op(ld_rowcol(scr, c, lane), w[c], x);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    zr = x;
    st_acc<T>(dst, x, lane);
  };
  T bo[NB][RPW][4];
  T wo[NB][4];
  {
    const int j = colj(0);
    T w0[4];
    if (wave == j % NW) ld_w(j, w0);
#pragma unroll
    for (int q = 0; q < NB; ++q) fetch(q, bo[q], wo[q]);
#pragma unroll
    for (int ri = 0; ri < RPW; ++ri)
      if (wave + NW * ri == j) solve_tile(z[ri], w0, xb);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
  auto step_once = [&](int st, const T (&b)[RPW][4], const T (&w)[4]) {
    const int j = colj(st);
    const int jn = st + 1 < nt ? colj(st + 1) : -1;
    const T* xj = xb + (st & 1) * TILE;
    T* xn = xb + ((st + 1) & 1) * TILE;
    T a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      a[c] = BACK ? -ld_rowcol(xj, c, lane) : -xj[(lane & 15) * TST + 4 * (lane >> 4) + c];
#pragma unroll
    for (int ri = 0; ri < RPW; ++ri) {
      const int i = wave + NW * ri;
      if (upd(i, j)) {
        V4 x = z[ri];
#pragma unroll
        for (int c = 0; c < 4; ++c) x = Mfma<T>::op(a[c], b[ri][c], x);
        z[ri] = x;
        if (i == jn) solve_tile(z[ri], w, xn);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  };
  for (int st = 0; st < nt; st += NB) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (st + q < nt) {
        step_once(st + q, bo[q], wo[q]);
        fetch(st + q + NB, bo[q], wo[q]);
      }
    }
  }
#pragma unroll
  for (int ri = 0; ri < RPW; ++ri) {
    const int i = wave + NW * ri;
    if (i < nt) st_acc<T>(tl(nt, i), z[ri], lane);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
}
// The same sweep as a separate function (the FP32 refinement loop calls it
// twice per step: inlined copies would add their registers to the kernel's).
template <typename T, int RPW, bool BACK, int OCC, int NW>
__device__ __noinline__ void sweep_call(T* Lb, T* rhs_row, int nt, T* xb, T* scr, int wave, int lane) {
  sweep_body<T, RPW, BACK, OCC, NW>(Lb, rhs_row, nt, xb, scr, wave, lane);
}
template <typename T, int RPW, bool BACK, int OCC, int NW>
__device__ __forceinline__ void sweep(T* Lb, T* rhs_row, int nt, T* xb, T* scr, int wave, int lane) {
  if constexpr (sizeof(T) == 4) sweep_call<T, RPW, BACK, OCC, NW>(Lb, rhs_row, nt, xb, scr, wave, lane);
  else sweep_body<T, RPW, BACK, OCC, NW>(Lb, rhs_row, nt, xb, scr, wave, lane);
}
}  // namespace ll

// OCC = 2: the register budget of two resident workgroups per CU (4 waves
// per SIMD, at most 128 registers per lane; two elements interleave their
// latencies), with one operand buffer.  NWV = 16: 16 waves per element
// (half the rows per wave, at most 128 registers per lane, twice the waves
// in flight).  MC: more than 16 right-hand sides, in chunks of 16 (built
// only where a batch has them, so the one-chunk instances keep their
// registers).  REF (FP64): the instance carries the FP64 refinement step;
// one without it leaves the elements that need the step to the FP64 pass
// that follows it (info -1), because the refinement code, although it runs
// only for those elements, costs the factorisation loop registers (FP64,
// s = 48, four-tile panels: 45 against 200 ms per 1024 elements).
template <typename T, bool FUSED, int PW, int RPW, int OCC, int NWV, bool MC, bool REF>
__global__ void __launch_bounds__(64 * NWV, (NWV / 4) * OCC) k_local_ll(BatchDev b, LocalArgs args) {
  typedef typename Mfma<T>::v4 V4;
  constexpr int NW = NWV;
  constexpr int NTHREADS = 64 * NW;
  // Row passes per block column: with ten rows per wave (8 waves), a panel
  // wider than 80 accumulator registers per lane (two FP32 or one FP64 tile
  // per row) would not fit next to the operands, so the rows are updated and
  // solved in passes of five or two; with 16 waves (128 registers) the limit
  // is 40, passes of one row.  The earlier columns' B tiles are loaded once
  // per pass, the A tiles (the bulk of the reads) still once per panel.
  constexpr int ACC = PW * 4 * (int)(sizeof(T) / 4);   // accumulator registers per row
  constexpr int RS = (MC || OCC != 1)            ? 1
                     : NW == 8 && RPW == 10       ? (10 * ACC <= 80 ? 1 : 5 * ACC <= 80 ? 2 : 5)
                     : NW == 16 && RPW == 5       ? (5 * ACC <= 40 ? 1 : 5)
                                                  : 1;
  constexpr int RH = RPW / RS;
  __shared__ Elem E;
  __shared__ int ok, bad, conv;
  __shared__ double be_prev;
  __shared__ double red[48];
  __shared__ double colsum[R_MAX];
  __shared__ double cx[16];
  __shared__ double gam;
  __shared__ double part_s[32 * (NTHREADS / 256)];
  __shared__ double rmax[16], xmax[16], bmax[16];
  extern __shared__ double dyn[];
  // the wave index is uniform: held in a scalar register, so the per-row
  // conditions below are scalar branches
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int NImax = nimax(b);
  const bool fp32 = sizeof(T) == 4;

  const int n_launch = launch_count(args, b.n_elem);
  for (int k_el = blockIdx.x; k_el < n_launch; k_el += gridDim.x) {
    const int e = launch_elem(args, k_el);
    __syncthreads();
    if (tid == 0) {
      int st = INFO_OK;
      if (args.only_fallback && args.info[e] != INFO_IR_FALLBACK) {
        ok = 0;
      } else {
        const bool good = load_elem(b, e, E) && E.rhs0 >= 0 && (FUSED || E.mat0 >= 0);
        const int nch_e = MC ? (E.r + R_CHUNK - 1) / R_CHUNK : 1;   // right-hand-side tile rows
        if (!good) st = INFO_BAD_DESC;
        else if ((args.fac ? nch_e * E.nt : (E.nt * (E.nt + 1)) / 2 + (nch_e + 1) * E.nt) > args.tile_cap ||
                 E.n > args.n_cap ||
                 (!MC && E.r > R_CHUNK) ||
                 E.nt + 1 > NW * RPW || (args.fac && args.fac_off[e] < 0) ||
                 (FUSED && E.NI * (E.s + 1) > args.f_cap))
          st = INFO_TOO_LARGE;
        ok = st == INFO_OK;
        // a pass over the elements an FP64 run deferred owns their info; the
        // FP64 pass of an FP32 run leaves -1 (and the FP32 step count) on them
        if (!ok || !args.only_fallback || args.fb_final) args.info[e] = st;
        if (args.ir_iters && (!args.only_fallback || args.fb_final)) args.ir_iters[e] = 0;
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
    T* stage = reinterpret_cast<T*>(ft + args.f_cap);  // 2 tiles
    T* Wt = stage + 2 * TILE;                            // the panel's PW diagonal inverses
    T* pub = Wt + PW * TILE;                             // PW x PW published panel tiles
    T* scr = pub + PW * PW * TILE + wave * TILE;         // this wave's scratch tile
    T* ws = reinterpret_cast<T*>(args.ws) + (int64_t)blockIdx.x * args.ws_slot;
    // Tiles of the factor (lower triangle, W_jj = L_jj^{-1} on the diagonal):
    // in the workgroup's workspace slot, or in the caller's factor store
    // (kept for later right-hand sides), with the right-hand-side row then
    // alone in the slot.
    T* Lb = args.fac ? reinterpret_cast<T*>(static_cast<char*>(args.fac) + args.fac_off[e]) : ws;
    T* rhs_row = args.fac ? ws : ws + (int64_t)((nt * (nt + 1)) / 2) * TILE;
    const bool reuse = args.fac && args.fac_state && args.fac_state[e] == 1;
    // Right-hand sides: one tile row of 16 columns per chunk.  The chunked
    // instances eliminate as many chunks as the waves have spare rows for
    // (tile rows nt .. nrows - 1 below the matrix) with the factorisation;
    // the others are swept on the finished factor one at a time.
    const int nch = MC ? (r + R_CHUNK - 1) / R_CHUNK : 1;
    const int nfused = MC && !reuse ? min(nch, NW * RPW - nt) : 1;
    const int nrows = nt + nfused;
    auto tl = [&](int I, int J) -> T* {
      if constexpr (MC) {
        if (I >= nt) return rhs_row + ((int64_t)(I - nt) * nt + J) * TILE;
      } else {
        if (I == nt) return rhs_row + (int64_t)J * TILE;
      }
      return Lb + (int64_t)((I * (I + 1)) / 2 + J) * TILE;
    };
    // row i of the panel loops: a right-hand-side row, or inside the rows held
    auto rhs_i = [&](int i) -> bool { return MC ? i >= nt : i == nt; };
    auto held_i = [&](int i) -> bool { return MC ? i < nrows : i <= nt; };
    // L_jj tiles (factor output only), after the right-hand-side rows
    auto ldiag = [&](int J) -> T* { return rhs_row + (int64_t)(nch * nt + J) * TILE; };
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
    // FP64: one refinement step with a double-double residual where a plain
    // FP64 solve is not accurate enough (the FP32 path always refines); an
    // instance without the step defers such an element
    const bool need64 = !fp32 && refine64_needed(args.refine64, kapg, s, red);
    if constexpr (!REF && sizeof(T) == 8) {
      if (need64) {
        if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
        continue;
      }
    }
    // FP32: an element whose contrast s^2 exceeds the same bound would take
    // many refinement steps (each one contracts the error by about the
    // element's condition number times the FP32 unit roundoff) or stall; in
    // the fused one-chunk form without a factor store it goes straight to the
    // FP64 pass that follows this launch (info -1, no refinement steps
    // counted), which factors it in FP64 with its refinement step.  (The
    // chunked instances keep the FP32 attempt: with the test their update
    // loop spills.)
    if constexpr (sizeof(T) == 4 && FUSED && !MC) {
      if (!args.fac && refine64_needed(args.refine64 < 0 ? -1 : 0, kapg, s, red)) {
        if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
        continue;
      }
    }
    const bool ref64 = REF && need64;
    // factor output: the three-call form, and the FP64 refinement pass over
    // the elements such a call deferred (that pass works from kappa)
    T* Lo = nullptr;
    if (args.Lout && E.mat0 >= 0) Lo = reinterpret_cast<T*>(args.Lout + E.mat0);

    // Tile (I, J) of the operator in the MFMA result layout: Ahat for I < nt,
    // the transposed right-hand sides Btilde^T for I >= nt (chunk I - nt).
    auto init_tile = [&](int I, int J) -> V4 {
      V4 v4;
      const int cl = lane & 15, grp = lane >> 4;
      const int q = 16 * J + cl;
      if (MC ? I >= nt : I == nt) {
        const int cb = MC ? R_CHUNK * (I - nt) : 0;   // the chunk's first column
        int qi = 0, qj = 0;
        if (FUSED && q < n) node_ij(q, s, qi, qj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = Mfma<T>::row(grp, v);
          double x = 0.0;
          const int col = cb + a;
          if (col < r && q < n) x = FUSED ? btilde_tab(E, ft, bf, c, colsum, col, q, qi, qj)
                                          : args.Btil[E.rhs0 + (int64_t)col * n + q];
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

    T* xb = stage;   // two published solution tiles of the sweeps (staging area)
    auto backward = [&](T* row) { ll::sweep<T, RPW, true, OCC, NW>(Lb, row, nt, xb, scr, wave, lane); };
    auto forward = [&](T* row) { ll::sweep<T, RPW, false, OCC, NW>(Lb, row, nt, xb, scr, wave, lane); };

    // ------------------------------------------------------ factorisation
    if (reuse) {
      // stored factor: only the new right-hand sides, Y = L^{-1} Btilde
      for (int J = wave; J < nt; J += NW) st_acc<T>(tl(nt, J), init_tile(nt, J), lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
      forward(rhs_row);
    }
    for (int j0 = 0; j0 < (reuse ? 0 : nt); j0 += PW) {
      const int pw = nt - j0 < PW ? nt - j0 : PW;
#pragma unroll 1
      for (int h = 0; h < RS; ++h) {
        // the rows of pass h start at j0 + NW RH h: past the last row no wave
        // holds any (nor in the later passes), so the pass and its sweep over
        // the earlier columns are skipped (the same for every wave)
        if (h > 0 && j0 + NW * RH * h >= (MC ? nrows : nt + 1)) break;
        // rows of this pass: slots h RH .. h RH + RH - 1 of the wave
        auto row_of = [&](int ri) { return j0 + wave + NW * (h * RH + ri); };
        V4 acc[RH][PW];
        // (a) the panel's accumulators start at zero: the earlier columns'
        // updates are summed first and the operator is added once, after (b).
        // Summed into the operator's entries instead, each of the n products
        // of a long dot product would be rounded at the size of the operator's
        // largest entries (high-contrast elements: K = 1e4 against pivots of
        // order one), which makes the factor an order of magnitude less
        // accurate.
#pragma unroll
        for (int ri = 0; ri < RH; ++ri) {
#pragma unroll
          for (int k = 0; k < PW; ++k) acc[ri][k] = V4{0, 0, 0, 0};
        }
        // (b) earlier tile columns, C_ij -= L_im L_jm^T for m < j0.  Each wave
        // loads its own operands for column m, the A tiles L_im of its rows
        // and the panel's B tiles L_jm (the same for every wave: they come
        // from the L1 / L2 after the first wave), straight into registers,
        // NB columns ahead.  There is no barrier in this loop (the tiles of
        // earlier panels were published by the barrier that ended each pass),
        // so the waves of a SIMD overlap one another's load latency, and a
        // wave without rows in this pass skips it.
        if (j0 > 0 && held_i(row_of(0))) {
          constexpr int W = (int)sizeof(T) / 4;
          // operand buffers (prefetch depth) within a register estimate:
          // accumulators plus NB stages of RH A rows and PW B tiles (256
          // registers per lane, or 128 with 16 waves or two workgroups per CU;
          // less where the row passes keep more state live across the loop,
          // which the compiler would otherwise spill inside it)
          constexpr int ACCR = RH * PW * 4 * W, STG = (RH + PW) * 4 * W;
          constexpr int BUD = (NW == 16 || OCC == 2) ? 88 : 150;
          constexpr int NB = ACCR + 3 * STG <= BUD ? 3 : ACCR + 2 * STG <= BUD ? 2 : 1;
          // (operands as 4-vectors: a row's values stay one register group)
          V4 ab[NB][RH];
          V4 bb[NB][PW];
          auto fetch = [&](int m, V4 (&a)[RH], V4 (&bt)[PW]) {
            if (m >= j0) return;
#pragma unroll
            for (int ri = 0; ri < RH; ++ri) {
              const int i = row_of(ri);
              if (held_i(i)) a[ri] = ll::ld_row4v(tl(i, m), lane);
            }
#pragma unroll
            for (int jj = 0; jj < PW; ++jj)
              if (jj < pw) bt[jj] = ll::ld_row4v(tl(j0 + jj, m), lane);
          };
          auto apply = [&](const V4 (&a)[RH], const V4 (&bt)[PW]) {
#pragma unroll
            for (int ri = 0; ri < RH; ++ri) {
              const int i = row_of(ri);
              if (held_i(i)) {
#pragma unroll
                for (int jj = 0; jj < PW; ++jj) {
                  if (jj < pw && (rhs_i(i) || i >= j0 + jj)) {
                    V4 x = acc[ri][jj];
#pragma unroll
                    for (int cch = 0; cch < 4; ++cch) x = Mfma<T>::op_sub(a[ri][cch], bt[jj][cch], x);
                    acc[ri][jj] = x;
                  }
                }
              }
            }
          };
          if constexpr (NB == 1) {
            // one operand set: row ri's A tile of column m + 1 is loaded
            // right after the MFMAs of column m that read it, so it has the
            // other rows' MFMAs to arrive; the B tiles are double-buffered.
            // Every load is unconditional (a row or tile outside the pass,
            // and the step past the last column, load a valid tile again),
            // so the waits count the loads exactly.
            V4 (&a)[RH] = ab[0];
            V4 bq0[PW], bq1[PW];
            const int r0 = row_of(0);
            auto ld_a = [&](int ri, int m) {
              const int i = row_of(ri);
              return ll::ld_row4v(tl(held_i(i) ? i : r0, m), lane);
            };
            auto ld_b = [&](int jj, int m) { return ll::ld_row4v(tl(j0 + (jj < pw ? jj : 0), m), lane); };
#pragma unroll
            for (int ri = 0; ri < RH; ++ri) a[ri] = ld_a(ri, 0);
#pragma unroll
            for (int jj = 0; jj < PW; ++jj) {
              bq0[jj] = ld_b(jj, 0);
              bq1[jj] = ld_b(jj, j0 > 1 ? 1 : 0);
            }
            auto step = [&](int m, V4 (&bc)[PW]) {
              const int mn = m + 1 < j0 ? m + 1 : m, mb = m + 2 < j0 ? m + 2 : m;
#pragma unroll
              for (int ri = 0; ri < RH; ++ri) {
                const int i = row_of(ri);
                if (held_i(i)) {
#pragma unroll
                  for (int jj = 0; jj < PW; ++jj) {
                    if (jj < pw && (rhs_i(i) || i >= j0 + jj)) {
                      V4 x = acc[ri][jj];
#pragma unroll
                      for (int cch = 0; cch < 4; ++cch) x = Mfma<T>::op_sub(a[ri][cch], bc[jj][cch], x);
                      acc[ri][jj] = x;
                    }
                  }
                }
                a[ri] = ld_a(ri, mn);
              }
#pragma unroll
              for (int jj = 0; jj < PW; ++jj) bc[jj] = ld_b(jj, mb);
            };
#pragma unroll 1
            for (int m = 0; m < j0; ++m) {
              step(m, bq0);
#pragma unroll
              for (int jj = 0; jj < PW; ++jj) {
                const V4 t = bq0[jj];
                bq0[jj] = bq1[jj];
                bq1[jj] = t;
              }
            }
          } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) fetch(q, ab[q], bb[q]);
            for (int m = 0; m < j0; m += NB) {
#pragma unroll
              for (int q = 0; q < NB; ++q) {
                if (m + q < j0) {
                  apply(ab[q], bb[q]);
                  fetch(m + q + NB, ab[q], bb[q]);
                }
              }
            }
          }
        }
        // the operator (Ahat, or Btilde^T in the right-hand-side rows): rows are
        // unrolled, the PW columns of a row run in a loop whose result is moved
        // into its register slot by selects (a branch chain here would leave
        // the panel array in scratch memory)
#pragma unroll
        for (int ri = 0; ri < RH; ++ri) {
          const int i = row_of(ri);
          if (held_i(i)) {
#pragma unroll 1
            for (int jj = 0; jj < pw; ++jj) {
              if (rhs_i(i) || i >= j0 + jj) {
                const V4 v = init_tile(i, j0 + jj);
#pragma unroll
                for (int k = 0; k < PW; ++k) acc[ri][k] = jj == k ? acc[ri][k] + v : acc[ri][k];
              }
            }
          }
        }
        // (c) factor the panel, one column at a time (run-time loop; the tile
        // code that touches the register panel matches the column statically).
        // The diagonal tiles and the panel's own rows belong to the first pass;
        // a second pass reuses their W_j and L tiles from LDS, wave by wave.
#pragma unroll 1
        for (int jj = 0; jj < pw; ++jj) {
          const int col = j0 + jj;
          T* Wj = Wt + jj * TILE;
          // diagonal tile (row col is local row jj: wave jj, slot 0 of pass 0)
          if (h == 0) {
            if (wave == jj) {
#pragma unroll
              for (int k = 0; k < PW; ++k)
                if (k == jj) st_acc<T>(Wj, acc[0][k], lane);
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
              const int bj = potrf_c<T>(Wj, nullptr, n, col, lane, Lo ? ldiag(col) : nullptr);
              if (lane == 0 && bj >= 0 && bad < 0) bad = 16 * col + bj;
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
              T* dst = tl(col, col);
              for (int idx = lane; idx < TILE; idx += 64) dst[idx] = Wj[idx];
            }
            __syncthreads();
          }
          // panel solve L_i,col = C_i,col W^T for the rows below, then the
          // in-panel update C_i,j -= L_i,col L_j,col^T of the later columns
#pragma unroll
          for (int k = 0; k < PW; ++k) {
            if (k == jj) {
#pragma unroll
              for (int ri = 0; ri < RH; ++ri) {
                const int i = row_of(ri);
                if (i > col && held_i(i)) {
                  st_acc<T>(scr, acc[ri][k], lane);
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                  V4 x = {0, 0, 0, 0};
#pragma unroll
                  for (int cch = 0; cch < 4; ++cch)
                    x = Mfma<T>::op(ld_rowcol(scr, cch, lane), ld_rowcol(Wj, cch, lane), x);
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                  acc[ri][k] = x;
                  st_acc<T>(tl(i, col), x, lane);
                  if (i < j0 + pw) st_acc<T>(pub + (jj * PW + i - j0) * TILE, x, lane);
                }
              }
            }
          }
          if (h == 0) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __syncthreads();
          }
#pragma unroll
          for (int k = 0; k < PW - 1; ++k) {
            if (k == jj && jj + 1 < pw) {
#pragma unroll
              for (int ri = 0; ri < RH; ++ri) {
                const int i = row_of(ri);
                if (i > col && held_i(i)) {
                  st_acc<T>(scr, acc[ri][k], lane);
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                  T a[4];
#pragma unroll
                  for (int cch = 0; cch < 4; ++cch) a[cch] = -ld_rowcol(scr, cch, lane);
#pragma unroll
                  for (int j2 = k + 1; j2 < PW; ++j2) {
                    if (j2 < pw && (rhs_i(i) || i >= j0 + j2)) {
                      V4 x = acc[ri][j2];
#pragma unroll
                      for (int cch = 0; cch < 4; ++cch)
                        x = Mfma<T>::op(a[cch], ld_rowcol(pub + (jj * PW + j2) * TILE, cch, lane), x);
                      acc[ri][j2] = x;
                    }
                  }
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
              }
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
      }
    }

    // -------------------------------------------- factor output (three-call)
    // L is written to the caller's matrix only here, from the finished tiles:
    // lanes run down a tile column (contiguous in the column-major output).
    if (Lo) {
      for (int t = wave; t < (nt * (nt + 1)) / 2; t += NW) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;
        const T* src = I == J ? ldiag(J) : tl(I, J);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int idx = lane + 64 * h, row = idx & 15, cc = idx >> 4;
          const int p = 16 * I + row, q = 16 * J + cc;
          if (p < n && q < n && p >= q) Lo[(int64_t)q * n + p] = src[row * TST + cc];
        }
      }
    }

    // ------------------------------------------------ solves on the RHS row
    // The right-hand sides go through the row in chunks of 16 columns: the
    // first chunk's forward solve ran with the factorisation (or the stored
    // factor's forward sweep above); later chunks (more than 15 face DoFs)
    // load their columns and run both sweeps on the finished factor, as
    // calls (the kernel's registers stay those of the first chunk).
    backward(rhs_row);
    const bool failed = bad >= 0;
    double* X = args.X + E.rhs0;
    const int ca = tid >> 4, cl16 = tid & 15;   // 32 groups of 16 lanes; groups 0..15 do column sums
    if constexpr (!MC && sizeof(T) == 8) {
      // FP64, one chunk, no refinement: the straight-line form (the chunked
      // loop below costs this kernel registers)
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
        continue;
      }
      if (!ref64) {
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
        if (FUSED && args.M) contrib_element(E, X, ft, colsum[E.NI], NImax, args.M, args.E, args.B, args.F, e);
        continue;
      }
    }
    if (failed) {
      if (fp32) {
        if (tid == 0) args.info[e] = INFO_IR_FALLBACK;
        continue;
      }
      for (int idx = tid; idx < n * r; idx += NTHREADS) X[idx] = __builtin_nan("");
      if (tid == 0) args.info[e] = bad + 1;
      if (FUSED && args.M) {
        for (int idx = tid; idx < NImax * NImax; idx += NTHREADS)
          args.M[(int64_t)e * NImax * NImax + idx] = __builtin_nan("");
        for (int a = tid; a < NImax; a += NTHREADS) {
          args.E[(int64_t)e * NImax + a] = __builtin_nan("");
          args.B[(int64_t)e * NImax + a] = __builtin_nan("");
        }
        if (tid == 0) args.F[e] = __builtin_nan("");
      }
      continue;
    }
    int it_max = 0;
    for (int c0 = 0; c0 < (MC ? r : 1); c0 += R_CHUNK) {
      const int ch = c0 / R_CHUNK;
      T* rowc = tl(nt + ch, 0);   // this chunk's tile row
      if (MC && c0 > 0) {
        __syncthreads();
        if (tid == 0) {
          E.c0 = c0;
          E.rc = r - c0 < R_CHUNK ? r - c0 : R_CHUNK;
        }
        __syncthreads();
        if (ch >= nfused) {   // not eliminated with the factorisation: forward sweep first
          for (int J = wave; J < nt; J += NW)
            st_acc<T>(rowc + (int64_t)J * TILE, init_tile(nt + ch, J), lane);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          __syncthreads();
          ll::sweep_call<T, RPW, false, OCC, NW>(Lb, rowc, nt, xb, scr, wave, lane);
        }
        ll::sweep_call<T, RPW, true, OCC, NW>(Lb, rowc, nt, xb, scr, wave, lane);
      }
      const int rc = E.rc;
      double* Xc = X + (int64_t)c0 * n;
      if (fp32 || ref64) {
        // ----------------------------------------------- FP64 refinement
        // FP32 factor: FP64 residuals until the backward error target;
        // FP64 factor: one step with a double-double residual.
        double* part = part_s;
        ir_accumulate<T>(Xc, rowc, c, n, rc, true, cx, xmax, part);
        const double* Btg = FUSED ? nullptr : args.Btil + E.rhs0;
        int it = 0;
        for (;; ++it) {
          if (!fp32 && it >= 1) {
            if (tid == 0) conv = 1;
            break;
          }
          const double anorm = ir_residual<T, FUSED, !fp32>(E, kapg, X, c, cx, g, ft, bf, colsum, Btg, rowc, red);
          if (fp32) {
            if (it == 0) ir_colmax<T, FUSED>(E, rowc, ft, bf, c, colsum, Btg, true, bmax, part);
            ir_colmax<T, FUSED>(E, rowc, ft, bf, c, colsum, Btg, false, rmax, part);
            if (tid == 0) {
              const double be = ir_backward_error(rmax, xmax, bmax, rc, anorm);
              conv = ir_decide(be, be_prev, it, args.max_iters, args.ir_tol);
              be_prev = be;
            }
            __syncthreads();
            if (conv != 0) break;
          }
          ll::sweep_call<T, RPW, false, OCC, NW>(Lb, rowc, nt, xb, scr, wave, lane);
          ll::sweep_call<T, RPW, true, OCC, NW>(Lb, rowc, nt, xb, scr, wave, lane);
          ir_accumulate<T>(Xc, rowc, c, n, rc, false, cx, xmax, part);
        }
        it_max = it > it_max ? it : it_max;
        if (conv < 0) break;
        // zero-mean projection: cx still holds c^T X of the converged iterate
        for (int idx = tid; idx < n * rc; idx += NTHREADS) Xc[idx] -= cx[idx / n] * E.inv_area;
        __syncthreads();
      } else {
        {
          double v = 0.0;
          if (ca < rc)
            for (int p = cl16; p < n; p += 16) v += c[p] * (double)rowc[(int64_t)(p >> 4) * TILE + ca * TST + (p & 15)];
          v = group16_sum(v);
          if (cl16 == 0 && ca < 16) cx[ca] = v * E.inv_area;
        }
        __syncthreads();
        for (int idx = tid; idx < n * rc; idx += NTHREADS) {
          const int a = idx / n, p = idx - a * n;
          Xc[idx] = (double)rowc[(int64_t)(p >> 4) * TILE + a * TST + (p & 15)] - cx[a];
        }
        __syncthreads();
      }
    }
    if ((fp32 || ref64) && tid == 0) {
      if (args.ir_iters && (!args.only_fallback || args.fb_final)) args.ir_iters[e] = it_max;
      if (conv < 0) args.info[e] = INFO_IR_FALLBACK;
    }
    if (fp32 && conv < 0) continue;
    if (FUSED && args.M) contrib_element(E, X, ft, colsum[E.NI], NImax, args.M, args.E, args.B, args.F, e);
  }
}

template <typename T, bool FUSED, int PW, int RPW, int OCC, int NWV = 8, bool MC = false, bool REF = MC>
static hipError_t launch_ll_t(const BatchDev& d, LocalArgs a, size_t lds, int grid, hipStream_t st) {
  auto kern = k_local_ll<T, FUSED, PW, RPW, OCC, NWV, MC, REF>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NWV), lds, st, d, a);
  return hipGetLastError();
}

}  // namespace mhm
