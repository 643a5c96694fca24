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
#include "mhm_common.h"
#include "mhm_kernels.h"

namespace mhm {

constexpr int NTHREADS = 256;
constexpr int NWAVES = NTHREADS / 64;

// =============================================================== k_assemble
constexpr int ASM_TAB = 256;   // elements of up to this many nodes use the stencil table
template <bool TAB>
__global__ void __launch_bounds__(NTHREADS) k_assemble(BatchDev b, double* Ahat, double* Btil, double* cout,
                                                        double* area, int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double red[48];
  __shared__ double colsum[R_MAX];
  __shared__ double gam;
  // kappa[s^2] | c[n] | bf[n] | ft[NI(s+1)] | stencil[7][tn] | j[tn].  TAB: a
  // stencil table for every element (tn = n_max); otherwise (where that
  // would not fit in LDS) tn = min(n_max, 256): the table serves the
  // elements of at most 256 nodes, and larger ones take each column's
  // stencil where its wave writes the column (more registers)
  extern __shared__ double dyn[];
  const int tid = threadIdx.x;
  const int smax = b.s_max, nmax = (smax + 1) * (smax + 2) / 2;
  const int tn = TAB || nmax < ASM_TAB ? nmax : ASM_TAB;
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
    double* sd = ft + nimax(b) * (smax + 1);      // the seven stencil values of node q at sd[k tn + q]
    int* sj = reinterpret_cast<int*>(sd + 7 * tn);  // lattice row j of node q
    const bool tab = TAB || n <= ASM_TAB;
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
      if (tab) {
        sd[p] = st.d;
        sd[tn + p] = st.e;
        sd[2 * tn + p] = st.w;
        sd[3 * tn + p] = st.n;
        sd[4 * tn + p] = st.so;
        sd[5 * tn + p] = st.nw;
        sd[6 * tn + p] = st.se;
        sj[p] = j;
      }
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
    // Ahat, column-major.  Small elements (n <= 256): as one contiguous run
    // of n^2 values, consecutive threads on consecutive entries (full cache
    // lines; a column of a few lanes' width would leave most of a wave's last
    // store idle), each from the stencil table of its column q.  Larger ones:
    // wave w writes columns q = w, w+4, ... with the column's stencil (from
    // the table, or from kappa in LDS, the same in every lane) in registers,
    // lanes sweeping rows.
    double* A = Ahat + E.mat0;
    if (n > ASM_TAB) {
      const int w = tid >> 6, lane = tid & 63;
      for (int q = w; q < n; q += NWAVES) {
        int j;
        double d, ve, vw, vn, vs, vnw, vse;
        if (tab) {
          j = sj[q];
          d = sd[q];
          ve = sd[tn + q];
          vw = sd[2 * tn + q];
          vn = sd[3 * tn + q];
          vs = sd[4 * tn + q];
          vnw = sd[5 * tn + q];
          vse = sd[6 * tn + q];
        } else {
          int i;
          node_ij(q, s, i, j);
          const Stencil sq = stencil(i, j, s, E.G, [&](int t) { return kap[t]; });
          d = sq.d;
          ve = sq.e;
          vw = sq.w;
          vn = sq.n;
          vs = sq.so;
          vnw = sq.nw;
          vse = sq.se;
        }
        const int pE = q + 1, pW = q - 1, pN = q + (s + 1 - j), pS = q - (s + 2 - j), pNW = q + (s - j),
                  pSE = q - (s + 1 - j);
        const double gcq = g * c[q];
        for (int p = lane; p < n; p += 64) {
          double v = gcq * c[p];
          v += (p == q) ? d : 0.0;
          v += (p == pE) ? ve : 0.0;
          v += (p == pW) ? vw : 0.0;
          v += (p == pN) ? vn : 0.0;
          v += (p == pS) ? vs : 0.0;
          v += (p == pNW) ? vnw : 0.0;
          v += (p == pSE) ? vse : 0.0;
          A[(int64_t)q * n + p] = v;
        }
      }
    } else {
      const int nn = n * n;
      const int dq = NTHREADS / n, dp = NTHREADS - dq * n;   // index step NTHREADS in (q, p)
      int q = tid / n, p = tid - q * n;
      for (int idx = tid; idx < nn; idx += NTHREADS) {
        const int j = sj[q], off = p - q;
        double v = g * c[q] * c[p];
        v += off == 0 ? sd[q] : 0.0;
        v += off == 1 ? sd[tn + q] : 0.0;
        v += off == -1 ? sd[2 * tn + q] : 0.0;
        v += off == s + 1 - j ? sd[3 * tn + q] : 0.0;
        v += off == -(s + 2 - j) ? sd[4 * tn + q] : 0.0;
        v += off == s - j ? sd[5 * tn + q] : 0.0;
        v += off == -(s + 1 - j) ? sd[6 * tn + q] : 0.0;
        A[idx] = v;
        p += dp;
        q += dq;
        if (p >= n) {
          p -= n;
          ++q;
        }
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

// --------------------------------------------------------------- k_contrib
// One DPP step of a wave reduction on a double (both halves moved alike);
// lanes of a masked-off row get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_step(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the 64 lanes of a wave (all lanes active), in every lane: lane
// xor 1 and xor 2 (quad permutes), the mirrored lane of each half row and of
// each row of 16 (every lane then holds its row's sum), lane 15 of rows 0 and
// 2 into rows 1 and 3, lane 31 into rows 2 and 3; lane 63 has the total.
__device__ __forceinline__ double wave_sum_rows(double v) {
  v += dpp_step<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_step<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_step<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_step<0x140, 0xf>(v);   // row_mirror
  v += dpp_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
  return readlane(v, 63);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)v), hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}
// Orders one wave's LDS accesses around it (a wavefront-scope fence pair).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The face loads R(a, k) of lattice node k on face ef for every DoF a of that
// face, written to ft[a (s + 1) + k]: the quantity face_load gives entry by
// entry (eq. (9)), taken here node by node so that the Gauss points of the
// node's two sub-edges and their Legendre values are computed once for all
// the DoFs.  The Legendre recurrence q P_q = (2q - 1) t P_(q-1) - (q - 1)
// P_(q-2) runs with its coefficients folded at compile time (q <= 4).
__device__ __forceinline__ void face_node_loads(const Elem& E, int ef, int k, double* ft) {
  constexpr int QN = MHM_L_LIMIT + 1;
  const double r15 = 0.38729833462074168852;  // sqrt(15)/10
  const double xg[3] = {0.5 - r15, 0.5, 0.5 + r15};
  const double wg[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  const int s = E.s, lp1 = E.l + 1, m = E.m, per = s / m, sp1 = s + 1;
  const bool fl = E.flip[ef] != 0;
  double acc[2][QN];
  int sg[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
#pragma unroll
    for (int q = 0; q < QN; ++q) acc[side][q] = 0.0;
    const int seg = side == 0 ? k - 1 : k;   // node k ends sub-edge k-1 and starts sub-edge k
    sg[side] = -1;
    if (seg < 0 || seg >= s) continue;
    const int sgf = (fl ? s - 1 - seg : seg) / per;   // the segment (of the m) holding the sub-edge
    sg[side] = sgf;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const double tau = (seg + xg[g]) * E.inv_s;
      const double gp = fl ? 1.0 - tau : tau;
      const double t = 2.0 * (m * gp - sgf) - 1.0;
      const double w = wg[g] * (side == 0 ? xg[g] : 1.0 - xg[g]);
      double p0 = 1.0, p1 = t;
      acc[side][0] += w;
      acc[side][1] += w * t;
#pragma unroll
      for (int q = 2; q < QN; ++q) {
        const double p2 = ((2.0 * q - 1.0) / q) * t * p1 - ((q - 1.0) / q) * p0;
        acc[side][q] += w * p2;
        p0 = p1;
        p1 = p2;
      }
    }
  }
  const double scale = -(double)E.sigma[ef] * E.flen[ef] * E.inv_s;
  double* col = ft + (size_t)ef * E.P * sp1 + k;
  for (int segf = 0; segf < m; ++segf) {
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      if (q < lp1) {
        const double v = (sg[0] == segf ? acc[0][q] : 0.0) + (sg[1] == segf ? acc[1][q] : 0.0);
        col[(size_t)(segf * lp1 + q) * sp1] = scale * v;
      }
    }
  }
}

// Step a6 alone (the three-call form), eq. (6): the element's blocks
//   M[a][b] = -sum_k R(a,k) X[node(ef,k)][b]  (b < NI),
//   E[a]    =  sum_k R(a,k) X[node(ef,k)][NI],   B[a] = -sum_k R(a,k),
// F = the integral of f, for the face DoFs a (face ef = a / P), k = 0..s
// over the face's lattice nodes, R(a,k) the face load.  One wave per element
// and no workgroup barriers: lane 0 decodes the element into the wave's LDS
// slot; the lanes build the wave's table of R, one lane per face node; then,
// per chunk of ccmax columns of X, the wave copies the face rows of
// those columns into LDS - one load per (column, face node), so a load
// instruction covers 64 entries instead of the few distinct nodes of a lane
// per (a, b) pair - and each lane sums over k for its (a, b) pairs from LDS,
// a fastest, so the stores of M run along its columns.  Dynamic LDS per wave
// (`cap` doubles): the R table (NImax (s_max + 1)), the staged face rows
// (ccmax 3 (s_max + 1)) and the 3 (s_max + 1) face-node offsets.
__global__ void __launch_bounds__(NTHREADS) k_contrib(BatchDev b, const double* X, double* M, double* Ev,
                                                       double* Bv, double* F, const int32_t* info, int cap,
                                                       int ccmax) {
  __shared__ Elem Ew[NWAVES];
  extern __shared__ double ctab[];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int NImax = nimax(b);
  Elem& E = Ew[wave];
  double* ft = ctab + (size_t)wave * cap;
  double* xs = ft + (size_t)NImax * (b.s_max + 1);
  int* fnode = (int*)(xs + (size_t)ccmax * 3 * (b.s_max + 1));
  for (int e = blockIdx.x * nw + wave; e < b.n_elem; e += gridDim.x * nw) {
    if (info != nullptr && info[e] != 0 && info[e] != INFO_IR_FALLBACK) continue;
    int ok = 0;
    wave_sync();   // the previous element's reads of E and of the tables are done
    if (lane == 0) ok = load_elem(b, e, E) && E.rhs0 >= 0;
    wave_sync();
    if (__builtin_amdgcn_readlane(ok, 0) == 0) continue;
    // the element's sizes are the same in every lane: keep them scalar
    const int s = uni(E.s), n = uni(E.n), r = uni(E.r), NI = uni(E.NI), P = uni(E.P), sp1 = s + 1;
    const int nf = 3 * sp1;   // face nodes, face by face (a corner appears on two faces)
    double* Me = M + (int64_t)e * NImax * NImax;
    double* Ee = Ev + (int64_t)e * NImax;
    double* Be = Bv + (int64_t)e * NImax;
    {
      double fs = 0.0;
      const double* fe = b.f + uni64(E.tri0);
#pragma unroll 8
      for (int t = lane; t < s * s; t += 64) fs += fe[t];
      fs = wave_sum_rows(fs);
      if (lane == 0) F[e] = fs * (E.area / ((double)s * s));
    }
    for (int idx = lane; idx < nf; idx += 64) {
      const int ef = idx / sp1, k = idx - ef * sp1;
      face_node_loads(E, ef, k, ft);
      fnode[idx] = 8 * face_node(ef, k, s);   // byte offset in a column of X
    }
    // padding of the blocks beyond NI (to NImax)
    for (int idx = lane; idx < NImax * NImax; idx += 64) {
      const int a = idx % NImax, bb = idx / NImax;
      if (a >= NI || bb >= NI) Me[idx] = 0.0;
    }
    for (int a = NI + lane; a < NImax; a += 64) {
      Ee[a] = 0.0;
      Be[a] = 0.0;
    }
    wave_sync();
    for (int a = lane; a < NI; a += 64) {
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < sp1; ++k) v += ft[a * sp1 + k];
      Be[a] = -v;
    }
    const char* Xc = (const char*)(X + uni64(E.rhs0));
    for (int b0 = 0; b0 < r; b0 += ccmax) {
      const int cc = r - b0 < ccmax ? r - b0 : ccmax;
      // stage: xs[c nf + j] = X[b0 + c][node j]; byte offsets stay below
      // 2^32 (r n 8 <= 49 * 2145 * 8)
#pragma unroll 8
      for (int idx = lane; idx < cc * nf; idx += 64) {
        const int c = idx / nf, j = idx - c * nf;
        xs[idx] = *(const double*)(Xc + (8u * (uint32_t)((b0 + c) * n) + (uint32_t)fnode[j]));
      }
      wave_sync();
      for (int idx = lane; idx < NI * cc; idx += 64) {
        const int c = idx / NI, a = idx - c * NI;
        const double* Ra = ft + a * sp1;
        const double* xa = xs + c * nf + (a / P) * sp1;
        double v = 0.0;
#pragma unroll 8
        for (int k = 0; k < sp1; ++k) v += Ra[k] * xa[k];
        const int bb = b0 + c;
        if (bb < NI) Me[(int64_t)bb * NImax + a] = -v;
        else Ee[a] = v;
      }
      wave_sync();   // the reads of xs are done before the next chunk overwrites it
    }
  }
}

template <typename T, bool IN_LDS, bool FUSED>
__global__ void __launch_bounds__(NTHREADS) k_local(BatchDev b, LocalArgs args) {
  typedef typename Mfma<T>::v4 V4;
  __shared__ Elem E;
  __shared__ int ok, bad, conv;
  __shared__ double be_prev;
  __shared__ double red[48];
  __shared__ double colsum[R_CHUNK];   // one chunk only (r <= 16)
  __shared__ double cx[16];          // (c^T X) per column
  __shared__ double gam;
  __shared__ double part_s[32 * (NTHREADS / 256)];
  __shared__ double rmax[16], xmax[16], bmax[16];
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NImax = nimax(b);
  const bool fp32 = sizeof(T) == 4;

  const int n_launch = launch_count(args, b.n_elem);
  for (int k_el = blockIdx.x; k_el < n_launch; k_el += gridDim.x) {
    const int e = launch_elem(args, k_el);
    __syncthreads();   // every thread is done with the previous element's shared flags
    if (tid == 0) {
      int st = INFO_OK;
      if (args.only_fallback && args.info[e] != INFO_IR_FALLBACK) {
        ok = 0;
      } else {
        const bool good = load_elem(b, e, E) && E.rhs0 >= 0 && (FUSED || E.mat0 >= 0);
        if (!good) st = INFO_BAD_DESC;
        else if ((E.nt * (E.nt + 1)) / 2 + E.nt > args.tile_cap || E.n > args.n_cap || E.r > R_CHUNK ||
                 (FUSED && E.NI * (E.s + 1) > args.f_cap) || (FUSED && IN_LDS && E.s * E.s > args.k_cap))
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
    // FP64: one refinement step with a double-double residual where a plain
    // FP64 solve is not accurate enough (the FP32 path always refines)
    const bool ref64 = !fp32 && refine64_needed(args.refine64, kapg, s, red);

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

    if ((fp32 || ref64) && !failed) {
      // ----------------------------------------------- FP64 refinement
      // FP32 factor: FP64 residuals until the backward error target;
      // FP64 factor: one step with a double-double residual.
      ir_accumulate_body<T>(X, tl(nt, 0), c, n, r, true, cx, xmax, part_s);
      const double* Btg = FUSED ? nullptr : args.Btil + E.rhs0;
      const double g = gam;
      int it = 0;
      for (;; ++it) {
        if (!fp32 && it >= 1) {
          if (tid == 0) conv = 1;
          __syncthreads();
          break;
        }
        const double anorm = ir_residual_body<T, FUSED, !fp32>(E, kap_lds ? kapl : kapg, X, c, cx, g, ft, bf,
                                                                colsum, Btg, tl(nt, 0), red);
        if (fp32) {
          if (it == 0) ir_colmax_body<T, FUSED>(E, tl(nt, 0), ft, bf, c, colsum, Btg, true, bmax, part_s);
          ir_colmax_body<T, FUSED>(E, tl(nt, 0), ft, bf, c, colsum, Btg, false, rmax, part_s);
          if (tid == 0) {
            const double be = ir_backward_error(rmax, xmax, bmax, r, anorm);
            conv = ir_decide(be, be_prev, it, args.max_iters, args.ir_tol);
            be_prev = be;
          }
          __syncthreads();
          if (conv != 0) break;
        }
        forward();
        backward();
        ir_accumulate_body<T>(X, tl(nt, 0), c, n, r, false, cx, xmax, part_s);
      }
      const bool cvd = conv > 0;
      if (tid == 0) {
        if (args.ir_iters && (!args.only_fallback || args.fb_final)) args.ir_iters[e] = it;
        if (!cvd) args.info[e] = INFO_IR_FALLBACK;
      }
      if (!cvd) continue;   // recomputed by the FP64 fallback pass
      // zero-mean projection of the FP64 iterate (cx is c^T X of the converged iterate)
      for (int idx = tid; idx < n * r; idx += NTHREADS) X[idx] -= cx[idx / n] * E.inv_area;
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

// ------------------------------------------------ computeSolution, scatter
// Eq. (4): u = u_0 + sum_a lambda_a eta^a + eta^f at the sub-mesh nodes of
// each element, with lambda_a = sol[gdof[e][a]] and u_0 = sol[erow[e]].
// One workgroup per element, nodes across the threads (coalesced X reads).
__global__ void __launch_bounds__(NTHREADS) k_reconstruct(BatchDev b, const double* X, const int32_t* gdof,
                                                           const int32_t* erow, const double* sol, int32_t n_rows,
                                                           double* u, const int32_t* info) {
  __shared__ Elem E;
  __shared__ int ok;
  __shared__ double lam[R_MAX];
  __shared__ double u0;
  const int tid = threadIdx.x;
  const int NImax = nimax(b);
  for (int e = blockIdx.x; e < b.n_elem; e += gridDim.x) {
    __syncthreads();
    if (tid == 0) {
      ok = load_elem(b, e, E) && E.rhs0 >= 0 && E.node0 >= 0 && (!info || info[e] == INFO_OK || info[e] == INFO_IR_FALLBACK);
      if (ok) u0 = (erow[e] >= 0 && erow[e] < n_rows) ? sol[erow[e]] : __longlong_as_double(0x7ff8000000000000ll);
    }
    if (tid < R_MAX) lam[tid] = 0.0;
    __syncthreads();
    if (!ok) continue;
    if (tid < E.NI) {
      const int32_t gi = gdof[(int64_t)e * NImax + tid];
      lam[tid] = (gi >= 0 && gi < n_rows) ? sol[gi] : __longlong_as_double(0x7ff8000000000000ll);
    }
    __syncthreads();
    const int n = E.n, NI = E.NI;
    const double* Xe = X + uni64(E.rhs0);
    for (int p = tid; p < n; p += NTHREADS) {
      double v = u0 + Xe[(int64_t)NI * n + p];
      for (int a = 0; a < NI; ++a) v += Xe[(int64_t)a * n + p] * lam[a];
      u[E.node0 + p] = v;
    }
  }
}

// Position of column `col` in row `row` of a CSR pattern with sorted columns
// (-1 if absent).
__device__ __forceinline__ int64_t csr_find(const int32_t* row_ptr, const int32_t* col_idx, int row, int col) {
  int lo = row_ptr[row], hi = row_ptr[row + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int cm = col_idx[mid];
    if (cm == col) return mid;
    if (cm < col) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// The element share of eq. (6) added into the skeleton system (the assembly
// part of reduceLocalProblems): rows and columns gdof[e][a] (multipliers) and
// erow[e] (the element's u_0), M into the multiplier block, B and B^T into
// the coupling, E and F into the right-hand side.  Vector FP64 atomics;
// entries missing from the pattern are counted in *missing.
__global__ void __launch_bounds__(NTHREADS) k_skeleton_scatter(BatchDev b, const double* M, const double* Ev,
                                                                const double* Bv, const double* F,
                                                                const int32_t* gdof, const int32_t* erow,
                                                                const int32_t* row_ptr, const int32_t* col_idx,
                                                                double* vals, double* rhs, const int32_t* info,
                                                                int32_t n_rows, int32_t* missing) {
  const int NImax = nimax(b);
  const int per = NImax * NImax + 2 * NImax + NImax + 1;   // M, B, B^T, E, F
  const int64_t total = (int64_t)b.n_elem * per;
  for (int64_t idx = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NTHREADS) {
    const int e = (int)(idx / per);
    int k = (int)(idx - (int64_t)e * per);
    if (info && info[e] != INFO_OK && info[e] != INFO_IR_FALLBACK) continue;
    const int l = b.l[e];
    const int m = b.m ? b.m[e] : 1;
    if (l < 0 || l > MHM_L_LIMIT || l > b.l_max || m < 1 || m * (l + 1) > b.p_max) continue;
    const int NI = 3 * m * (l + 1);
    const int32_t* g = gdof + (int64_t)e * NImax;
    int row = -1, col = -1;
    double v = 0.0;
    bool to_rhs = false, used = true;
    if (k < NImax * NImax) {
      const int a = k % NImax, c = k / NImax;
      used = a < NI && c < NI;
      if (used) {
        row = g[a];
        col = g[c];
        v = M[(int64_t)e * NImax * NImax + k];
      }
    } else if ((k -= NImax * NImax) < NImax) {
      used = k < NI;
      if (used) {
        row = erow[e];
        col = g[k];
        v = Bv[(int64_t)e * NImax + k];
      }
    } else if ((k -= NImax) < NImax) {
      used = k < NI;
      if (used) {
        row = g[k];
        col = erow[e];
        v = Bv[(int64_t)e * NImax + k];
      }
    } else if ((k -= NImax) < NImax) {
      used = k < NI;
      if (used) {
        row = g[k];
        v = Ev[(int64_t)e * NImax + k];
        to_rhs = true;
      }
    } else {
      row = erow[e];
      v = F[e];
      to_rhs = true;
    }
    if (!used) continue;
    const bool in_range = row >= 0 && row < n_rows && (to_rhs || (col >= 0 && col < n_rows));
    if (in_range && to_rhs) {
      atomicAdd(rhs + row, v);
    } else {
      const int64_t pos = in_range ? csr_find(row_ptr, col_idx, row, col) : -1;
      if (pos >= 0) atomicAdd(vals + pos, v);
      else if (missing) atomicAdd(missing, 1);
    }
  }
}

hipError_t launch_reconstruct(const mhm_batch* bt, const double* X, const int32_t* gdof, const int32_t* erow,
                              const double* sol, int32_t n_rows, double* u, const int32_t* info, int grid,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_reconstruct, dim3(grid), dim3(NTHREADS), 0, st, to_dev(bt), X, gdof, erow, sol, n_rows, u,
                     info);
  return hipGetLastError();
}

hipError_t launch_skeleton_scatter(const mhm_batch* bt, const double* M, const double* E, const double* B,
                                   const double* F, const int32_t* gdof, const int32_t* erow, const int32_t* row_ptr,
                                   const int32_t* col_idx, int32_t n_rows, double* vals, double* rhs,
                                   const int32_t* info, int32_t* missing, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_skeleton_scatter, dim3(grid), dim3(NTHREADS), 0, st, to_dev(bt), M, E, B, F, gdof, erow,
                     row_ptr, col_idx, vals, rhs, info, n_rows, missing);
  return hipGetLastError();
}

// ------------------------------------------------------- size-class binning
// Element e goes to the first class c with s[e] <= s_hi[c] (an s outside
// [1, MHM_S_LIMIT] to class 0, whose kernel reports the descriptor).  Class c's
// list is elist[c * n_elem ...], in element order; counts[c] is its length.
// One workgroup of 1024 threads, chunks of 1024 elements, wave ballots for
// the in-chunk positions: nothing needs clearing beforehand.
__global__ void __launch_bounds__(1024) k_bin(const int32_t* s, int n_elem, BinClasses cls, int32_t* elist,
                                              int32_t* counts) {
  __shared__ int wsum[16][BIN_MAX_CLASSES];
  __shared__ int run[BIN_MAX_CLASSES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < cls.n) run[tid] = 0;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = 0; base < n_elem; base += 1024) {
    const int e = base + tid;
    int c = -1;
    if (e < n_elem) {
      const int se = s[e];
      c = 0;
      if (se >= 1 && se <= MHM_S_LIMIT)
        while (c < cls.n - 1 && se > cls.s_hi[c]) ++c;
    }
    unsigned long long mine = 0;
    for (int k = 0; k < cls.n; ++k) {
      const unsigned long long m = __ballot64(c == k);
      if (c == k) mine = m;
      if (lane == 0) wsum[wave][k] = __popcll(m);
    }
    __syncthreads();
    if (c >= 0) {
      int pos = run[c] + __popcll(mine & below);
      for (int w = 0; w < wave; ++w) pos += wsum[w][c];
      elist[(int64_t)c * n_elem + pos] = e;
    }
    __syncthreads();
    if (tid < cls.n) {
      int t = 0;
      for (int w = 0; w < 16; ++w) t += wsum[w][tid];
      run[tid] += t;
    }
    __syncthreads();
  }
  if (tid < cls.n) counts[tid] = run[tid];
}

hipError_t launch_bin(const mhm_batch* bt, const BinClasses& cls, int32_t* elist, int32_t* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_bin, dim3(1), dim3(1024), 0, st, bt->s, bt->n_elem, cls, elist, counts);
  return hipGetLastError();
}

// ------------------------------------------------------------- host launchers
int local_face_cap(const mhm_batch* bt) { return nimax(to_dev(bt)) * (bt->s_max + 1); }

hipError_t launch_assemble(const mhm_batch* bt, double* Ahat, double* Btil, double* c, double* area, int32_t* info,
                           int grid, hipStream_t st) {
  const int smax = bt->s_max;
  const int nmax = (smax + 1) * (smax + 2) / 2;
  auto lds_of = [&](int tn) {
    return sizeof(double) * ((size_t)smax * smax + 2 * (size_t)nmax + local_face_cap(bt) + 7 * (size_t)tn) +
           sizeof(int) * (size_t)tn;
  };
  // the full stencil table where it fits in the CU's 160 KB of LDS next to
  // the kernel's static arrays (4 KB kept for them; s_max <= 53 at the
  // largest p_max), else the table for the small elements only
  const bool full = lds_of(nmax) + 4096 <= 160 * 1024;
  const size_t lds = lds_of(full || nmax < ASM_TAB ? nmax : ASM_TAB);
  const void* kern = full ? (const void*)k_assemble<true> : (const void*)k_assemble<false>;
  hipError_t err = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  if (full) hipLaunchKernelGGL(k_assemble<true>, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), Ahat, Btil, c, area, info);
  else hipLaunchKernelGGL(k_assemble<false>, dim3(grid), dim3(NTHREADS), lds, st, to_dev(bt), Ahat, Btil, c, area, info);
  return hipGetLastError();
}

hipError_t launch_contrib(const mhm_batch* bt, const double* X, double* M, double* E, double* B, double* F,
                          const int32_t* info, int grid, hipStream_t st) {
  // one wave per element.  LDS bounds how many elements run at once on a CU
  // (160 KB): the staged columns per chunk (ccmax, 16 down to 4) are the
  // most that keep a wave's tables within 10 KB (four workgroups of four
  // waves per CU) where that leaves at least four, as many waves per
  // workgroup (up to four) as fit their tables in 64 KB, a workgroup for
  // every nw elements (capped: the waves loop over the rest)
  (void)grid;
  const int fcap = local_face_cap(bt), nf = 3 * (bt->s_max + 1), ncap = (nf + 1) / 2;
  int ccmax = 16;
  while (ccmax > 4 && (size_t)(fcap + ccmax * nf + ncap) * sizeof(double) > 10240) ccmax /= 2;
  const int cap = fcap + ccmax * nf + ncap;
  int nw = (int)(65536 / (sizeof(double) * (size_t)cap));
  nw = nw < 1 ? 1 : nw > NWAVES ? NWAVES : nw;
  const size_t lds = sizeof(double) * (size_t)cap * nw;
  hipError_t err = hipFuncSetAttribute((const void*)k_contrib, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  const int64_t need = ((int64_t)bt->n_elem + nw - 1) / nw;
  const int g = (int)(need < 65535 ? (need > 0 ? need : 1) : 65535);
  hipLaunchKernelGGL(k_contrib, dim3(g), dim3(64 * nw), lds, st, to_dev(bt), X, M, E, B, F, info, cap, ccmax);
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
