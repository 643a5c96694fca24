// Device-side building blocks of the MHM local-problem kernels (gfx950).
//
// Element geometry, sub-mesh lattice indexing, the P1 7-point stencil of the
// Darcy form, the face quadrature of the multiplier loads, and the 16x16
// MFMA tile primitives used by the Cholesky factorisation and the solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhm.h"

namespace mhm {

// Element-level info codes (see mhm.h).
constexpr int INFO_OK = 0;
constexpr int INFO_IR_FALLBACK = -1;
constexpr int INFO_BAD_DESC = -2;
constexpr int INFO_TOO_LARGE = -3;
constexpr int INFO_NO_FACTOR = -4;
// Right-hand sides per element: at most R_MAX = 3 MHM_P_LIMIT + 1; the
// kernels solve them in chunks of R_CHUNK (one 16-wide tile row).  The
// register-resident and right-looking kernels take one chunk only.
constexpr int R_CHUNK = 16;
constexpr int R_MAX = 3 * MHM_P_LIMIT + 1;

// Batch descriptor as passed to kernels (by value).
struct BatchDev {
  int n_elem, s_max, l_max;
  const int32_t* s;
  const int32_t* l;
  const double* vert;
  const int8_t* sigma;
  const int8_t* flip;
  const double* kappa;
  const double* f;
  const int64_t* tri_off;
  const int64_t* mat_off;
  const int64_t* rhs_off;
  const int64_t* node_off;
  int64_t tri_total, mat_total, rhs_total, node_total;
  const int32_t* m;   // segments per face, null = 1
  int p_max;          // bound on m (l + 1): contribution blocks are 3 p_max wide
};

// Padded width of the contribution blocks M, E, B.
__host__ __device__ inline int nimax(const BatchDev& b) { return 3 * b.p_max; }

inline BatchDev to_dev(const mhm_batch* p) {
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
  d.m = p->m;
  d.p_max = p->p_max > 0 ? p->p_max : p->l_max + 1;
  return d;
}

// One element's geometry and offsets, decoded once per workgroup.
struct Elem {
  int s, l, n, NI, r, nt;   // nt = ceil(n / 16) tiles per matrix edge
  int m, P;                 // segments per face, face DoFs per face m (l + 1); NI = 3 P
  int c0, rc;               // right-hand-side chunk in work: columns c0 .. c0 + rc - 1 (rc <= 16)
  double area;              // |K|
  double G[3][3];           // D_a . D_b / (4 |K|): P1 stiffness of any sub-triangle / kappa
  double flen[3];           // |F_e|
  double cunit;             // |K| / (3 s^2): mass of one sub-triangle corner
  double inv_area, inv_s;
  int sigma[3], flip[3];
  int64_t tri0, mat0, rhs0, node0;
};

__device__ __forceinline__ int row_start(int j, int s) { return j * (2 * s + 3 - j) / 2; }
__device__ __forceinline__ int node_idx(int i, int j, int s) { return row_start(j, s) + i; }
__device__ __forceinline__ int tri_up(int i, int j, int s) { return j * (2 * s - j) + 2 * i; }
__device__ __forceinline__ int tri_dn(int i, int j, int s) { return j * (2 * s - j) + 2 * i + 1; }

// Lattice coordinates of node p.
__device__ __forceinline__ void node_ij(int p, int s, int& i, int& j) {
  const double b = 2.0 * s + 3.0;
  int jj = (int)((b - sqrt(b * b - 8.0 * p)) * 0.5);
  if (jj < 0) jj = 0;
  if (jj > s) jj = s;
  while (jj < s && row_start(jj + 1, s) <= p) ++jj;
  while (jj > 0 && row_start(jj, s) > p) --jj;
  j = jj;
  i = p - row_start(jj, s);
}

// Decode and validate element e.  Returns false for an inconsistent descriptor.
__device__ __forceinline__ bool load_elem(const BatchDev& b, int e, Elem& E) {
  const int s = b.s[e];
  const int l = b.l[e];
  const int m = b.m ? b.m[e] : 1;
  if (s < 1 || s > MHM_S_LIMIT || s > b.s_max || l < 0 || l > MHM_L_LIMIT || l > b.l_max) return false;
  if (m < 1 || s % m != 0 || m * (l + 1) > b.p_max || m * (l + 1) > MHM_P_LIMIT) return false;
  E.s = s;
  E.l = l;
  E.m = m;
  E.P = m * (l + 1);
  E.n = (s + 1) * (s + 2) / 2;
  E.NI = 3 * E.P;
  E.c0 = 0;
  E.r = E.NI + 1;
  E.rc = E.r < R_CHUNK ? E.r : R_CHUNK;
  E.nt = (E.n + 15) / 16;
  const int64_t t0 = b.tri_off[e], t1 = b.tri_off[e + 1];
  if (t0 < 0 || t1 - t0 != (int64_t)s * s || t1 > b.tri_total) return false;
  E.tri0 = t0;
  if (b.mat_off) {
    const int64_t m0 = b.mat_off[e], m1 = b.mat_off[e + 1];
    if (m0 < 0 || m1 - m0 != (int64_t)E.n * E.n || m1 > b.mat_total) return false;
    E.mat0 = m0;
  } else {
    E.mat0 = -1;
  }
  if (b.rhs_off) {
    const int64_t r0 = b.rhs_off[e], r1 = b.rhs_off[e + 1];
    if (r0 < 0 || r1 - r0 != (int64_t)E.n * E.r || r1 > b.rhs_total) return false;
    E.rhs0 = r0;
  } else {
    E.rhs0 = -1;
  }
  if (b.node_off) {
    const int64_t n0 = b.node_off[e], n1 = b.node_off[e + 1];
    if (n0 < 0 || n1 - n0 != (int64_t)E.n || n1 > b.node_total) return false;
    E.node0 = n0;
  } else {
    E.node0 = -1;
  }
  double v[6];
  for (int k = 0; k < 6; ++k) v[k] = b.vert[6 * (int64_t)e + k];
  for (int k = 0; k < 3; ++k) {
    const int sg = b.sigma[3 * (int64_t)e + k];
    const int fl = b.flip[3 * (int64_t)e + k];
    if ((sg != 1 && sg != -1) || (fl != 0 && fl != 1)) return false;
    E.sigma[k] = sg;
    E.flip[k] = fl;
  }
  const double cross = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
  if (!(cross > 0.0)) return false;
  E.area = 0.5 * cross;
  // D_a: edge opposite vertex a; gradient of the barycentric coordinate of
  // vertex a is rot(D_a) / (2|K|), so every sub-triangle (a translate or a
  // point reflection of K scaled by 1/s) has stiffness kappa D_a.D_b/(4|K|).
  const double D[3][2] = {{v[4] - v[2], v[5] - v[3]}, {v[0] - v[4], v[1] - v[5]}, {v[2] - v[0], v[3] - v[1]}};
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) E.G[a][c] = (D[a][0] * D[c][0] + D[a][1] * D[c][1]) / (4.0 * E.area);
  // face e is the edge opposite vertex e, i.e. D_e
  for (int k = 0; k < 3; ++k) E.flen[k] = sqrt(D[k][0] * D[k][0] + D[k][1] * D[k][1]);
  E.cunit = E.area / (3.0 * s * s);
  E.inv_area = 1.0 / E.area;
  E.inv_s = 1.0 / s;
  return true;
}

// The 7-point stencil of row/column (i,j) of A (P1 stiffness, kappa constant per
// sub-triangle).  Off-diagonal neighbours: E (i+1,j), W (i-1,j), N (i,j+1),
// S (i,j-1), NW (i-1,j+1), SE (i+1,j-1).  `cnt` counts the sub-triangles around
// the node (1 at a corner, 3 on an edge, 6 inside).
struct Stencil {
  double d, e, w, n, so, nw, se;
  int cnt;
};

template <class KAP>
__device__ __forceinline__ Stencil stencil(int i, int j, int s, const double (&G)[3][3], KAP kap) {
  Stencil st = {0, 0, 0, 0, 0, 0, 0, 0};
  const int ij = i + j;
  if (ij <= s - 1) {  // up (i,j): (i,j)=0, (i+1,j)=1, (i,j+1)=2
    const double k = kap(tri_up(i, j, s));
    st.d += k * G[0][0]; st.e += k * G[0][1]; st.n += k * G[0][2]; st.cnt++;
  }
  if (i >= 1 && ij <= s) {  // up (i-1,j): (i-1,j)=0, (i,j)=1, (i-1,j+1)=2
    const double k = kap(tri_up(i - 1, j, s));
    st.d += k * G[1][1]; st.w += k * G[0][1]; st.nw += k * G[1][2]; st.cnt++;
  }
  if (j >= 1 && ij <= s) {  // up (i,j-1): (i,j-1)=0, (i+1,j-1)=1, (i,j)=2
    const double k = kap(tri_up(i, j - 1, s));
    st.d += k * G[2][2]; st.so += k * G[0][2]; st.se += k * G[1][2]; st.cnt++;
  }
  if (i >= 1 && j >= 1 && ij <= s) {  // down (i-1,j-1): (i,j)=0, (i-1,j)=1, (i,j-1)=2
    const double k = kap(tri_dn(i - 1, j - 1, s));
    st.d += k * G[0][0]; st.w += k * G[0][1]; st.so += k * G[0][2]; st.cnt++;
  }
  if (i >= 1 && ij <= s - 1) {  // down (i-1,j): (i,j+1)=0, (i-1,j+1)=1, (i,j)=2
    const double k = kap(tri_dn(i - 1, j, s));
    st.d += k * G[2][2]; st.n += k * G[0][2]; st.nw += k * G[1][2]; st.cnt++;
  }
  if (j >= 1 && ij <= s - 1) {  // down (i,j-1): (i+1,j)=0, (i,j)=1, (i+1,j-1)=2
    const double k = kap(tri_dn(i, j - 1, s));
    st.d += k * G[1][1]; st.e += k * G[0][1]; st.se += k * G[1][2]; st.cnt++;
  }
  return st;
}

// Number of sub-triangles around node (i,j): the closed form of c_j / (|K|/(3s^2)).
__device__ __forceinline__ int node_tri_count(int i, int j, int s) {
  const int ij = i + j;
  int c = 0;
  c += (ij <= s - 1);
  c += (i >= 1 && ij <= s);
  c += (j >= 1 && ij <= s);
  c += (i >= 1 && j >= 1 && ij <= s);
  c += (i >= 1 && ij <= s - 1);
  c += (j >= 1 && ij <= s - 1);
  return c;
}

// Legendre polynomial P_q(t), q <= 4.
__device__ __forceinline__ double legendre(int q, double t) {
  double p0 = 1.0, p1 = t;
  if (q == 0) return p0;
  for (int k = 1; k < q; ++k) {
    const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// R[node at position k of face e][column e(l+1)+q] = -sigma_e (P_q, phi)_{F_e}:
// exact for q <= 4 with the 3-point Gauss rule on each of the s face segments.
// Face load of face DoF a at lattice position k (0..s) of its face:
// -sigma_e times the integral of psi_a phi_k over the face (eq. (9)).  DoF
// a = (e m + seg)(l + 1) + q is P_q(t) on segment seg of the m-partition of
// face e; segments and t in [-1, 1] run along the global orientation (from
// the lower global vertex id), so with the global face parameter g = tau
// (or 1 - tau when flip[e]), t = 2 (m g - seg) - 1.  Each sub-edge lies in one
// segment (m divides s); 3-point Gauss on each sub-edge is exact (degree
// q + 1 <= 5).
__device__ __forceinline__ double face_load(const Elem& E, int a, int k) {
  const double r15 = 0.38729833462074168852;  // sqrt(15)/10
  const double xg[3] = {0.5 - r15, 0.5, 0.5 + r15};
  const double wg[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  const int s = E.s, lp1 = E.l + 1;
  const int e = a / E.P, rem = a - e * E.P;
  const int segf = rem / lp1, q = rem - segf * lp1;
  const int per = s / E.m;                    // sub-edges per segment
  const bool fl = E.flip[e] != 0;
  double acc = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int seg = side == 0 ? k - 1 : k;   // node k is the right end of sub-edge k-1, left end of k
    if (seg < 0 || seg >= s) continue;
    if ((fl ? s - 1 - seg : seg) / per != segf) continue;
    for (int g = 0; g < 3; ++g) {
      const double tau = (seg + xg[g]) * E.inv_s;
      const double gp = fl ? 1.0 - tau : tau;
      const double t = 2.0 * (E.m * gp - segf) - 1.0;
      const double hat = side == 0 ? xg[g] : 1.0 - xg[g];
      acc += wg[g] * legendre(q, t) * hat;
    }
  }
  return -(double)E.sigma[e] * E.flen[e] * E.inv_s * acc;
}

// Lattice node at position k (0..s) along face e, from v[e+1] to v[e+2].
__device__ __forceinline__ int face_node(int e, int k, int s) {
  if (e == 0) return node_idx(s - k, k, s);
  if (e == 1) return node_idx(0, s - k, s);
  return node_idx(k, 0, s);
}

// Position of lattice node (i,j) on face e, or -1.
__device__ __forceinline__ int face_pos(int e, int i, int j, int s) {
  if (e == 0) return (i + j == s) ? j : -1;
  if (e == 1) return (i == 0) ? s - j : -1;
  return (j == 0) ? i : -1;
}

// ------------------------------------------------- FP64 refinement criterion
// The forward error of a plain FP64 Cholesky solve of Ahat grows like its
// condition number, roughly (max K / min K) s^2 (times a constant of the
// element's shape): well below 1e-13 on smooth fields (contrast up to a few
// hundred), but about 1e-10 for a contrast of 1e4 at s = 32.  Elements above
// this bound get one refinement step with a double-double residual in the
// FP64 path.
constexpr double REFINE64_SCALE = 1048576.0;   // 2^20: contrast 1024 at s = 32, 455 at s = 48

// mode > 0: every element, mode < 0: none, 0: contrast s^2 above the bound.
// Called by every thread of the block (two barriers); `red` holds one double
// per wave.
__device__ __forceinline__ bool refine64_needed(int mode, const double* kap, int s, double* red) {
  if (mode != 0) return mode > 0;
  double kmax = 0.0, kinv = 0.0;
  for (int t = threadIdx.x; t < s * s; t += blockDim.x) {
    const double k = kap[t];
    kmax = fmax(kmax, k);
    kinv = fmax(kinv, 1.0 / k);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    kmax = fmax(kmax, __shfl_xor(kmax, o, 64));
    kinv = fmax(kinv, __shfl_xor(kinv, o, 64));
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = kmax * kinv;
  __syncthreads();
  double con = red[0];
  for (int k = 1; k < nw; ++k) con = fmax(con, red[k]);
  // a NaN or infinite contrast (bad coefficients) also takes the refinement
  return !(con * ((double)s * s) <= REFINE64_SCALE);
}

// Double-double accumulation (error-free transformations; contraction off
// so that the error terms are exact): (hi, lo) += a b.
__device__ __forceinline__ void dd_add_prod(double& hi, double& lo, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double pe = __builtin_fma(a, b, -p);
  const double t = hi + p;
  const double bb = t - hi;
  const double e = (hi - (t - bb)) + (p - bb);
  hi = t;
  lo += e + pe;
}
// b - (hi + lo), rounded once more to double.
__device__ __forceinline__ double dd_sub_from(double b, double hi, double lo) {
#pragma clang fp contract(off)
  const double t = b - hi;
  const double bb = t - b;
  const double e = (b - (t - bb)) + (-hi - bb);
  return t + (e - lo);
}

// ------------------------------------------------------------------ MFMA tiles
// Result layout of v_mfma_*_16x16x4 (one block): lane l holds column l%16 and
// four rows, item v = 0..3.  For f32 they are rows 4*(l/16)+v; for f64 the
// rows are interleaved, row (l/16)+4v.  row(g, v) gives the row of item v in
// lane group g = l/16; grp(r), item(r) invert it.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // c - a b: on gfx950 the last immediate of the FP64 instruction is its
  // negate modifier (bit 0: operand A), so the sign costs no instruction
  static __device__ __forceinline__ v4 op_sub(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
  }
  static __host__ __device__ constexpr int row(int g, int v) { return g + 4 * v; }
  static __host__ __device__ constexpr int grp(int r) { return r & 3; }
  static __host__ __device__ constexpr int item(int r) { return r >> 2; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ v4 op_sub(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int row(int g, int v) { return 4 * g + v; }
  static __host__ __device__ constexpr int grp(int r) { return r >> 2; }
  static __host__ __device__ constexpr int item(int r) { return r & 3; }
};

// A stored 16x16 tile is row-major with a padded row stride so that the 16
// rows read by one MFMA operand load fall in distinct LDS banks.
constexpr int TST = 17;
constexpr int TILE = 16 * TST;

// Operand layouts of v_mfma_*_16x16x4 (one block): lane l supplies
//   A[l%16][l/16]   (16x4 chunk of A),   B[l/16][l%16]   (4x16 chunk of B).
template <typename T>
__device__ __forceinline__ T ld_rowcol(const T* t, int c, int lane) {  // t[l%16][4c + l/16]
  return t[(lane & 15) * TST + 4 * c + (lane >> 4)];
}
template <typename T>
__device__ __forceinline__ T ld_colrow(const T* t, int c, int lane) {  // t[4c + l/16][l%16]
  return t[(4 * c + (lane >> 4)) * TST + (lane & 15)];
}
template <typename T>
__device__ __forceinline__ typename Mfma<T>::v4 ld_acc(const T* t, int lane) {
  typename Mfma<T>::v4 a;
  const int cc = lane & 15, g = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) a[v] = t[Mfma<T>::row(g, v) * TST + cc];
  return a;
}
template <typename T>
__device__ __forceinline__ void st_acc(T* t, const typename Mfma<T>::v4& a, int lane) {
  const int cc = lane & 15, g = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) t[Mfma<T>::row(g, v) * TST + cc] = a[v];
}

// acc -= X * Y^T   (X, Y stored tiles)
template <typename T>
__device__ __forceinline__ void mma_sub_nt(typename Mfma<T>::v4& acc, const T* X, const T* Y, int lane) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc = Mfma<T>::op(-ld_rowcol(X, c, lane), ld_rowcol(Y, c, lane), acc);
}
// acc -= X * Y     (X, Y stored tiles)
template <typename T>
__device__ __forceinline__ void mma_sub_nn(typename Mfma<T>::v4& acc, const T* X, const T* Y, int lane) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc = Mfma<T>::op(-ld_rowcol(X, c, lane), ld_colrow(Y, c, lane), acc);
}
// acc += X * Y^T
template <typename T>
__device__ __forceinline__ void mma_add_nt(typename Mfma<T>::v4& acc, const T* X, const T* Y, int lane) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc = Mfma<T>::op(ld_rowcol(X, c, lane), ld_rowcol(Y, c, lane), acc);
}
// acc += X * Y
template <typename T>
__device__ __forceinline__ void mma_add_nn(typename Mfma<T>::v4& acc, const T* X, const T* Y, int lane) {
#pragma unroll
  for (int c = 0; c < 4; ++c) acc = Mfma<T>::op(ld_rowcol(X, c, lane), ld_colrow(Y, c, lane), acc);
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, 64);
}

}  // namespace mhm
