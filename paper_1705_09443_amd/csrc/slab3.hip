// The 3D sparsified system and moving-PML sweep (Sec. 3.1; Sec. 2.2 and 2.3
// with d = 3).
//
// Stencils: 27-point neighbourhood mu = {-1,0,1}^3, neighbour index
// o = 9 (d1+1) + 3 (d2+1) + (d3+1). Rows of H at I^h = [0, n+1]^3 use
// conj(alpha_o) + omega^2 conj(beta_o) m_{i+o}; PML rows use conj(gamma_i,o)
// by per-axis class; auxiliary-PML rows of a slab use the gamma of their
// depth, transverse classes and sampled local frequency.
//
// Slabs: the subproblem of slab k lives on t lines [first, hi] (b auxiliary
// lines, then the lines of D_k) times the L x L transverse points. Ordered by
// the transverse index e2 it is block tridiagonal,
//     B_j x_{j-1} + A_j x_j + C_j x_{j+1} = r_j,
// with blocks of nb = t L unknowns (a, e3), index a L + e3, each block row
// holding at most 9 entries per row (offsets d1, d3). Block elimination
//     S_0 = A_0,  S_j = A_j - B_j S_{j-1}^{-1} C_{j-1}
// is done in float64 for all slabs at once; S_j^{-1} is formed by blocked
// in-place Gauss-Jordan with partial pivoting (32-column panels) and kept
// (cast to the working precision) as the factor F_j. A slab solve is
//     y_j = F_j (r_j - B_j y_{j-1}),  x_{L-1} = y_{L-1},
//     x_j = y_j - F_j (C_j x_{j+1}),
// one dense matrix-vector product per block and direction.
#include "kernels.hpp"

namespace lsw {

namespace {

__device__ inline int class3(int i, int n, int b) {
  if (i < 0) return i + b + 1;
  if (i > n + 1) return i - (n + 2) + b + 1;
  return 0;
}

__device__ inline double2 dconj(double2 v) { return make_double2(v.x, -v.y); }

// Coefficient of H in the row of grid point (i1, i2, i3) for neighbour o.
__device__ double2 h3_coef(const Stencil3& S, int i1, int i2, int i3, int o) {
  const int n = S.n;
  if (i1 >= 0 && i1 <= n + 1 && i2 >= 0 && i2 <= n + 1 && i3 >= 0 && i3 <= n + 1) {
    const int j1 = i1 + o / 9 - 1, j2 = i2 + (o / 3) % 3 - 1, j3 = i3 + o % 3 - 1;
    double mm = 0.0;
    if (j1 >= 1 && j1 <= n && j2 >= 1 && j2 <= n && j3 >= 1 && j3 <= n)
      mm = S.m[((size_t)(j1 - 1) * n + (j2 - 1)) * n + (j3 - 1)];
    const double2 al = S.alpha[o], be = S.beta[o];
    return make_double2(al.x + S.omega2 * be.x * mm, -al.y - S.omega2 * be.y * mm);
  }
  const int NC = 2 * S.b + 1;
  const int c1 = class3(i1, n, S.b), c2 = class3(i2, n, S.b), c3 = class3(i3, n, S.b);
  return dconj(S.gglob[(((size_t)c1 * NC + c2) * NC + c3) * 27 + o]);
}

// Coefficient of the subproblem of slab p in the row of local point
// (a, e2, e3) for neighbour o; zero where the neighbour lies outside the
// subproblem (Dirichlet line left of the auxiliary PML, D_{k+1}, or beyond
// the extended grid).
__device__ double2 sub3_coef(const Stencil3& S, const Slab3& p, int a, int e2, int e3, int o) {
  const int L = S.L, b = S.b;
  const int a2 = a + o / 9 - 1, f2 = e2 + (o / 3) % 3 - 1, f3 = e3 + o % 3 - 1;
  if (a2 < 0 || a2 >= p.t || f2 < 0 || f2 >= L || f3 < 0 || f3 >= L) return make_double2(0.0, 0.0);
  const int line = p.first + a;
  if (a < p.naux) {
    const int q = p.lo - 1 - line;
    const int ks = S.kmap[((size_t)(line + b) * L + e2) * L + e3];
    const int NC = 2 * b + 1;
    const int c2 = class3(e2 - b, S.n, b), c3 = class3(e3 - b, S.n, b);
    return dconj(S.gaux[((((size_t)q * NC + c2) * NC + c3) * S.ns + ks) * 27 + o]);
  }
  return h3_coef(S, line, e2 - b, e3 - b, o);
}

__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- stencil applies ---------------------------------------------------------

// f = Q r on the extended cube: alpha^* r_{mu_i} on I^h, zero on the PML
template <typename T>
__global__ void k3_apply_Q(Stencil3 S, const C<T>* __restrict__ r, int nrhs, C<T>* __restrict__ f) {
  const int L = S.L, n = S.n, b = S.b;
  const size_t E = (size_t)L * L * L;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * nrhs) return;
  const size_t rhs = idx / E, e = idx % E;
  const int i1 = (int)(e / ((size_t)L * L)) - b, i2 = (int)((e / L) % L) - b, i3 = (int)(e % L) - b;
  C<T> acc = mk<T>(0, 0);
  if (i1 >= 0 && i1 <= n + 1 && i2 >= 0 && i2 <= n + 1 && i3 >= 0 && i3 <= n + 1) {
    const C<T>* rr = r + rhs * (size_t)n * n * n;
    for (int o = 0; o < 27; ++o) {
      const int j1 = i1 + o / 9 - 1, j2 = i2 + (o / 3) % 3 - 1, j3 = i3 + o % 3 - 1;
      if (j1 < 1 || j1 > n || j2 < 1 || j2 > n || j3 < 1 || j3 > n) continue;
      const double2 al = S.alpha[o];
      const C<T> c = mk<T>((T)al.x, (T)(-al.y));
      acc = cadd<T>(acc, cmul<T>(c, rr[((size_t)(j1 - 1) * n + (j2 - 1)) * n + (j3 - 1)]));
    }
  }
  f[idx] = acc;
}

// y = H u on the extended cube (Dirichlet ring dropped)
template <typename T>
__global__ void k3_apply_H(Stencil3 S, const C<T>* __restrict__ u, int nrhs, C<T>* __restrict__ y) {
  const int L = S.L, b = S.b;
  const size_t E = (size_t)L * L * L;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * nrhs) return;
  const size_t rhs = idx / E, e = idx % E;
  const int e1 = (int)(e / ((size_t)L * L)), e2 = (int)((e / L) % L), e3 = (int)(e % L);
  const C<T>* uu = u + rhs * E;
  C<T> acc = mk<T>(0, 0);
  for (int o = 0; o < 27; ++o) {
    const int f1 = e1 + o / 9 - 1, f2 = e2 + (o / 3) % 3 - 1, f3 = e3 + o % 3 - 1;
    if (f1 < 0 || f1 >= L || f2 < 0 || f2 >= L || f3 < 0 || f3 >= L) continue;
    const double2 c = h3_coef(S, e1 - b, e2 - b, e3 - b, o);
    acc = cadd<T>(acc, cmul<T>(mk<T>((T)c.x, (T)c.y), uu[((size_t)f1 * L + f2) * L + f3]));
  }
  y[idx] = acc;
}

// z = u restricted to the interior grid I
template <typename T>
__global__ void k3_extract(const C<T>* __restrict__ u, int n, int b, int nrhs, C<T>* __restrict__ z) {
  const int L = n + 2 + 2 * b;
  const size_t N = (size_t)n * n * n;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nrhs) return;
  const size_t rhs = idx / N, i = idx % N;
  const int i1 = (int)(i / ((size_t)n * n)) + 1, i2 = (int)((i / n) % n) + 1, i3 = (int)(i % n) + 1;
  z[idx] = u[rhs * (size_t)L * L * L + ((size_t)(i1 + b) * L + (i2 + b)) * L + (i3 + b)];
}

// ---- factorization (float64, two chains per slab, all slabs at once) ----
//
// Two-ended block elimination: for the middle block m = L/2 the top chain
// eliminates blocks 0 .. m-1 downwards (S_j = A_j - B_j S_{j-1}^{-1} C_{j-1}),
// the bottom chain blocks L-1 .. m+1 upwards (S_j = A_j - C_j S_{j+1}^{-1}
// B_{j+1}), and the middle block takes both Schur terms. Work entry e is the
// top (dir = +1) or bottom (dir = -1) chain of a slab; blockIdx.z selects the
// entry estride z + eoff.
struct ChainStep {
  int s;        // chain step: top chains take block s, bottom chains L - 1 - s
  int m;        // middle block
  int middle;   // 1: every entry takes the middle block m
  int estride;  // entry = blockIdx.z * estride + eoff
  int eoff;
};

__device__ inline int cs_entry(const ChainStep& cs) { return blockIdx.z * cs.estride + cs.eoff; }

// block of the entry at this step; false when its chain is done
__device__ inline bool cs_block(const ChainStep& cs, int dir, int L, int* j) {
  if (cs.middle) {
    *j = cs.m;
    return true;
  }
  if (dir > 0) {
    *j = cs.s;
    return cs.s < cs.m;
  }
  *j = L - 1 - cs.s;
  return cs.s < L - 1 - cs.m;
}

__device__ inline bool cs_has_prev(const ChainStep& cs) { return cs.middle || cs.s > 0; }

// cf[0]: A_j (d2 = 0); cf[1]: the rows of block j at d2 = -dir (coupling to
// the chain's previous block j - dir); cf[2]: the rows of block j - dir at
// d2 = +dir (coupling back to j); each [nb][9] by (d1, d3)
__global__ void k3_coefs(Stencil3 S, const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works,
                         ChainStep cs) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int j;
  if (!cs_block(cs, w.dir, S.L, &j)) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.nb * 9) return;
  const int r = idx / 9, o9 = idx % 9, a = r / S.L, e3 = r % S.L;
  const int d1 = o9 / 3 - 1, d3 = o9 % 3 - 1;
  const size_t s3 = (size_t)p.nb * 9;
  w.cf[idx] = sub3_coef(S, p, a, j, e3, (d1 + 1) * 9 + 3 + (d3 + 1));
  const double2 zero = make_double2(0.0, 0.0);
  const bool prev = cs_has_prev(cs);
  w.cf[s3 + idx] = prev ? sub3_coef(S, p, a, j, e3, (d1 + 1) * 9 + (1 - w.dir) * 3 + (d3 + 1)) : zero;
  w.cf[2 * s3 + idx] = prev ? sub3_coef(S, p, a, j - w.dir, e3, (d1 + 1) * 9 + (1 + w.dir) * 3 + (d3 + 1)) : zero;
}

// W = Sp cf2: column c = (a, e3) of the coupling back to j has its entries in
// rows (a - d1, e3 - d3) of the previous block, coefficient cf[2][row][(d1, d3)]
__global__ void k3_schur_w(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L,
                           ChainStep cs) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int j;
  if (!cs_block(cs, w.dir, L, &j) || !cs_has_prev(cs)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= p.nb || r >= p.nb) return;
  const int a = c / L, e3 = c % L;
  const double2* cc = w.cf + 2 * (size_t)p.nb * 9;
  const double2* sp = w.Sp + (size_t)r * p.nb;
  double2 acc = make_double2(0.0, 0.0);
  for (int o9 = 0; o9 < 9; ++o9) {
    const int a2 = a - (o9 / 3 - 1), f3 = e3 - (o9 % 3 - 1);
    if (a2 < 0 || a2 >= p.t || f3 < 0 || f3 >= L) continue;
    const int rr = a2 * L + f3;
    const double2 v = zmul(sp[rr], cc[(size_t)rr * 9 + o9]);
    acc.x += v.x;
    acc.y += v.y;
  }
  w.W[(size_t)r * p.nb + c] = acc;
}

// S = A_j - cf1 W (with a previous block) or A_j; row r = (a, e3) of the
// coupling cf1 has its entries in rows (a + d1, e3 + d3) of W
__global__ void k3_schur_s(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L,
                           ChainStep cs) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int j;
  if (!cs_block(cs, w.dir, L, &j)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= p.nb || r >= p.nb) return;
  const int a = r / L, e3 = r % L, ca = c / L, c3 = c % L;
  double2 v = make_double2(0.0, 0.0);
  const int d1 = ca - a, d3 = c3 - e3;
  if (d1 >= -1 && d1 <= 1 && d3 >= -1 && d3 <= 1) v = w.cf[(size_t)r * 9 + (d1 + 1) * 3 + (d3 + 1)];
  if (cs_has_prev(cs)) {
    const double2* cb = w.cf + (size_t)p.nb * 9 + (size_t)r * 9;
    for (int o9 = 0; o9 < 9; ++o9) {
      const int a2 = a + o9 / 3 - 1, f3 = e3 + o9 % 3 - 1;
      if (a2 < 0 || a2 >= p.t || f3 < 0 || f3 >= L) continue;
      const double2 t = zmul(cb[o9], w.W[(size_t)(a2 * L + f3) * p.nb + c]);
      v.x -= t.x;
      v.y -= t.y;
    }
  }
  w.S[(size_t)r * p.nb + c] = v;
}

// middle block: S -= cf1 W of the partner entry (the slab's bottom chain,
// entry e + 1): the second Schur term C_m S_{m+1}^{-1} B_{m+1}
__global__ void k3_schur_sub(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L,
                             ChainStep cs) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e], v2 = works[e + 1];
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= p.nb || r >= p.nb) return;
  const int a = r / L, e3 = r % L;
  const double2* cb = v2.cf + (size_t)p.nb * 9 + (size_t)r * 9;
  double2 v = w.S[(size_t)r * p.nb + c];
  for (int o9 = 0; o9 < 9; ++o9) {
    const int a2 = a + o9 / 3 - 1, f3 = e3 + o9 % 3 - 1;
    if (a2 < 0 || a2 >= p.t || f3 < 0 || f3 >= L) continue;
    const double2 t = zmul(cb[o9], v2.W[(size_t)(a2 * L + f3) * p.nb + c]);
    v.x -= t.x;
    v.y -= t.y;
  }
  w.S[(size_t)r * p.nb + c] = v;
}

// Gauss-Jordan on the panel columns [k0, k0 + kp) of S, pivots k0..k0+kp-1
// chosen by partial pivoting over the rows not yet used; every row swap is
// recorded in piv and applied to the other columns by k3_gj_swap.
constexpr int kGjPanel = 32;
constexpr int kGjThreads = 512;

// Largest candidate (modulus squared bv at row br) over the workgroup, the
// first row on ties; every thread gets the row.
__device__ int gj_pick(double bv, int br, double* best_v, int* best_r, int* pick) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int orr = __shfl_xor(br, off);
    if (ov > bv || (ov == bv && orr < br)) {
      bv = ov;
      br = orr;
    }
  }
  if (lane == 0) {
    best_v[wid] = bv;
    best_r[wid] = br;
  }
  __syncthreads();
  if (tid == 0) {
    double v = best_v[0];
    int rr = best_r[0];
    for (int q = 1; q < kGjThreads / 64; ++q)
      if (best_v[q] > v || (best_v[q] == v && best_r[q] < rr)) {
        v = best_v[q];
        rr = best_r[q];
      }
    *pick = rr;
  }
  __syncthreads();
  return *pick;
}

// Sub-panel width whose nb x width complex128 columns fit in LDS (150 KB).
__host__ __device__ inline int gj_subpanel(int nb) { return nb <= 2400 ? 4 : 2; }
constexpr size_t kGjLdsBytes = 150 * 1024;

// The panel is worked through in sub-panels of SW columns, each held in LDS
// for all nb rows: its pivots are found, swapped and eliminated there (the
// same in-place Gauss-Jordan steps), it is written back, and its row
// interchanges and rank-SW transform are applied to the panel's other
// columns in global memory before the next sub-panel is loaded.
template <int SW>
__global__ __launch_bounds__(kGjThreads) void k3_gj_panel(const Slab3* __restrict__ slabs,
                                                          const Slab3Work* __restrict__ works, int L, ChainStep cs,
                                                          int k0, int* __restrict__ status) {
  constexpr int RU = 8;  // rows in flight per thread in the global update
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int jb;
  if (!cs_block(cs, w.dir, L, &jb)) return;
  const int nb = p.nb;
  if (k0 >= nb || gj_subpanel(nb) != SW) return;
  const int kp = min(kGjPanel, nb - k0);
  const int tid = threadIdx.x;
  extern __shared__ unsigned char smem_raw[];
  double2* buf = reinterpret_cast<double2*>(smem_raw);  // [nb][SW]
  __shared__ double best_v[kGjThreads / 64];
  __shared__ int best_r[kGjThreads / 64];
  __shared__ int pick_s;
  __shared__ double2 prow[SW];
  __shared__ double2 rk[SW][kGjPanel];
  __shared__ int spiv[SW];
  double2* S = w.S;
  for (int c0 = k0; c0 < k0 + kp; c0 += SW) {
    const int sw = min(SW, k0 + kp - c0);
    // 1. the sub-panel columns into LDS
    for (int idx = tid; idx < nb * SW; idx += kGjThreads) {
      const int r = idx / SW, q = idx % SW;
      buf[idx] = q < sw ? S[(size_t)r * nb + c0 + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // 2. its pivots, in LDS
    for (int pp = 0; pp < sw; ++pp) {
      const int cp = c0 + pp;
      double bv = -1.0;
      int br = nb;
      for (int r = cp + tid; r < nb; r += kGjThreads) {
        const double2 v = buf[r * SW + pp];
        const double m2 = v.x * v.x + v.y * v.y;
        if (m2 > bv) {
          bv = m2;
          br = r;
        }
      }
      int pr = gj_pick(bv, br, best_v, best_r, &pick_s);
      if (pr >= nb) pr = cp;
      if (tid == 0) {
        w.piv[cp] = pr;
        spiv[pp] = pr;
      }
      if (pr != cp && tid < SW) {
        const double2 a = buf[cp * SW + tid], b = buf[pr * SW + tid];
        buf[cp * SW + tid] = b;
        buf[pr * SW + tid] = a;
      }
      __syncthreads();
      if (tid < SW) {
        const double2 pv = buf[cp * SW + pp];
        const double d = pv.x * pv.x + pv.y * pv.y;
        double2 inv = make_double2(0.0, 0.0);
        if (!(d > 0.0) || !(d < INFINITY)) {
          if (tid == 0) atomicMax(status, e / 2 + 1);
        } else {
          inv = make_double2(pv.x / d, -pv.y / d);
        }
        prow[tid] = tid == pp ? inv : zmul(buf[cp * SW + tid], inv);
      }
      __syncthreads();
      if (tid < SW) buf[cp * SW + tid] = prow[tid];
      // eliminate column cp from every other row; the SW entries of a row
      // share a wave, which reads the row's column-cp entry before lane pp
      // overwrites it
      for (int idx = tid; idx < nb * SW; idx += kGjThreads) {
        const int r = idx / SW, q = idx % SW;
        if (r == cp) continue;
        const double2 f = buf[r * SW + pp];
        double2 v = q == pp ? make_double2(0.0, 0.0) : buf[idx];
        const double2 t = zmul(f, prow[q]);
        v.x -= t.x;
        v.y -= t.y;
        buf[idx] = v;
      }
      __syncthreads();
    }
    // 3. back to global memory
    for (int idx = tid; idx < nb * SW; idx += kGjThreads) {
      const int r = idx / SW, q = idx % SW;
      if (q < sw) S[(size_t)r * nb + c0 + q] = buf[idx];
    }
    // 4. the other panel columns: interchanges in order, then
    //    M[:, c] += X M[Ksub, c] with X = the sub-panel minus the identity on
    //    its pivot rows
    if (tid < kp && (k0 + tid < c0 || k0 + tid >= c0 + sw)) {
      const int c = k0 + tid;
      for (int q = 0; q < sw; ++q) {
        const int r1 = c0 + q, r2 = spiv[q];
        if (r2 != r1) {
          const double2 a = S[(size_t)r1 * nb + c], b = S[(size_t)r2 * nb + c];
          S[(size_t)r1 * nb + c] = b;
          S[(size_t)r2 * nb + c] = a;
        }
      }
      for (int q = 0; q < sw; ++q) rk[q][tid] = S[(size_t)(c0 + q) * nb + c];
    }
    __syncthreads();
    {
      const int c = tid % kGjPanel, rg = tid / kGjPanel;
      constexpr int RG = kGjThreads / kGjPanel;
      const bool col = c < kp && (k0 + c < c0 || k0 + c >= c0 + sw);
      if (col) {
        for (int rb = rg; rb < nb; rb += RG * RU) {
          double2 v[RU];
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int r = rb + RG * u;
            v[u] = r < nb ? S[(size_t)r * nb + k0 + c] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int r = rb + RG * u;
            if (r >= nb) continue;
            double2 acc = v[u];
            for (int q = 0; q < sw; ++q) {
              double2 x = buf[r * SW + q];
              if (r == c0 + q) x.x -= 1.0;
              const double2 t = zmul(x, rk[q][c]);
              acc.x += t.x;
              acc.y += t.y;
            }
            S[(size_t)r * nb + k0 + c] = acc;
          }
        }
      }
    }
    __syncthreads();
  }
}

// The panel's row swaps applied, in order, to every column outside the
// panel; the pivot rows of those columns copied to Xr [kp][nb]
__global__ void k3_gj_swap(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L, ChainStep cs,
                           int k0) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int jb;
  if (!cs_block(cs, w.dir, L, &jb)) return;
  const int nb = p.nb;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (k0 >= nb || c >= nb) return;
  const int kp = min(kGjPanel, nb - k0);
  if (c >= k0 && c < k0 + kp) return;
  double2* S = w.S;
  for (int q = 0; q < kp; ++q) {
    const int r1 = k0 + q, r2 = w.piv[r1];
    if (r2 != r1) {
      const double2 a = S[(size_t)r1 * nb + c], b = S[(size_t)r2 * nb + c];
      S[(size_t)r1 * nb + c] = b;
      S[(size_t)r2 * nb + c] = a;
    }
  }
  for (int q = 0; q < kp; ++q) w.Xr[(size_t)q * nb + c] = S[(size_t)(k0 + q) * nb + c];
}

// S[:, c] += X Xr[:, c] for columns c outside the panel, X = S[:, panel]
// minus the identity on the pivot rows: 64 x 64 tiles, 256 threads, each
// thread 4 x 4 entries (rows ty + 16 i, columns tx + 16 q)
__global__ __launch_bounds__(256) void k3_gj_update(const Slab3* __restrict__ slabs,
                                                    const Slab3Work* __restrict__ works, int L, ChainStep cs,
                                                    int k0) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int jb;
  if (!cs_block(cs, w.dir, L, &jb)) return;
  const int nb = p.nb;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  if (k0 >= nb || r0 >= nb || c0 >= nb) return;
  const int kp = min(kGjPanel, nb - k0);
  if (c0 >= k0 && c0 + 64 <= k0 + kp) return;  // the whole tile is panel columns
  __shared__ double2 Xs[kGjPanel][64];  // X tile, k-major
  __shared__ double2 Rs[kGjPanel][64];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double2* S = w.S;
  for (int idx = tid; idx < 64 * kGjPanel; idx += 256) {
    const int rr = idx / kGjPanel, q = idx % kGjPanel, r = r0 + rr;
    double2 v = make_double2(0.0, 0.0);
    if (r < nb && q < kp) {
      v = S[(size_t)r * nb + k0 + q];
      if (r == k0 + q) v.x -= 1.0;
    }
    Xs[q][rr] = v;
  }
  for (int idx = tid; idx < kGjPanel * 64; idx += 256) {
    const int q = idx / 64, cc = idx % 64, c = c0 + cc;
    Rs[q][cc] = (q < kp && c < nb) ? w.Xr[(size_t)q * nb + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = make_double2(0.0, 0.0);
  for (int k = 0; k < kp; ++k) {
    double2 xa[4], rb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) xa[i] = Xs[k][ty + 16 * i];
#pragma unroll
    for (int q = 0; q < 4; ++q) rb[q] = Rs[k][tx + 16 * q];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[i][q].x += xa[i].x * rb[q].x - xa[i].y * rb[q].y;
        acc[i][q].y += xa[i].x * rb[q].y + xa[i].y * rb[q].x;
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty + 16 * i;
    if (r >= nb) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c0 + tx + 16 * q;
      if (c >= nb || (c >= k0 && c < k0 + kp)) continue;
      double2 v = S[(size_t)r * nb + c];
      v.x += acc[i][q].x;
      v.y += acc[i][q].y;
      S[(size_t)r * nb + c] = v;
    }
  }
}

// Column order of the inverse: in-place Gauss-Jordan with row interchanges
// leaves S^{-1} with its columns permuted; replaying the interchanges in
// reverse on the index list gives perm, and S^{-1}[:, c] = S[:, perm[c]].
__global__ void k3_gj_perm(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L, ChainStep cs) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int jb;
  if (!cs_block(cs, w.dir, L, &jb) || threadIdx.x != 0) return;
  for (int c = 0; c < p.nb; ++c) w.perm[c] = c;
  for (int c = p.nb - 1; c >= 0; --c) {
    const int q = w.piv[c];
    const int t = w.perm[c];
    w.perm[c] = w.perm[q];
    w.perm[q] = t;
  }
}

// Sp = S^{-1} (float64, for the next block) and F_j = S^{-1} in the working precision
template <typename T>
__global__ void k3_gj_store(const Slab3* __restrict__ slabs, const Slab3Work* __restrict__ works, int L, ChainStep cs,
                            C<T>* const* __restrict__ factors) {
  const int e = cs_entry(cs);
  const Slab3 p = slabs[e];
  const Slab3Work w = works[e];
  int j;
  if (!cs_block(cs, w.dir, L, &j)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= p.nb || r >= p.nb) return;
  const double2 v = w.S[(size_t)r * p.nb + w.perm[c]];
  w.Sp[(size_t)r * p.nb + c] = v;
  factors[e][((size_t)j * p.nb + r) * p.nb + c] = mk<T>((T)v.x, (T)v.y);
}

// Apply-time coefficients of slab z: cbc [L][2][nb][9] (B_j, then C_j, by
// (d1, d3)), and the couplings to the neighbouring slabs: cm [L][L][9] from
// the rows of line lo to line lo - 1 (k > 0), cp from the rows of line hi to
// line hi + 1 (k < l - 1), by (d2, d3).
template <typename T>
__global__ void k3_apply_coefs(Stencil3 S, const Slab3* __restrict__ slabs, C<T>* const* __restrict__ cbc,
                               C<T>* const* __restrict__ cm, C<T>* const* __restrict__ cpl) {
  const Slab3 p = slabs[blockIdx.z];
  const int L = S.L, b = S.b;
  const size_t per = (size_t)p.nb * 9;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)L * 2 * per) {
    const int j = (int)(idx / (2 * per)), side = (int)((idx / per) % 2);
    const int r = (int)((idx % per) / 9), o9 = (int)(idx % 9);
    const int a = r / L, e3 = r % L;
    const double2 v = sub3_coef(S, p, a, j, e3, (o9 / 3) * 9 + (side ? 6 : 0) + o9 % 3);
    cbc[blockIdx.z][idx] = mk<T>((T)v.x, (T)v.y);
  }
  if (idx < (size_t)L * L * 9) {
    const int e2 = (int)(idx / ((size_t)L * 9)), e3 = (int)((idx / 9) % L), o9 = (int)(idx % 9);
    const int d2 = o9 / 3 - 1, d3 = o9 % 3 - 1;
    const bool in = e2 + d2 >= 0 && e2 + d2 < L && e3 + d3 >= 0 && e3 + d3 < L;
    if (cm[blockIdx.z]) {
      const double2 v = in ? h3_coef(S, p.lo, e2 - b, e3 - b, 0 * 9 + o9) : make_double2(0.0, 0.0);
      cm[blockIdx.z][idx] = mk<T>((T)v.x, (T)v.y);
    }
    if (cpl[blockIdx.z]) {
      const double2 v = in ? h3_coef(S, p.hi, e2 - b, e3 - b, 2 * 9 + o9) : make_double2(0.0, 0.0);
      cpl[blockIdx.z][idx] = mk<T>((T)v.x, (T)v.y);
    }
  }
}

// ---- slab solves -------------------------------------------------------------

// z_j = r_j - (B_j y_{j-1}) - (C_j y_{j+1}) for the blocks of one step (the
// terms each block takes are in st.terms; blockIdx.y = block of the step):
// r_j from the source lines (D part), minus the coupling to line lo - 1 on the
// first line of D (cmode 1), plus the coupling to line hi + 1 on the last line
// (cmode 2)
template <typename T>
__global__ void k3_zf(Slab3Apply<T> A, Slab3Step st) {
  const Slab3 p = A.p;
  const int L = A.L, nb = p.nb, task = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (task >= st.nt || idx >= nb * A.nrhs) return;
  const int j = st.j[task], terms = st.terms[task];
  const int rhs = idx / nb, c = idx % nb, a = c / L, e3 = c % L;
  C<T> v = mk<T>(0, 0);
  if (a >= p.naux && A.src) v = A.src[rhs * A.src_rs + ((size_t)(a - p.naux) * L + j) * L + e3];
  if ((A.cmode == 1 && a == p.naux) || (A.cmode == 2 && a == p.t - 1)) {
    const C<T>* cf = (A.cmode == 1 ? A.cm : A.cp) + ((size_t)j * L + e3) * 9;
    const C<T>* cu = A.cu + rhs * A.cu_rs;
    C<T> s = mk<T>(0, 0);
    for (int o9 = 0; o9 < 9; ++o9) {
      const int f2 = j + o9 / 3 - 1, f3 = e3 + o9 % 3 - 1;
      if (f2 < 0 || f2 >= L || f3 < 0 || f3 >= L) continue;
      s = cadd<T>(s, cmul<T>(cf[o9], cu[(size_t)f2 * L + f3]));
    }
    v = A.cmode == 1 ? csub<T>(v, s) : cadd<T>(v, s);
  }
  for (int side = 0; side < 2; ++side) {
    if (!(terms & (1 << side))) continue;
    // all 18 loads issued together: out-of-range neighbours read entry c and
    // are masked (their coefficients are zero as well)
    const C<T>* cf = A.cbc + ((size_t)(2 * j + side) * nb + c) * 9;
    const C<T>* y = A.Y + ((size_t)rhs * L + (side ? j + 1 : j - 1)) * nb;
    C<T> cv[9], yv[9];
    bool ok[9];
#pragma unroll
    for (int o9 = 0; o9 < 9; ++o9) {
      const int a2 = a + o9 / 3 - 1, f3 = e3 + o9 % 3 - 1;
      ok[o9] = a2 >= 0 && a2 < p.t && f3 >= 0 && f3 < L;
      cv[o9] = cf[o9];
      yv[o9] = y[ok[o9] ? a2 * L + f3 : c];
    }
#pragma unroll
    for (int o9 = 0; o9 < 9; ++o9)
      if (ok[o9]) v = csub<T>(v, cmul<T>(cv[o9], yv[o9]));
  }
  A.z[((size_t)task * A.nrhs + rhs) * nb + c] = v;
}

// z = B_j x_{j-1} (st.terms 0) or C_j x_{j+1} (st.terms 1) for the blocks of
// one step of the outward pass
template <typename T>
__global__ void k3_zb(Slab3Apply<T> A, Slab3Step st) {
  const Slab3 p = A.p;
  const int L = A.L, nb = p.nb, task = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (task >= st.nt || idx >= nb * A.nrhs) return;
  const int j = st.j[task], side = st.terms[task];
  const int rhs = idx / nb, c = idx % nb, a = c / L, e3 = c % L;
  const C<T>* cf = A.cbc + ((size_t)(2 * j + side) * nb + c) * 9;
  const C<T>* x = A.Y + ((size_t)rhs * L + (side ? j + 1 : j - 1)) * nb;
  C<T> v = mk<T>(0, 0);
  C<T> cv[9], xv[9];
  bool ok[9];
#pragma unroll
  for (int o9 = 0; o9 < 9; ++o9) {
    const int a2 = a + o9 / 3 - 1, f3 = e3 + o9 % 3 - 1;
    ok[o9] = a2 >= 0 && a2 < p.t && f3 >= 0 && f3 < L;
    cv[o9] = cf[o9];
    xv[o9] = x[ok[o9] ? a2 * L + f3 : c];
  }
#pragma unroll
  for (int o9 = 0; o9 < 9; ++o9)
    if (ok[o9]) v = cadd<T>(v, cmul<T>(cv[o9], xv[o9]));
  A.z[((size_t)task * A.nrhs + rhs) * nb + c] = v;
}

// Y_j = F_j z (sub = 0) or Y_j -= F_j z (sub = 1) for the right-hand sides
// [r0, r0 + rc); z staged in LDS ([rhs][nb]); each wave takes R consecutive
// rows, its lanes W consecutive columns per load (W = 2: 16-byte loads of two
// complex64), U loads per row in flight; with out, the D part of the result
// also goes to dst
template <int W, typename T>
struct WVec;
template <>
struct WVec<1, float> {
  using type = float2;
};
template <>
struct WVec<2, float> {
  using type = float4;
};
template <>
struct WVec<1, double> {
  using type = double2;
};

// kernel geometry: 16 waves per workgroup, kGemvRows rows, each row split
// into two column halves (one wave each); partial sums meet in LDS
constexpr int kGemvRows = 8;
constexpr int kGemvThreads = 1024;

template <typename T, int KC, int W>
__global__ __launch_bounds__(kGemvThreads) void k3_gemv(Slab3Apply<T> A, Slab3Step stp, int sub, int out, int r0,
                                                        int rc) {
  constexpr int RW = kGemvRows, H = kGemvThreads / 64 / RW, U = 8, ZU = 4;
  using V = typename WVec<W, T>::type;
  extern __shared__ unsigned char smem_raw[];
  C<T>* zl = reinterpret_cast<C<T>*>(smem_raw);
  __shared__ C<T> part[kGemvThreads / 64][KC];
  const Slab3 p = A.p;
  const int L = A.L, nb = p.nb, task = blockIdx.y;
  if (task >= stp.nt) return;
  const int j = stp.j[task];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rr = wv % RW, hh = wv / RW;
  const int row = blockIdx.x * RW + rr;
  const V* rp = reinterpret_cast<const V*>(A.F + ((size_t)j * nb + min(row, nb - 1)) * nb);
  const int nv = nb / W;  // vectors per row (nb is a multiple of W)
  const int nvh = (nv + H - 1) / H, vb = min(hh * nvh, nv), ve = min(nv, vb + nvh);
  // z of right-hand sides r0 .. r0 + rc - 1 (one contiguous run of nz
  // vectors): the first ZU per thread are requested before the matrix, so
  // that they return first; the barrier orders LDS only, the matrix loads
  // stay in flight across it
  const V* zs = reinterpret_cast<const V*>(A.z + ((size_t)task * A.nrhs + r0) * nb);
  V* zd = reinterpret_cast<V*>(zl);
  const int nz = rc * nb / W;
  V tz[ZU];
#pragma unroll
  for (int u = 0; u < ZU; ++u) {
    const int i = threadIdx.x + u * kGemvThreads;
    tz[u] = zs[i < nz ? i : 0];
  }
  V f[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int v = vb + lane + 64 * u;
    f[u] = rp[v < ve ? v : 0];
  }
#pragma unroll
  for (int u = 0; u < ZU; ++u) {
    const int i = threadIdx.x + u * kGemvThreads;
    if (i < nz) zd[i] = tz[u];
  }
  for (int i = threadIdx.x + ZU * kGemvThreads; i < nz; i += kGemvThreads) zd[i] = zs[i];
  lds_barrier();
  T ax[KC], ay[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) ax[k] = ay[k] = T(0);
  for (int v0 = vb + lane; v0 < ve; v0 += 64 * U) {
    if (v0 != vb + lane) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int v = v0 + 64 * u;
        f[u] = rp[v < ve ? v : 0];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + 64 * u;
      if (v >= ve) break;
      const T* fv = reinterpret_cast<const T*>(&f[u]);
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        if (k < rc) {
          // the W complex of z that meet this vector, one LDS read
          const V zz = reinterpret_cast<const V*>(zl)[(k * nb) / W + v];
          const T* zv = reinterpret_cast<const T*>(&zz);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const T fx = fv[2 * w], fy = fv[2 * w + 1], zx = zv[2 * w], zy = zv[2 * w + 1];
            ax[k] += fx * zx - fy * zy;
            ay[k] += fx * zy + fy * zx;
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KC; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      ax[k] += __shfl_xor(ax[k], off);
      ay[k] += __shfl_xor(ay[k], off);
    }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < KC; ++k) part[wv][k] = mk<T>(ax[k], ay[k]);
  }
  __syncthreads();
  // thread t < RW KC: row t / KC of the workgroup, right-hand side t % KC
  const int t = threadIdx.x, q = t / KC, k = t % KC, r = blockIdx.x * RW + q;
  if (t < RW * KC && k < rc && r < nb) {
    C<T> v = part[q][k];
    for (int h = 1; h < H; ++h) v = cadd<T>(v, part[h * RW + q][k]);
    const int rhs = r0 + k;
    C<T>* y = A.Y + ((size_t)rhs * L + j) * nb + r;
    if (sub) v = csub<T>(*y, v);
    *y = v;
    const int a = r / L, e3 = r % L;
    if (out && a >= p.naux) {
      C<T>* d = A.dst + rhs * A.dst_rs + ((size_t)(a - p.naux) * L + j) * L + e3;
      *d = A.dop ? csub<T>(*d, v) : v;
    }
  }
}

}  // namespace

// ---- launchers -----------------------------------------------------------------

template <typename T>
hipError_t launch3_apply_Q(const Stencil3& S, const C<T>* r, int nrhs, C<T>* f, hipStream_t st) {
  const size_t tot = (size_t)S.L * S.L * S.L * nrhs;
  hipLaunchKernelGGL(k3_apply_Q<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, r, nrhs, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch3_apply_H(const Stencil3& S, const C<T>* u, int nrhs, C<T>* y, hipStream_t st) {
  const size_t tot = (size_t)S.L * S.L * S.L * nrhs;
  hipLaunchKernelGGL(k3_apply_H<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, u, nrhs, y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch3_extract(const C<T>* u, int n, int b, int nrhs, C<T>* z, hipStream_t st) {
  const size_t tot = (size_t)n * n * n * nrhs;
  hipLaunchKernelGGL(k3_extract<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, u, n, b, nrhs, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch3_factor(const Stencil3& S, const Slab3* slabs, const Slab3Work* works, int nentries, int maxnb,
                          C<T>* const* factors, int* status, hipStream_t st) {
  const int L = S.L, m = L / 2, steps = std::max(m, L - 1 - m);
  const dim3 gm((maxnb + 255) / 256, maxnb);
  if (maxnb > kSlab3MaxBlock) return hipErrorInvalidValue;
  {
    hipError_t e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(k3_gj_panel<4>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGjLdsBytes)) != hipSuccess ||
        (e = hipFuncSetAttribute(reinterpret_cast<const void*>(k3_gj_panel<2>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGjLdsBytes)) != hipSuccess)
      return e;
  }
  // one block of every entry named by cs: Schur complement (unless skip_s),
  // then its inverse
  auto invert = [&](ChainStep cs, int ne) {
    for (int k0 = 0; k0 < maxnb; k0 += kGjPanel) {
      // entries whose block size takes the other sub-panel width return at once
      hipLaunchKernelGGL(k3_gj_panel<4>, dim3(1, 1, ne), dim3(kGjThreads),
                         (size_t)std::min(maxnb, 2400) * 4 * sizeof(double2), st, slabs, works, L, cs, k0, status);
      if (maxnb > 2400)
        hipLaunchKernelGGL(k3_gj_panel<2>, dim3(1, 1, ne), dim3(kGjThreads), (size_t)maxnb * 2 * sizeof(double2), st,
                           slabs, works, L, cs, k0, status);
      hipLaunchKernelGGL(k3_gj_swap, dim3((maxnb + 255) / 256, 1, ne), dim3(256), 0, st, slabs, works, L, cs, k0);
      hipLaunchKernelGGL(k3_gj_update, dim3((maxnb + 63) / 64, (maxnb + 63) / 64, ne), dim3(256), 0, st, slabs,
                         works, L, cs, k0);
    }
    hipLaunchKernelGGL(k3_gj_perm, dim3(1, 1, ne), dim3(64), 0, st, slabs, works, L, cs);
    hipLaunchKernelGGL(k3_gj_store<T>, dim3(gm.x, gm.y, ne), dim3(256), 0, st, slabs, works, L, cs, factors);
  };
  for (int s = 0; s < steps; ++s) {
    const ChainStep cs{s, m, 0, 1, 0};
    hipLaunchKernelGGL(k3_coefs, dim3((maxnb * 9 + 255) / 256, 1, nentries), dim3(256), 0, st, S, slabs, works, cs);
    hipLaunchKernelGGL(k3_schur_w, dim3(gm.x, gm.y, nentries), dim3(256), 0, st, slabs, works, L, cs);
    hipLaunchKernelGGL(k3_schur_s, dim3(gm.x, gm.y, nentries), dim3(256), 0, st, slabs, works, L, cs);
    invert(cs, nentries);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // the middle block: both chains' couplings (every entry), then on the top
  // entries S = A_m - B_m W_top - C_m W_bottom and its inverse
  const ChainStep all{0, m, 1, 1, 0}, top{0, m, 1, 2, 0};
  const int nslab = nentries / 2;
  hipLaunchKernelGGL(k3_coefs, dim3((maxnb * 9 + 255) / 256, 1, nentries), dim3(256), 0, st, S, slabs, works, all);
  hipLaunchKernelGGL(k3_schur_w, dim3(gm.x, gm.y, nentries), dim3(256), 0, st, slabs, works, L, all);
  hipLaunchKernelGGL(k3_schur_s, dim3(gm.x, gm.y, nslab), dim3(256), 0, st, slabs, works, L, top);
  hipLaunchKernelGGL(k3_schur_sub, dim3(gm.x, gm.y, nslab), dim3(256), 0, st, slabs, works, L, top);
  invert(top, nslab);
  return hipGetLastError();
}

template <typename T>
hipError_t launch3_apply_coefs(const Stencil3& S, const Slab3* slabs, int nslab, int maxnb, C<T>* const* cbc,
                               C<T>* const* cm, C<T>* const* cpl, hipStream_t st) {
  const size_t tot = std::max((size_t)S.L * 2 * maxnb * 9, (size_t)S.L * S.L * 9);
  hipLaunchKernelGGL(k3_apply_coefs<T>, dim3((unsigned)((tot + 255) / 256), 1, nslab), dim3(256), 0, st, S, slabs,
                     cbc, cm, cpl);
  return hipGetLastError();
}

size_t slab3_gemv_lds(int nb, int rc, size_t cs) { return (size_t)rc * nb * cs; }

// complex per load of the wide matrix-vector form (complex64 only)
template <typename T>
struct WideW {
  static constexpr int value = 1;
};
template <>
struct WideW<float> {
  static constexpr int value = 2;
};

template <typename T>
hipError_t launch3_slab_solve(const Slab3Apply<T>& A, hipStream_t st) {
  const int nb = A.p.nb, L = A.L;
  const int zt = (nb * A.nrhs + 255) / 256;
  // right-hand sides per product: as many as 64 KB of LDS hold, at most 8
  // right-hand sides per product: as many as 60 KB of LDS hold (the kernel's
  // static partial sums take the rest of the default 64 KB), at most 8
  int kc = (int)std::min<size_t>(8, 61440 / ((size_t)nb * sizeof(C<T>)));
  if (kc < 1) kc = 1;
  // complex64 with an even block size: 16-byte loads of two complex
  const bool wide = sizeof(T) == 4 && nb % 2 == 0;
  const dim3 gg((nb + kGemvRows - 1) / kGemvRows);
  {
    // beyond 60 KB only single right-hand-side products run (kc = 1)
    const size_t lds = slab3_gemv_lds(nb, std::min(kc, A.nrhs), sizeof(C<T>));
    if (lds + 2048 > 163840) return hipErrorInvalidValue;
    if (lds > 61440) {
      hipError_t e;
      if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(k3_gemv<T, 1, 1>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
        return e;
      if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(k3_gemv<T, 1, WideW<T>::value>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
        return e;
    }
  }
  auto gemv = [&](const Slab3Step& sp, int sub, int out) {
    const dim3 g(gg.x, sp.nt);
    for (int r0 = 0; r0 < A.nrhs; r0 += kc) {
      const int rc = std::min(kc, A.nrhs - r0);
      const size_t lds = slab3_gemv_lds(nb, rc, sizeof(C<T>));
      if (wide) {
        if (rc > 4)
          hipLaunchKernelGGL((k3_gemv<T, 8, WideW<T>::value>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
        else if (rc > 1)
          hipLaunchKernelGGL((k3_gemv<T, 4, WideW<T>::value>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
        else
          hipLaunchKernelGGL((k3_gemv<T, 1, WideW<T>::value>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
      } else {
        if (rc > 4)
          hipLaunchKernelGGL((k3_gemv<T, 8, 1>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
        else if (rc > 1)
          hipLaunchKernelGGL((k3_gemv<T, 4, 1>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
        else
          hipLaunchKernelGGL((k3_gemv<T, 1, 1>), g, dim3(kGemvThreads), lds, st, A, sp, sub, out, r0, rc);
      }
    }
  };
  // two-ended elimination: the top chain takes blocks 0 .. m-1, the bottom
  // chain L-1 .. m+1, one block of each per launch; then the middle block;
  // then both chains outwards
  const int m = L / 2, lt = m, lb = L - 1 - m, steps = std::max(lt, lb);
  for (int s = 0; s < steps; ++s) {
    Slab3Step sp{};
    if (s < lt) {
      sp.j[sp.nt] = s;
      sp.terms[sp.nt++] = s > 0 ? 1 : 0;
    }
    if (s < lb) {
      sp.j[sp.nt] = L - 1 - s;
      sp.terms[sp.nt++] = s > 0 ? 2 : 0;
    }
    hipLaunchKernelGGL(k3_zf<T>, dim3(zt, sp.nt), dim3(256), 0, st, A, sp);
    gemv(sp, 0, 0);
  }
  {
    Slab3Step sp{};
    sp.nt = 1;
    sp.j[0] = m;
    sp.terms[0] = 3;
    hipLaunchKernelGGL(k3_zf<T>, dim3(zt, 1), dim3(256), 0, st, A, sp);
    gemv(sp, 0, 1);
  }
  for (int s = 0; s < steps; ++s) {
    Slab3Step sp{};
    if (s < lt) {
      sp.j[sp.nt] = m - 1 - s;
      sp.terms[sp.nt++] = 1;  // C_j x_{j+1}
    }
    if (s < lb) {
      sp.j[sp.nt] = m + 1 + s;
      sp.terms[sp.nt++] = 0;  // B_j x_{j-1}
    }
    hipLaunchKernelGGL(k3_zb<T>, dim3(zt, sp.nt), dim3(256), 0, st, A, sp);
    gemv(sp, 1, 1);
  }
  return hipGetLastError();
}

#define LSW_SLAB3_INST(T)                                                                                         \
  template hipError_t launch3_apply_Q<T>(const Stencil3&, const C<T>*, int, C<T>*, hipStream_t);                  \
  template hipError_t launch3_apply_H<T>(const Stencil3&, const C<T>*, int, C<T>*, hipStream_t);                  \
  template hipError_t launch3_extract<T>(const C<T>*, int, int, int, C<T>*, hipStream_t);                         \
  template hipError_t launch3_factor<T>(const Stencil3&, const Slab3*, const Slab3Work*, int, int, C<T>* const*, \
                                        int*, hipStream_t);                                                      \
  template hipError_t launch3_apply_coefs<T>(const Stencil3&, const Slab3*, int, int, C<T>* const*,               \
                                             C<T>* const*, C<T>* const*, hipStream_t);                            \
  template hipError_t launch3_slab_solve<T>(const Slab3Apply<T>&, hipStream_t);
LSW_SLAB3_INST(double)
LSW_SLAB3_INST(float)

}  // namespace lsw
