// Sparsified system and moving-PML sweep on the GPU.
//
// Stencils (Sec. 2.2): rows of H at grid points of I^h = [0, n+1]^2 use
// conj(alpha_o) + omega^2 conj(beta_o) m_{i+o} (eq. local_c_approx); rows in
// the PML use conj(gamma_i,o) (eq. PML_stencil); u = 0 on the Dirichlet ring.
//
// Slices (Sec. 2.3): D_k is a range of lines i1; the subproblem of slice k
// (eq. Hwv_approx) lives on t lines [first_k, hi_k] x L transverse points:
// b auxiliary PML lines (k > 0, gamma rows at the sampled local frequency)
// followed by the lines of D_k (rows of H, coupling to D_{k+1} dropped).
// Ordered by the transverse index j, the subproblem is block tridiagonal with
// t x t blocks
//     B_j x_{j-1} + A_j x_j + C_j x_{j+1} = r_j,
// each block itself tridiagonal (9-point stencil). Block elimination
//     S_0 = A_0,  S_j = A_j - B_j G_{j-1},  G_j = S_j^{-1} C_j
// is done in float64 with partial pivoting inside each S_j; the factors kept
// per block are S_j^{-1} (dense), G_j (dense) and the three diagonals of B_j.
// A solve is then
//     y_j = S_j^{-1} (r_j - B_j y_{j-1}),   x_{L-1} = y_{L-1},  x_j = y_j - G_j x_{j+1}.
//
// Sweep (Algorithm 2): forward u_1 = T_1 f_1, u_k = T_k (f_k - H_[k,k-1] u_{k-1});
// backward u_k -= T_k (H_[k,k+1] u_{k+1}). Only the first line of D_k couples
// to the last line of D_{k-1} (and the last to the first of D_{k+1}), three
// coefficients per transverse point, kept in Hm and Hp.
#include "kernels.hpp"

namespace lsw {

namespace {

__device__ inline int d_axis_class(int i, int n, int b) {
  if (i < 0) return i + b + 1;
  if (i > n + 1) return i - (n + 2) + b + 1;
  return 0;
}

// Coefficient of H in the row of grid point (i1, i2) for neighbour (d1, d2).
__device__ double2 h_coef(const StencilTables& S, int i1, int i2, int d1, int d2) {
  const int o = (d1 + 1) * 3 + (d2 + 1);
  const int n = S.n;
  if (i1 >= 0 && i1 <= n + 1 && i2 >= 0 && i2 <= n + 1) {
    const int j1 = i1 + d1, j2 = i2 + d2;
    double mm = 0.0;
    if (j1 >= 1 && j1 <= n && j2 >= 1 && j2 <= n) mm = S.m[(size_t)(j1 - 1) * n + (j2 - 1)];
    const double2 al = S.alpha[o], be = S.beta[o];
    return make_double2(al.x + S.omega2 * be.x * mm, -al.y - S.omega2 * be.y * mm);
  }
  const int NC = 2 * S.b + 1;
  const int c1 = d_axis_class(i1, n, S.b), c2 = d_axis_class(i2, n, S.b);
  const double2 g = S.gglob[((size_t)c1 * NC + c2) * 9 + o];
  return make_double2(g.x, -g.y);
}

// Coefficient of an auxiliary-PML row at depth q, transverse grid index i2,
// sample ks, neighbour (d1, d2).
__device__ double2 aux_coef(const StencilTables& S, int q, int i2, int ks, int d1, int d2) {
  const int o = (d1 + 1) * 3 + (d2 + 1);
  const int NC = 2 * S.b + 1;
  const int c2 = d_axis_class(i2, S.n, S.b);
  const double2 g = S.gaux[(((size_t)q * NC + c2) * S.ns + ks) * 9 + o];
  return make_double2(g.x, -g.y);
}

template <typename T>
__device__ inline C<T> shfl_xor_c(C<T> v, int mask) {
  return mk<T>(__shfl_xor(v.x, mask), __shfl_xor(v.y, mask));
}

// ---- Q and H applies ---------------------------------------------------
template <typename T>
__global__ void k_apply_Q(StencilTables S, const C<T>* __restrict__ r, int nrhs, C<T>* __restrict__ f) {
  const int L = S.L, n = S.n, b = S.b;
  const size_t plane = (size_t)L * L;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= plane * nrhs) return;
  const int rhs = (int)(idx / plane);
  const int e = (int)(idx % plane);
  const int i1 = e / L - b, i2 = e % L - b;
  C<T> acc = mk<T>(0, 0);
  if (i1 >= 0 && i1 <= n + 1 && i2 >= 0 && i2 <= n + 1) {
    const C<T>* rr = r + (size_t)rhs * n * n;
    for (int o = 0; o < 9; ++o) {
      const int j1 = i1 + o / 3 - 1, j2 = i2 + o % 3 - 1;
      if (j1 < 1 || j1 > n || j2 < 1 || j2 > n) continue;
      const double2 al = S.alpha[o];
      acc = cfma<T>(acc, mk<T>((T)al.x, (T)-al.y), rr[(size_t)(j1 - 1) * n + (j2 - 1)]);
    }
  }
  f[idx] = acc;
}

template <typename T>
__global__ void k_apply_H(StencilTables S, const C<T>* __restrict__ u, int nrhs, C<T>* __restrict__ y) {
  const int L = S.L, b = S.b;
  const size_t plane = (size_t)L * L;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= plane * nrhs) return;
  const int rhs = (int)(idx / plane);
  const int e = (int)(idx % plane);
  const int e1 = e / L, e2 = e % L;
  const C<T>* ur = u + (size_t)rhs * plane;
  C<T> acc = mk<T>(0, 0);
  for (int o = 0; o < 9; ++o) {
    const int d1 = o / 3 - 1, d2 = o % 3 - 1;
    const int f1 = e1 + d1, f2 = e2 + d2;
    if (f1 < 0 || f1 >= L || f2 < 0 || f2 >= L) continue;
    const double2 c = h_coef(S, e1 - b, e2 - b, d1, d2);
    acc = cfma<T>(acc, mk<T>((T)c.x, (T)c.y), ur[(size_t)f1 * L + f2]);
  }
  y[idx] = acc;
}

// Q into the interleaved layout f[e1][e2][nrhs] (right-hand side fastest).
// A workgroup owns a strip of 64 columns, kQRows consecutive extended rows
// and 16 right-hand sides, and slides down the strip in chunks of CH rows: a
// ring of CH + 2 input rows (66 columns, the strip and its two neighbours,
// for 16 right-hand sides) sits in LDS, so every input row is fetched once
// per strip (plus two halo rows per strip). A chunk's CH input rows are
// loaded at once (CH x 5 loads per thread in flight), then its CH output rows
// are formed; each crosses LDS and leaves with the right-hand side fastest.
// R64: right-hand side q read from r64[q] (float64), narrowed to T when it
// enters the ring.
constexpr int kQRows = 32;
constexpr int kQCols = 66;                          // 64 outputs + 2 halo columns
constexpr int kQLoads = (16 * kQCols + 255) / 256;  // input loads per thread and row
constexpr int kQRingRows = kQLoads * 256 / kQCols + 1;  // every load slot has a place

template <typename T, bool R64>
__global__ __launch_bounds__(256) void k_apply_Q_il(StencilTables S, const C<T>* __restrict__ r, int nrhs,
                                                    C<T>* __restrict__ f, const double2* const* __restrict__ r64) {
  constexpr int CH = sizeof(T) == 4 ? 4 : 2;  // rows per chunk (the LDS ring holds CH + 2)
  constexpr int RS = CH + 2;
  __shared__ C<T> ring[RS][kQRingRows][kQCols];
  __shared__ C<T> tile[2][64][17];
  const int L = S.L, n = S.n, b = S.b;
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * kQRows, q0 = blockIdx.z * 16;
  const int r1 = min(r0 + kQRows, L);
  const int t = threadIdx.x, c = t & 63, sub = t >> 6;
  // this thread's load slots: right-hand side lq[s], input column
  // c0 - b - 1 + lc[s]; lv[s] false for slots off the interior columns or
  // past the 16 right-hand sides (their values are zeroed)
  int lq[kQLoads], lc[kQLoads], col[kQLoads];
  bool lv[kQLoads];
  // the grids of this thread's right-hand sides (global address space:
  // global loads, not flat ones)
  using G64 = const __attribute__((address_space(1))) double;
  using GT = const __attribute__((address_space(1))) T;
  G64* rp64[kQLoads];
  GT* rpT[kQLoads];
#pragma unroll
  for (int s = 0; s < kQLoads; ++s) {
    const int idx = t + 256 * s;
    lq[s] = idx / kQCols;
    lc[s] = idx % kQCols;
    const int j2 = c0 - b - 1 + lc[s];
    lv[s] = idx < 16 * kQCols && q0 + lq[s] < nrhs && j2 >= 1 && j2 <= n;
    col[s] = min(max(j2, 1), n) - 1;
    const int q = min(q0 + lq[s], nrhs - 1);
    if constexpr (R64) rp64[s] = (G64*)r64[q];
    else rpT[s] = (GT*)(r + (size_t)q * n * n);  // scalar view of the complex grid
  }
  // raw values of input rows, in the input's precision
  using RT = typename std::conditional<R64, double2, C<T>>::type;
  auto load_row = [&](int j1, RT(&rg)[kQLoads]) {
    const size_t base = (size_t)(min(max(j1, 1), n) - 1) * n;
#pragma unroll
    for (int s = 0; s < kQLoads; ++s) {
      const size_t at = base + col[s];
      if constexpr (R64) rg[s] = make_double2(rp64[s][2 * at], rp64[s][2 * at + 1]);
      else rg[s] = mk<T>(rpT[s][2 * at], rpT[s][2 * at + 1]);
    }
  };
  // ring slot of input row j1 (rows from r0 - b - 1 on)
  auto slot = [&](int j1) { return (j1 - (r0 - b - 1)) % RS; };
  auto store_row = [&](int j1, const RT(&rg)[kQLoads]) {
    const int sl = slot(j1);
    const bool rowok = j1 >= 1 && j1 <= n;
#pragma unroll
    for (int s = 0; s < kQLoads; ++s) {
      // zero off the interior by a factor, not a branch
      const T msk = (rowok && lv[s]) ? T(1) : T(0);
      ring[sl][lq[s]][lc[s]] = mk<T>((T)rg[s].x * msk, (T)rg[s].y * msk);
    }
  };
  C<T> al[9];
#pragma unroll
  for (int o = 0; o < 9; ++o) al[o] = mk<T>((T)S.alpha[o].x, (T)-S.alpha[o].y);
  const int i2 = c0 + c - b;
  const bool colok = c0 + c < L && i2 >= 0 && i2 <= n + 1;
  {
    RT rg[2][kQLoads];
    load_row(r0 - b - 1, rg[0]);
    load_row(r0 - b, rg[1]);
    store_row(r0 - b - 1, rg[0]);
    store_row(r0 - b, rg[1]);
  }
  for (int e0 = r0; e0 < r1; e0 += CH) {
    // input rows e0 - b + 1 .. e0 - b + CH (clamped rows past the strip's end
    // are loaded and dropped)
    {
      RT rg[CH][kQLoads];
#pragma unroll
      for (int k = 0; k < CH; ++k) load_row(e0 - b + 1 + k, rg[k]);
#pragma unroll
      for (int k = 0; k < CH; ++k) store_row(e0 - b + 1 + k, rg[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e1 = e0 + k, i1 = e1 - b;
      const bool ok = colok && i1 >= 0 && i1 <= n + 1;
      const int s0 = slot(i1 - 1), s1 = slot(i1), s2 = slot(i1 + 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int rr = sub + 4 * s;
        C<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const int sl = o < 3 ? s0 : (o < 6 ? s1 : s2);
          acc = cfma<T>(acc, al[o], ring[sl][rr][c + o % 3]);
        }
        tile[k & 1][c][rr] = ok ? acc : mk<T>(0, 0);
      }
      __syncthreads();
      // output row e1 through a buffer of that row: columns past L and right-
      // hand sides past nrhs are dropped by the range check, and a row past
      // the strip's end has an empty buffer
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          f + (size_t)min(e1, L - 1) * L * nrhs, 0, e1 < r1 ? (int)(L * nrhs * sizeof(C<T>)) : 0, 0x00020000);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int idx = t + 256 * s;
        const int rr = idx & 15, cc = idx >> 4;
        const int e2 = c0 + cc, q = q0 + rr;
        const int off = (e2 < L && q < nrhs) ? (e2 * nrhs + q) * (int)sizeof(C<T>) : -1;
        store_or_drop<T>(rs, off, tile[k & 1][cc][rr]);
      }
    }
  }
}

// z[nrhs][n][n] = the interior of the interleaved u[e1][e2][nrhs], through LDS
// as in k_apply_Q_il.
// zp: right-hand side q written to the grid zp[q] instead of z
template <typename T>
__global__ __launch_bounds__(256) void k_extract_il(int n, int b, const C<T>* __restrict__ uext, int nrhs,
                                                    C<T>* __restrict__ z, C<T>* const* __restrict__ zp) {
  __shared__ C<T> tile[16][65];
  const int L = n + 2 + 2 * b;
  const int c0 = blockIdx.x * 64, a1 = blockIdx.y, q0 = blockIdx.z * 16;
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int idx = t + 256 * s;
    const int rr = idx & 15, cc = idx >> 4;
    const int a2 = c0 + cc, q = q0 + rr;
    if (a2 < n && q < nrhs) tile[rr][cc] = uext[((size_t)(a1 + 1 + b) * L + a2 + 1 + b) * nrhs + q];
  }
  __syncthreads();
  const int c = t & 63, sub = t >> 6;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int rr = sub + 4 * s, q = q0 + rr;
    if (c0 + c < n && q < nrhs) {
      const size_t at = (size_t)a1 * n + c0 + c;
      if (zp) {
        // the grids are device memory: global stores, not flat ones
        using G = __attribute__((address_space(1))) T;
        G* zq = (G*)zp[q];
        zq[2 * at] = tile[rr][c].x;
        zq[2 * at + 1] = tile[rr][c].y;
      } else {
        z[(size_t)q * n * n + at] = tile[rr][c];
      }
    }
  }
}

template <typename T>
__global__ void k_extract(int n, int b, const C<T>* __restrict__ uext, int nrhs, C<T>* __restrict__ z) {
  const size_t nn = (size_t)n * n;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * nrhs) return;
  const int rhs = (int)(idx / nn);
  const int a = (int)(idx % nn);
  const int a1 = a / n, a2 = a % n;
  const int L = n + 2 + 2 * b;
  z[idx] = uext[(size_t)rhs * L * L + (size_t)(a1 + 1 + b) * L + (a2 + 1 + b)];
}

// ---- slice assembly and block elimination (one workgroup per slice) ------
constexpr int kTMax = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_factor(StencilTables S, SliceTables P, C<T>* __restrict__ FS,
                                                C<T>* __restrict__ FG, C<T>* __restrict__ Hm,
                                                C<T>* __restrict__ Hp, int* __restrict__ status) {
  const int k = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lo = P.lo[k], hi = P.hi[k], t = P.t[k];
  const int naux = P.naux[k], org = P.org[k], dir = P.dir[k];
  const int L = S.L, b = S.b;
  const int W = 2 * t;
  const int tw = hi - lo + 1;  // lines of D_k
  const int tt = t * t, fstride = factor_stride(t, tw), gstride = factor_stride(t, 0);
  __shared__ double2 Gp[kTMax * kTMax];
  __shared__ double2 M[kTMax * 2 * kTMax];
  __shared__ double2 At[kTMax * 3], Bt[kTMax * 3], Ct[kTMax * 3];
  __shared__ double2 fcol[kTMax];
  __shared__ int piv_s;
  __shared__ double2 ipiv_s;
  C<T>* fs = FS + P.fs_off[k];
  C<T>* fg = FG + P.fg_off[k];
  for (int j = 0; j < L; ++j) {
    // 1. the three tridiagonal blocks of block row j
    // local lines a and offsets d1: grid line org + dir a, grid offset dir d1
    for (int idx = tid; idx < t * 9; idx += nt) {
      const int a = idx / 9, o = idx % 9, d1 = o / 3 - 1, d2 = o % 3 - 1;
      const int line = org + dir * a, i2 = j - b;
      double2 c = make_double2(0.0, 0.0);
      if (a + d1 >= 0 && a + d1 < t && j + d2 >= 0 && j + d2 < L) {
        if (a < naux) {  // auxiliary PML before D_k, depth q from D_k's edge
          const int ks = S.kmap[(size_t)(line + b) * L + j];
          c = aux_coef(S, naux - 1 - a, i2, ks, d1, d2);
        } else if (a >= naux + tw) {  // after D_k: the same stencils, mirrored
          const int ks = S.kmap[(size_t)(line + b) * L + j];
          c = aux_coef(S, a - naux - tw, i2, ks, -d1, d2);
        } else {
          c = h_coef(S, line, i2, dir * d1, d2);
        }
      }
      double2* dst = d2 < 0 ? Bt : (d2 == 0 ? At : Ct);
      dst[a * 3 + d1 + 1] = c;
    }
    lds_barrier();
    // 2. S_j = A_j - B_j G_{j-1}, augmented with the identity
    for (int idx = tid; idx < t * W; idx += nt) {
      const int a = idx / W, c = idx % W;
      double2 v = make_double2(0.0, 0.0);
      if (c < t) {
        if (c - a >= -1 && c - a <= 1) v = At[a * 3 + (c - a) + 1];
        if (j > 0) {
          for (int d = -1; d <= 1; ++d) {
            const int a2 = a + d;
            if (a2 < 0 || a2 >= t) continue;
            const double2 bb = Bt[a * 3 + d + 1], g = Gp[a2 * kTMax + c];
            v.x -= bb.x * g.x - bb.y * g.y;
            v.y -= bb.x * g.y + bb.y * g.x;
          }
        }
      } else if (c - t == a) {
        v.x = 1.0;
      }
      M[a * (2 * kTMax) + c] = v;
    }
    lds_barrier();
    // 3. Gauss-Jordan with partial pivoting: [S | I] -> [I | S^{-1}]
    for (int p = 0; p < t; ++p) {
      if (tid < 64) {
        double best = -1.0;
        int br = p;
        for (int r = p + tid; r < t; r += 64) {
          const double2 v = M[r * (2 * kTMax) + p];
          const double a2 = v.x * v.x + v.y * v.y;
          if (a2 > best) {
            best = a2;
            br = r;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int orr = __shfl_xor(br, off);
          if (ob > best || (ob == best && orr < br)) {
            best = ob;
            br = orr;
          }
        }
        if (tid < t) {
          const int src = tid == p ? br : (tid == br ? p : tid);
          fcol[tid] = M[src * (2 * kTMax) + p];
        }
        if (tid == 0) {
          piv_s = br;
          const double2 pv = M[br * (2 * kTMax) + p];
          const double d = pv.x * pv.x + pv.y * pv.y;
          if (!(d > 0.0) || !(d < INFINITY)) {
            atomicMax(status, k + 1);
            ipiv_s = make_double2(0.0, 0.0);
          } else {
            ipiv_s = make_double2(pv.x / d, -pv.y / d);
          }
        }
      }
      lds_barrier();
      const int pr = piv_s;
      const double2 ip = ipiv_s;
      for (int c = tid; c < W; c += nt) {  // swap rows p, pr and scale the pivot row
        const double2 vp = M[p * (2 * kTMax) + c], vr = M[pr * (2 * kTMax) + c];
        M[p * (2 * kTMax) + c] = make_double2(vr.x * ip.x - vr.y * ip.y, vr.x * ip.y + vr.y * ip.x);
        if (pr != p) M[pr * (2 * kTMax) + c] = vp;
      }
      lds_barrier();
      for (int idx = tid; idx < t * W; idx += nt) {
        const int r = idx / W, c = idx % W;
        if (r == p) continue;
        const double2 fr = fcol[r], pc = M[p * (2 * kTMax) + c];
        double2 v = M[r * (2 * kTMax) + c];
        v.x -= fr.x * pc.x - fr.y * pc.y;
        v.y -= fr.x * pc.y + fr.y * pc.x;
        M[r * (2 * kTMax) + c] = v;
      }
      lds_barrier();
    }
    // 4. W_j = S_j^{-1} B_j and G_j = S_j^{-1} C_j (B_j, C_j tridiagonal); the
    //    columns of S_j^{-1} on the lines of D_k (the only nonzero right-hand side rows)
    for (int idx = tid; idx < tt; idx += nt) {
      const int a = idx / t, c = idx % t;
      double2 g = make_double2(0.0, 0.0), wv = make_double2(0.0, 0.0);
      for (int d = -1; d <= 1; ++d) {
        const int c2 = c - d;  // rows c2 of B_j, C_j have their entry at column c2 + d = c
        if (c2 < 0 || c2 >= t) continue;
        const double2 s = M[a * (2 * kTMax) + t + c2], cc = Ct[c2 * 3 + d + 1], bb = Bt[c2 * 3 + d + 1];
        g.x += s.x * cc.x - s.y * cc.y;
        g.y += s.x * cc.y + s.y * cc.x;
        wv.x += s.x * bb.x - s.y * bb.y;
        wv.y += s.x * bb.y + s.y * bb.x;
      }
      Gp[a * kTMax + c] = g;
      fg[(size_t)j * gstride + idx] = ccast<T, double>(g);
      fs[(size_t)j * fstride + idx] = ccast<T, double>(wv);
    }
    for (int idx = tid; idx < t * tw; idx += nt) {
      const int a = idx / tw, c = idx % tw;
      fs[(size_t)j * fstride + tt + idx] = ccast<T, double>(M[a * (2 * kTMax) + t + naux + c]);
    }
    lds_barrier();
  }
  // couplings to the slices before and after in the front's order: Hm from
  // D_k's first local line one line back, Hp from its last local line one
  // line on (H_[k,k-1] and H_[k,k+1] of the one-front sweep)
  const int dfirst = org + dir * naux, dlast = org + dir * (naux + tw - 1);
  for (int idx = tid; idx < 3 * L; idx += nt) {
    const int j = idx / 3, d2 = idx % 3 - 1;
    const bool ok = j + d2 >= 0 && j + d2 < L;
    double2 cm = make_double2(0.0, 0.0), cp = make_double2(0.0, 0.0);
    if (ok && P.prev[k] >= 0) cm = h_coef(S, dfirst, j - b, -dir, d2);
    if (ok && P.next[k] >= 0) cp = h_coef(S, dlast, j - b, dir, d2);
    Hm[(size_t)k * L * 3 + idx] = ccast<T, double>(cm);
    Hp[(size_t)k * L * 3 + idx] = ccast<T, double>(cp);
  }
}

// One 64-point x 16-column tile per workgroup through LDS, so that both the
// point-fastest and the column-fastest sides move in contiguous runs.
template <typename T>
__global__ __launch_bounds__(256) void k_interleave(const C<T>* __restrict__ in, int nb, size_t E,
                                                    C<T>* __restrict__ out, int to_il) {
  __shared__ C<T> tile[64][17];
  const size_t p0 = (size_t)blockIdx.x * 64;
  const int q0 = blockIdx.y * 16;
  const int t = threadIdx.x;
  for (int s = 0; s < 4; ++s) {
    const int idx = t + 256 * s;
    if (to_il) {  // read [q][p]: 64 consecutive points of a column
      const int pp = idx & 63, qq = idx >> 6;
      if (p0 + pp < E && q0 + qq < nb) tile[pp][qq] = in[(size_t)(q0 + qq) * E + p0 + pp];
    } else {      // read [p][q]: 16 consecutive columns of a point
      const int qq = idx & 15, pp = idx >> 4;
      if (p0 + pp < E && q0 + qq < nb) tile[pp][qq] = in[(p0 + pp) * nb + q0 + qq];
    }
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    const int idx = t + 256 * s;
    if (to_il) {
      const int qq = idx & 15, pp = idx >> 4;
      if (p0 + pp < E && q0 + qq < nb) out[(p0 + pp) * nb + q0 + qq] = tile[pp][qq];
    } else {
      const int pp = idx & 63, qq = idx >> 6;
      if (p0 + pp < E && q0 + qq < nb) out[(size_t)(q0 + qq) * E + p0 + pp] = tile[pp][qq];
    }
  }
}

// ---- slice solves and the sweep (one workgroup per right-hand side) -------
enum SolveKind { kFwd = 0, kBwd = 1, kTest = 2 };

template <typename T>
__device__ void slice_solve(int kind, int k, const SliceTables& P, int L, int b,
                            const C<T>* __restrict__ FS, const C<T>* __restrict__ FG,
                            const C<T>* __restrict__ Hm, const C<T>* __restrict__ Hp,
                            const C<T>* __restrict__ in, C<T>* __restrict__ out, C<T>* __restrict__ yg,
                            C<T> (*ybuf)[kTMax], C<T>* zbuf) {
  const int lo = P.lo[k], hi = P.hi[k], first = P.first[k], t = P.t[k];
  const int naux = lo - first;
  const int a = threadIdx.x >> 3, cb = threadIdx.x & 7;
  const int tt = t * t, fstride = factor_stride(t, t - naux), gstride = factor_stride(t, 0);
  const C<T>* fs = FS + P.fs_off[k];
  const C<T>* fg = FG + P.fg_off[k];
  const bool own = (cb == 0) && (a < t);
  const int tw = t - naux;
  // forward elimination: y_j = S_j^{-1} r_j - W_j y_{j-1} (r_j nonzero on the lines of D_k only)
  for (int j = 0; j < L; ++j) {
    const int cur = j & 1;
    if (own) {
      C<T> z = mk<T>(0, 0);
      if (kind == kFwd) {
        if (a >= naux) {
          z = in[(size_t)(first + a + b) * L + j];
          if (a == naux && k > 0) {
            const C<T>* hm = Hm + ((size_t)k * L + j) * 3;
            const C<T>* prev = out + (size_t)(lo - 1 + b) * L;
            for (int d = -1; d <= 1; ++d)
              if (j + d >= 0 && j + d < L) z = csub<T>(z, cmul<T>(hm[d + 1], prev[j + d]));
          }
        }
      } else if (kind == kBwd) {
        if (a == t - 1) {
          const C<T>* hp = Hp + ((size_t)k * L + j) * 3;
          const C<T>* next = out + (size_t)(hi + 1 + b) * L;
          for (int d = -1; d <= 1; ++d)
            if (j + d >= 0 && j + d < L) z = cfma<T>(z, hp[d + 1], next[j + d]);
        }
      } else {
        if (a >= naux) z = in[(size_t)(a - naux) * L + j];
      }
      zbuf[a] = z;
    }
    __syncthreads();
    C<T> acc = mk<T>(0, 0);
    if (a < t) {
      const C<T>* Wj = fs + (size_t)j * fstride + a * t;
      const C<T>* Sd = fs + (size_t)j * fstride + tt + a * tw;
      for (int c = cb; c < tw; c += 8) acc = cfma<T>(acc, Sd[c], zbuf[naux + c]);
      if (j > 0)
        for (int c = cb; c < t; c += 8) acc = csub<T>(acc, cmul<T>(Wj[c], ybuf[cur ^ 1][c]));
    }
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 1));
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 2));
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 4));
    if (own) {
      ybuf[cur][a] = acc;
      yg[(size_t)j * kTMax + a] = acc;
    }
    __syncthreads();
  }
  // back substitution
  int cur = (L - 1) & 1;
  auto emit = [&](int j, C<T> x) {
    if (a < naux) return;
    if (kind == kFwd) {
      out[(size_t)(first + a + b) * L + j] = x;
    } else if (kind == kBwd) {
      C<T>* o = out + (size_t)(first + a + b) * L + j;
      *o = csub<T>(*o, x);
    } else {
      out[(size_t)(a - naux) * L + j] = x;
    }
  };
  if (own) emit(L - 1, ybuf[cur][a]);
  for (int j = L - 2; j >= 0; --j) {
    C<T> acc = mk<T>(0, 0);
    if (a < t) {
      const C<T>* Gj = fg + (size_t)j * gstride + a * t;
      for (int c = cb; c < t; c += 8) acc = cfma<T>(acc, Gj[c], ybuf[cur][c]);
    }
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 1));
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 2));
    acc = cadd<T>(acc, shfl_xor_c<T>(acc, 4));
    if (own) {
      const C<T> x = csub<T>(yg[(size_t)j * kTMax + a], acc);
      ybuf[cur ^ 1][a] = x;
      emit(j, x);
    }
    __syncthreads();
    cur ^= 1;
  }
  __threadfence();
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_sweep(SliceTables P, int L, int b, const C<T>* __restrict__ FS,
                                               const C<T>* __restrict__ FG, const C<T>* __restrict__ Hm,
                                               const C<T>* __restrict__ Hp, const C<T>* __restrict__ f,
                                               C<T>* __restrict__ u, C<T>* __restrict__ yscr, int mode,
                                               int slice) {
  __shared__ C<T> ybuf[2][kTMax];
  __shared__ C<T> zbuf[kTMax];
  const int rhs = blockIdx.x;
  C<T>* yg = yscr + (size_t)rhs * L * kTMax;
  if (mode == kSweepFull) {
    const size_t plane = (size_t)L * L;
    const C<T>* fr = f + rhs * plane;
    C<T>* ur = u + rhs * plane;
    for (int k = 0; k < P.nslices; ++k)
      slice_solve<T>(kFwd, k, P, L, b, FS, FG, Hm, Hp, fr, ur, yg, ybuf, zbuf);
    for (int k = P.nslices - 2; k >= 0; --k)
      slice_solve<T>(kBwd, k, P, L, b, FS, FG, Hm, Hp, fr, ur, yg, ybuf, zbuf);
  } else {
    const int lines = P.hi[slice] - P.lo[slice] + 1;
    const size_t sz = (size_t)lines * L;
    slice_solve<T>(kTest, slice, P, L, b, FS, FG, Hm, Hp, f + rhs * sz, u + rhs * sz, yg, ybuf, zbuf);
  }
}

inline unsigned blocks_for(size_t total, int nt) { return (unsigned)((total + nt - 1) / nt); }

}  // namespace

template <typename T>
hipError_t launch_apply_Q(const StencilTables& S, const C<T>* r, int nrhs, C<T>* f, bool interleaved,
                          hipStream_t st, const double2* const* r64) {
  if (interleaved) {
    const dim3 g((S.L + 63) / 64, (S.L + kQRows - 1) / kQRows, (nrhs + 15) / 16);
    if (r64)
      hipLaunchKernelGGL((k_apply_Q_il<T, true>), g, dim3(256), 0, st, S, r, nrhs, f, r64);
    else
      hipLaunchKernelGGL((k_apply_Q_il<T, false>), g, dim3(256), 0, st, S, r, nrhs, f, r64);
    return hipGetLastError();
  }
  if (r64) return hipErrorInvalidValue;
  const size_t tot = (size_t)S.L * S.L * nrhs;
  hipLaunchKernelGGL(k_apply_Q<T>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, S, r, nrhs, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_H(const StencilTables& S, const C<T>* u, int nrhs, C<T>* y, hipStream_t st) {
  const size_t tot = (size_t)S.L * S.L * nrhs;
  hipLaunchKernelGGL(k_apply_H<T>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, S, u, nrhs, y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_extract(int n, int b, const C<T>* uext, int nrhs, C<T>* z, bool interleaved, hipStream_t st,
                          C<T>* const* zp) {
  if (interleaved) {
    hipLaunchKernelGGL(k_extract_il<T>, dim3((n + 63) / 64, n, (nrhs + 15) / 16), dim3(256), 0, st, n, b, uext, nrhs, z,
                       zp);
    return hipGetLastError();
  }
  if (zp) return hipErrorInvalidValue;
  const size_t tot = (size_t)n * n * nrhs;
  hipLaunchKernelGGL(k_extract<T>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, n, b, uext, nrhs, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interleave(const C<T>* in, int nb, size_t E, C<T>* out, bool to_il, hipStream_t st) {
  const dim3 grid((unsigned)((E + 63) / 64), (unsigned)((nb + 15) / 16));
  hipLaunchKernelGGL(k_interleave<T>, grid, dim3(256), 0, st, in, nb, E, out, to_il ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_interleave<double>(const double2*, int, size_t, double2*, bool, hipStream_t);
template hipError_t launch_interleave<float>(const float2*, int, size_t, float2*, bool, hipStream_t);

template <typename T>
hipError_t launch_factor_slices(const StencilTables& S, const SliceTables& P, C<T>* FS, C<T>* FG,
                                C<T>* Hm, C<T>* Hp, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_factor<T>, dim3(P.nslices), dim3(256), 0, st, S, P, FS, FG, Hm, Hp, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SliceTables& P, int L, int b, const C<T>* FS, const C<T>* FG,
                        const C<T>* Hm, const C<T>* Hp, const C<T>* f, C<T>* u, C<T>* yscratch,
                        int nrhs, int mode, int slice, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep<T>, dim3(nrhs), dim3(256), 0, st, P, L, b, FS, FG, Hm, Hp, f, u, yscratch,
                     mode, slice);
  return hipGetLastError();
}

#define LSW_INST(T)                                                                                  \
  template hipError_t launch_apply_Q<T>(const StencilTables&, const C<T>*, int, C<T>*, bool, hipStream_t,    \
                                        const double2* const*);                                               \
  template hipError_t launch_apply_H<T>(const StencilTables&, const C<T>*, int, C<T>*, hipStream_t); \
  template hipError_t launch_extract<T>(int, int, const C<T>*, int, C<T>*, bool, hipStream_t,        \
                                        C<T>* const*);                                               \
  template hipError_t launch_factor_slices<T>(const StencilTables&, const SliceTables&, C<T>*,       \
                                              C<T>*, C<T>*, C<T>*, int*, hipStream_t);               \
  template hipError_t launch_sweep<T>(const SliceTables&, int, int, const C<T>*, const C<T>*,        \
                                      const C<T>*, const C<T>*, const C<T>*, C<T>*, C<T>*, int, int, \
                                      int, hipStream_t);
LSW_INST(double)
LSW_INST(float)
#undef LSW_INST

}  // namespace lsw
