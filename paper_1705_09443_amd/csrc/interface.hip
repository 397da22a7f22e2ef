// Interface form of the moving-PML sweep (Algorithm 2) for the GPU.
//
// The sweep couples slice k to its neighbours only through one line each:
// H_[k,k-1] reads the last line of D_{k-1}, H_[k,k+1] the first line of
// D_{k+1}. Write E (F) for the restriction to the last (first) line of D_k,
// J_E (J_F) for the injection into the right-hand side rows of that line and
// Hm_k, Hp_k for the three-coefficient coupling rows. With
//     lambda_k = E u_k(forward pass),   mu_k = F u_k(final),
// Algorithm 2 is equivalent to
//     lambda_0 = E T_0 f_0,   lambda_k = E T_k f_k - M_k lambda_{k-1},
//     mu_{l-1} = F T_{l-1} f_{l-1} - P_{l-1} lambda_{l-2},
//     mu_k     = F T_k f_k - P_k lambda_{k-1} - N_k mu_{k+1},
//     u_k      = T_k (f_k - J_F Hm_k lambda_{k-1} - J_E Hp_k mu_{k+1}),
// with the L x L interface maps M_k = E T_k J_F Hm_k, P_k = F T_k J_F Hm_k,
// N_k = F T_k J_E Hp_k built once at setup (slice solves with the L
// columns of J_F Hm_k or J_E Hp_k as right-hand sides). Every slice solve
// is then independent: all slices run at once (phase A: the boundary lines
// of T_k f_k; phase C: the final fields), and only the two short recurrences
// for lambda and mu remain sequential, each step a dense L x L product.
// The result is that of the sequential sweep up to rounding.
//
// Slice solves: block elimination along the transverse index j with the
// factors of k_factor (W_j = S_j^{-1} B_j, the columns of S_j^{-1} on the
// lines of D_k, G_j = S_j^{-1} C_j). A workgroup solves one slice, one wave
// per right-hand side; factor blocks stream into LDS D steps ahead by direct
// global-to-LDS copies, so the dependent chain of 2L block steps reads LDS
// only and needs no workgroup barrier per step.
#include "kernels.hpp"

#include <cstdlib>

namespace lsw {

namespace {

constexpr int kNT = 256;

template <typename T>
__device__ inline C<T> shfl_xor_c(C<T> v, int mask) {
  return mk<T>(__shfl_xor(v.x, mask), __shfl_xor(v.y, mask));
}

// complex values per 16-byte direct-to-LDS copy
template <typename T>
constexpr int kCpl = 16 / (int)sizeof(C<T>);
// block steps staged per chunk (16-line or 32-line subproblems)
template <int TP>
constexpr int kDepth = TP == 16 ? 8 : 2;

// exchanges within lane quads: quad_perm(1,0,3,2) = 0xB1, quad_perm(2,3,0,1) = 0x4E
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline float dpp(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ inline double dpp(double v) { return dpp_d<CTRL>(v); }

// threads of a slice-solve workgroup: W computing waves, at least 4 (float)
// or 8 (double) waves so that staging a chunk takes few registers per thread
template <typename T, int W>
constexpr int slice_threads() {
  constexpr int hw = sizeof(T) == 8 ? 8 : 4;
  return 64 * (W > hw ? W : hw);
}

// Dynamic LDS of k_slice_solve for SB stage elements per buffer.
template <typename T, int TP, int W>
constexpr size_t slice_lds_bytes(size_t SB) {
  return (2 * SB + (size_t)W * (4 * kDepth<TP> * TP + 2 * TP)) * sizeof(C<T>);
}

// Wait for every outstanding global load and store of the wave. Issued once,
// outside any branch, so that the compiler knows at the loop head that no
// load is still in flight (a wait it places inside a branch that may be
// skipped would make it wait again there, on stores as well).
__device__ __attribute__((always_inline)) inline void wait_vm_all() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unconstrained
}

// Chunk staging through registers: load count values (this thread's share)
// while the previous chunk is in use, store them to LDS when it is done.
// Loads are unconditional (clamped to element 0, which every caller owns) so
// no wait ends up inside a branch.
template <typename T, int NREG>
struct Stager {
  T re[NREG], im[NREG];
  __device__ __attribute__((always_inline)) inline void load(const C<T>* g, int count, int tid, int nt) {
#pragma unroll
    for (int q = 0; q < NREG; ++q) {
      const int e = tid + q * nt;
      const C<T> v = g[e < count ? e : 0];
      re[q] = v.x;
      im[q] = v.y;
    }
  }
  __device__ __attribute__((always_inline)) inline void store(C<T>* l, int count, int tid, int nt) {
    wait_vm_all();
#pragma unroll
    for (int q = 0; q < NREG; ++q) {
      const int e = tid + q * nt;
      if (e < count) l[e] = mk<T>(re[q], im[q]);
    }
  }
};

// One slice subproblem per workgroup, one right-hand side per wave. Lanes:
// S = 4 (16-line) or 2 (32-line) lanes per row, each lane a stride-S set of
// columns, reductions within lane quads by DPP. The dependent chain
//   y_j = S_j^{-1} r_j - W_j y_{j-1}   (forward),   x_j = y_j - G_j x_{j+1}   (backward)
// passes the t-vector through the wave's own LDS row (LDS operations of a
// wave complete in order, so no barrier per step).
template <typename T, int TP, int W>
__device__ __attribute__((always_inline)) inline void slice_body(const SliceSolveArgs<T>& A, int k, int sl,
                                                                 int group, int ngroups) {
  constexpr int NT = slice_threads<T, W>();
  constexpr int CB = 4;  // columns per lane loaded and used together
  constexpr int S = TP == 16 ? 4 : 2;
  constexpr int D = kDepth<TP>;
  constexpr int NR = (D * TP + 63) / 64;
  // largest chunk: D blocks of the forward factors (t^2 + t tw <= 2 TP^2)
  constexpr int NSTAGE = (D * 2 * TP * TP + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  C<T>* lds = reinterpret_cast<C<T>*>(smem_raw);

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool computes = wv < W;  // waves beyond W only help staging
  const int a = lane / S, cq = lane % S;
  const int rr = group * W + wv;
  const bool rvalid = computes && rr < A.nrhs;
  const int L = A.L, b = A.b;
  const int lo = A.P.lo[k], hi = A.P.hi[k], t = A.P.t[k];
  const int naux = A.P.naux[k], tw = hi - lo + 1, org = A.P.org[k], dir = A.P.dir[k];
  const int tt = t * t, fstride = factor_stride(t, tw), gstride = factor_stride(t, 0);
  // grid line (+ b) of local line a, and the row of D_k's local line c in a
  // slice array (grid order)
  auto gline = [&](int a) { return org + dir * a + b; };
  auto srow = [&](int c) { return dir > 0 ? c : tw - 1 - c; };
  const C<T>* fs = A.FS + A.P.fs_off[k];
  const C<T>* fg = A.FG + A.P.fg_off[k];
  const bool unit_src = A.src_kind >= kSrcUnitF;
  const C<T>* hrow = A.src_kind == kSrcUnitF ? A.Hm : A.Hp;
  const int unit_c = A.src_kind == kSrcUnitF ? 0 : tw - 1;  // right-hand side line within D_k
  const int col = A.col0 + rr;                               // column of the unit sources
  const bool arow = a < t;

  const size_t SB = A.stage;
  C<T>* stage = lds;                                     // [2][SB] factor chunks (shared)
  C<T>* wreg = lds + 2 * SB + (size_t)(computes ? wv : 0) * (4 * D * TP + 2 * TP);
  C<T>* rst = wreg;                                      // [2][D][TP] right-hand sides
  C<T>* yst = wreg + 2 * D * TP;                         // [2][D][TP] forward results
  C<T>* yb = wreg + 4 * D * TP;                          // [TP] exchange row
  // scratch by global slice index: launches over disjoint slice ranges may run concurrently
  C<T>* yg = A.yscr + (((size_t)k * ngroups + group) * W + (computes ? wv : 0)) * (size_t)L * 32;
  const int tid = threadIdx.x;
  Stager<T, NSTAGE> stg;
  Stager<T, NR> ystg;

  const int nchunks = (L + D - 1) / D;
  C<T> rreg[NR];
  auto load_rhs = [&](int c) {  // element e = line * D + jj (consecutive j in memory)
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = lane + q * 64;
      const int jj = e % D, cl = e / D;
      const int j = c * D + jj;
      bool ok = rvalid && cl < tw && j < L;
      const C<T>* base = A.src;
      size_t off;
      if (A.src_kind == kSrcGrid) {
        off = ((size_t)gline(naux + (cl < tw ? cl : 0)) * L + j) * A.nrhs + rr;
      } else if (A.src_kind == kSrcSlice) {
        off = ((size_t)rr * tw + srow(cl < tw ? cl : 0)) * L + j;
      } else {
        const int dj = col - j;
        ok = ok && cl == unit_c && dj >= -1 && dj <= 1;
        base = hrow;
        off = ((size_t)k * L + j) * 3 + dj + 1;
      }
      // one unconditional load per element (element 0 when masked)
      const C<T> v = base[ok ? off : 0];
      rreg[q] = ok ? v : mk<T>(0, 0);
    }
  };
  auto store_rhs = [&](int buf) {
    wait_vm_all();
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = lane + q * 64;
      if (e < D * TP) rst[buf * D * TP + (e % D) * TP + e / D] = rreg[q];
    }
  };
  auto reduce = [&](C<T> v) {
    v.x += dpp<0xB1>(v.x);
    v.y += dpp<0xB1>(v.y);
    if (S == 4) {
      v.x += dpp<0x4E>(v.x);
      v.y += dpp<0x4E>(v.y);
    }
    return v;
  };

  // ---------------- forward elimination ----------------
  if (computes && lane < TP) yb[lane] = mk<T>(0, 0);
  {
    const int cnt = (L < D ? L : D) * fstride;
    stg.load(fs, cnt, tid, NT);
    if (computes) load_rhs(0);
    stg.store(stage, cnt, tid, NT);
    if (computes) store_rhs(0);
    lds_barrier();
  }
  C<T> ylast = mk<T>(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const int j1 = (c + 1) * D;
    const bool more = c + 1 < nchunks;
    const int cnt1 = more ? (L - j1 < D ? L - j1 : D) * fstride : 0;
    // the prefetch and its LDS store run on every chunk (nothing is copied
    // after the last): straight-line code keeps the compiler's wait analysis exact
    stg.load(fs + (more ? (size_t)j1 * fstride : 0), cnt1, tid, NT);
    if (computes) load_rhs(c + 1);
    const C<T>* F = stage + buf * SB;
    const C<T>* RB = rst + buf * D * TP;
    const int jend = (L - c * D < D) ? L - c * D : D;
    for (int jj = 0; jj < jend && computes; ++jj) {
      const int j = c * D + jj;
      // rows a >= t and columns >= t read in-range LDS garbage that the masks drop
      const C<T>* Wj = F + jj * fstride + a * t;
      const C<T>* Sd = F + jj * fstride + tt + a * tw;
      C<T> acc = mk<T>(0, 0);
      const bool chain = j > 0;
#pragma unroll
      for (int blk = 0; blk < TP / S / CB; ++blk) {
        C<T> wv[CB], yv[CB], sv[CB], rv[CB];
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          const int cc = cq + (blk * CB + i) * S;
          const int cw = cc < t ? cc : 0, cs = cc < tw ? cc : 0;
          wv[i] = Wj[cw];
          yv[i] = yb[cw];
          sv[i] = Sd[cs];
          rv[i] = RB[jj * TP + cs];
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          // selects, not multiplications by 0: masked operands may hold any bits
          const int cc = cq + (blk * CB + i) * S;
          C<T> pw = cmul<T>(wv[i], yv[i]), ps = cmul<T>(sv[i], rv[i]);
          if (!(cc < t && chain)) pw = mk<T>(0, 0);
          if (!(cc < tw)) ps = mk<T>(0, 0);
          acc.x += ps.x - pw.x;
          acc.y += ps.y - pw.y;
        }
      }
      if (!arow) acc = mk<T>(0, 0);
      acc = reduce(acc);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (cq == 0 && arow) {
        yb[a] = acc;
        yst[buf * D * TP + jj * TP + a] = acc;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      ylast = acc;
    }
    lds_barrier();  // every wave is done with buffer buf ^ 1's previous contents
    stg.store(stage + (buf ^ 1) * SB, cnt1, tid, NT);
    if (computes) store_rhs(buf ^ 1);
    lds_barrier();
    // the chunk's results go out after the loads above were waited for, so the
    // next chunk's wait covers these stores too, one chunk after they issued
    if (computes) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int e = lane + q * 64;
        if (e < jend * TP) yg[(size_t)c * D * TP + e] = yst[buf * D * TP + e];
      }
    }
  }
  // the forward results in yg are read back below
  __threadfence_block();
  __syncthreads();

  // ---------------- back substitution ----------------
  const bool inD = a >= naux && a < naux + tw;
  auto emit = [&](int j, C<T> x) {
    if (!rvalid || !arow || cq != 0) return;
    if (A.dst_kind == kDstGrid) {
      if (inD) A.dst[((size_t)gline(a) * L + j) * A.nrhs + rr] = x;
    } else if (A.dst_kind == kDstSlice) {
      if (inD) A.dst[((size_t)rr * tw + srow(a - naux)) * L + j] = x;
    } else {
      const size_t ci = unit_src ? (size_t)col : (size_t)rr;
      if (a == naux + tw - 1 && A.dstE) A.dstE[k * A.sk + ci * A.sr + (size_t)j * A.sj] = x;
      if (a == naux && A.dstF) A.dstF[k * A.sk + ci * A.sr + (size_t)j * A.sj] = x;
    }
  };
  emit(L - 1, ylast);  // x_{L-1} = y_{L-1}; it is also what yb holds
  // outputs of a backward chunk wait in the wave's (now unused) right-hand side
  // buffer and leave together, consecutive j per lane group
  C<T>* xo = rst;
  auto flush_bwd = [&](int c, int buf) {
    if (!rvalid) return;
    const int j0 = c * D;
    const int n = (L - 1 - j0 < D ? L - 1 - j0 : D);
    if (A.dst_kind == kDstLines) {
      const size_t ci = unit_src ? (size_t)col : (size_t)rr;
      if (lane < 2 * D) {
        const int jj = lane % D;
        const bool isE = lane < D;
        C<T>* dl = isE ? A.dstE : A.dstF;
        const int ar = isE ? naux + tw - 1 : naux;
        if (dl && jj < n) dl[k * A.sk + ci * A.sr + (size_t)(j0 + jj) * A.sj] = xo[buf * D * TP + jj * TP + ar];
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = lane + q * 64;
      const int jj = e % D, ar = e / D;
      if (jj < n && ar >= naux && ar < naux + tw) {
        const C<T> x = xo[buf * D * TP + jj * TP + ar];
        if (A.dst_kind == kDstGrid)
          A.dst[((size_t)gline(ar) * L + j0 + jj) * A.nrhs + rr] = x;
        else
          A.dst[((size_t)rr * tw + srow(ar - naux)) * L + j0 + jj] = x;
      }
    }
  };
  const int nbch = (L - 1 + D - 1) / D;  // chunks of j in [c D, c D + D) cover 0..L-2
  // chunk c of the backward pass; on == false copies nothing (the last chunk)
  auto bwd_count = [&](int c, bool on) {
    const int j0 = c * D;
    return on ? (L - 1 - j0 < D ? L - 1 - j0 : D) : 0;
  };
  auto load_bwd = [&](int c, bool on) {
    const int j0 = c * D, n = bwd_count(c, on);
    stg.load(fg + (size_t)j0 * gstride, n * gstride, tid, NT);
    if (computes) ystg.load(yg + (size_t)j0 * TP, n * TP, lane, 64);  // this wave's own rows
  };
  auto store_bwd = [&](int c, int buf, bool on) {
    const int n = bwd_count(c, on);
    stg.store(stage + buf * SB, n * gstride, tid, NT);
    if (computes) ystg.store(yst + buf * D * TP, n * TP, lane, 64);
  };
  if (nbch > 0) {
    load_bwd(nbch - 1, true);
    store_bwd(nbch - 1, 0, true);
    lds_barrier();
  }
  for (int ci = 0; ci < nbch; ++ci) {
    const int c = nbch - 1 - ci;
    const int buf = ci & 1;
    const bool more = ci + 1 < nbch;
    load_bwd(more ? c - 1 : 0, more);
    const C<T>* G = stage + buf * SB;
    const C<T>* Y = yst + buf * D * TP;
    for (int jj = D - 1; jj >= 0 && computes; --jj) {
      const int j = c * D + jj;
      if (j > L - 2) continue;
      const C<T>* Gj = G + jj * gstride + a * t;
      C<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int blk = 0; blk < TP / S / CB; ++blk) {
        C<T> gv[CB], xv[CB];
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          const int cc = cq + (blk * CB + i) * S;
          const int cw = cc < t ? cc : 0;
          gv[i] = Gj[cw];
          xv[i] = yb[cw];
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          C<T> p = cmul<T>(gv[i], xv[i]);
          if (!(cq + (blk * CB + i) * S < t)) p = mk<T>(0, 0);
          acc.x += p.x;
          acc.y += p.y;
        }
      }
      if (!arow) acc = mk<T>(0, 0);
      acc = reduce(acc);
      C<T> x = mk<T>(0, 0);
      if (arow) x = csub<T>(Y[jj * TP + a], acc);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (cq == 0 && arow) {
        yb[a] = x;
        xo[buf * D * TP + jj * TP + a] = x;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    lds_barrier();
    store_bwd(more ? c - 1 : 0, buf ^ 1, more);
    lds_barrier();
    if (computes) flush_bwd(c, buf);
  }
}

// One launch covers a range of slices: blockIdx.x is the group of W
// right-hand sides, blockIdx.y the slice, the last slice of the range first
// (it is the longest: the far PML makes it the only 32-line class), so that it
// starts before the others rather than after them. BIG: the range holds a
// 32-line slice.
template <typename T, int W, bool BIG>
__global__ __launch_bounds__((slice_threads<T, W>())) void k_slice_solve(SliceSolveArgs<T> A) {
  const int sl = gridDim.y - 1 - blockIdx.y;
  const int k = A.slice0 + sl;
  if (BIG && A.P.t[k] > 16)
    slice_body<T, 32, W>(A, k, sl, blockIdx.x, gridDim.x);
  else
    slice_body<T, 16, W>(A, k, sl, blockIdx.x, gridDim.x);
}

// ---- interface recurrences: y = add - M x for a batch of right-hand sides --
// The L x L maps are stored in the operand order of the matrix-core product:
// slice k is [row tile r][contraction block b], 16 x 16 complex values per
// (r, b), zero-padded to whole tiles. Lane l of a block holds row
// 16 r + l % 16 and the 4 columns 16 b + iface_k(l / 16, j), j = 0..3, in
// 16-byte chunks (2 complex64 or 1 complex128), chunk c of every lane side by
// side: each 16-byte load of the wave reads one contiguous kilobyte. The
// contraction index within a block is permuted so that a lane's chunk c
// holds consecutive indices, and the four lane groups' chunks c are
// consecutive: the same loads of x then read contiguous runs of each column.
// The padding removes every bounds test on M. x, add, y: [nrhs][Lp] per slice.
template <typename T>
__host__ __device__ constexpr int iface_ch() { return 16 / (int)sizeof(C<T>); }
// contraction index (within a 16-block) of lane group g4's j-th value
template <typename T>
__host__ __device__ constexpr int iface_k(int g4, int j) {
  return (j / iface_ch<T>()) * 4 * iface_ch<T>() + g4 * iface_ch<T>() + j % iface_ch<T>();
}
// position of lane l's j-th value within its 256-value block
template <typename T>
__host__ __device__ constexpr int iface_pos(int l, int j) {
  return ((j / iface_ch<T>()) * 64 + l) * iface_ch<T>() + j % iface_ch<T>();
}
__host__ __device__ inline int iface_tiles(int L) { return (L + 15) / 16; }
// x, add, y rows (one per right-hand side) are padded to whole 16-blocks:
// [nrhs][Lp] per slice, with zeros in [L, Lp) that nothing writes. (The
// transposed layout, right-hand side fastest, measured slower in the chain.)
__host__ __device__ inline int iface_vec_len(int L) { return 16 * iface_tiles(L); }

// lane's 4 values of one map block (laid out by iface_pos), whole 16-byte loads
__device__ __attribute__((always_inline)) inline void load_m4(const float2* blk, int lane, float2* out) {
  const float4 u = reinterpret_cast<const float4*>(blk)[lane], v = reinterpret_cast<const float4*>(blk)[64 + lane];
  out[0] = make_float2(u.x, u.y);
  out[1] = make_float2(u.z, u.w);
  out[2] = make_float2(v.x, v.y);
  out[3] = make_float2(v.z, v.w);
}
__device__ __attribute__((always_inline)) inline void load_m4(const double2* blk, int lane, double2* out) {
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j] = blk[j * 64 + lane];
}
// lane group g4's 4 values of one 16-block of a column of x (indices iface_k)
__device__ __attribute__((always_inline)) inline void load_x4(const float2* col, int g4, float2* out) {
  const float4 u = reinterpret_cast<const float4*>(col)[g4], v = reinterpret_cast<const float4*>(col)[4 + g4];
  out[0] = make_float2(u.x, u.y);
  out[1] = make_float2(u.z, u.w);
  out[2] = make_float2(v.x, v.y);
  out[3] = make_float2(v.z, v.w);
}
__device__ __attribute__((always_inline)) inline void load_x4(const double2* col, int g4, double2* out) {
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j] = col[4 * j + g4];
}

template <typename T>
__global__ void k_swizzle_maps(const C<T>* __restrict__ src, C<T>* __restrict__ dst, int L, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int nt = iface_tiles(L);
  const size_t per = (size_t)nt * nt * 256;
  const size_t k = e / per, rem = e % per;
  const int r = (int)(rem / ((size_t)nt * 256)), b = (int)((rem / 256) % nt);
  constexpr int ch = iface_ch<T>();
  const int in = (int)(rem % 256);
  const int l = (in / ch) % 64, j = in / (64 * ch) * ch + in % ch;  // iface_pos<T>(l, j) == in
  const int row = 16 * r + (l & 15), col = 16 * b + iface_k<T>(l >> 4, j);
  dst[e] = (row < L && col < L) ? src[(k * L + row) * (size_t)L + col] : mk<T>(0, 0);
}

// At most 4 right-hand sides: a workgroup per 16-row tile, its NW waves
// taking every NW-th contraction block; each lane accumulates its row's
// partial dot products over the block's 4 columns it holds, the four lanes of
// a row then reduce by shuffles and the waves through LDS.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_iface_gemv(IfaceProds<T> ps, int L, int nrhs) {
  constexpr int MAXB = 6;  // blocks of one wave in flight at once
  __shared__ C<T> red[NW][4][16];
  const int nt = iface_tiles(L);
  const IfaceProd<T> pr = ps.p[blockIdx.z];
  const C<T>* add = pr.add;
  C<T>* y = pr.y;
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g4 = lane >> 4;
  const int Lp = iface_vec_len(L);
  const C<T>* Mr = pr.M + (size_t)r * nt * 256;
  const C<T>* xk = pr.x;
  C<T> acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = mk<T>(0, 0);
  for (int b0 = wave; b0 < nt; b0 += NW * MAXB) {
    C<T> a[MAXB][4];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = min(b0 + i * NW, nt - 1);  // clamped: blocks past the end are loaded, not used
      load_m4(Mr + (size_t)b * 256, lane, a[i]);
    }
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = b0 + i * NW;
      if (b < nt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q < nrhs) {
            C<T> xv[4];
            load_x4(xk + (size_t)q * Lp + 16 * b, g4, xv);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q] = cfma<T>(acc[q], a[i][j], xv[j]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc[q] = cadd<T>(acc[q], shfl_xor_c<T>(acc[q], 16));
    acc[q] = cadd<T>(acc[q], shfl_xor_c<T>(acc[q], 32));
    if (g4 == 0) red[wave][q][li] = acc[q];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 64) {
    const int q = t >> 4, row = 16 * r + (t & 15);
    if (q < nrhs && row < L) {
      C<T> s = red[0][q][t & 15];
#pragma unroll
      for (int w = 1; w < NW; ++w) s = cadd<T>(s, red[w][q][t & 15]);
      const size_t o = (size_t)q * Lp + row;
      y[o] = csub<T>(add[o], s);
    }
  }
}

// The products on the matrix cores. A workgroup owns a 16-row x 16-column
// (right-hand sides) output tile and splits the contraction over its NW
// waves. Each complex 16x16x4 block is three real MFMAs (Karatsuba's form:
// with M = A + iB and x = c + id, P1 = A (c + d), P2 = (A + B) d and
// P3 = (B - A) c give Re = P1 - P2 and Im = P1 + P3), the sums and differences
// formed on the vector ALUs. In the j-th MFMA of a block, lane l supplies
// column iface_k(l / 16, j) of M's row l % 16 and the same contraction index of
// x's column l % 16: the index is permuted the same way in both operands,
// which leaves the sum unchanged. A wave keeps PF blocks of loads in flight
// ahead of its MFMAs. Tiles of one row block share M's rows; they go to
// workgroups with equal id mod 8, i.e. the same XCD.
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __attribute__((always_inline)) v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element j of lane l is row out_row(l / 16, j), column l % 16
  static __device__ __attribute__((always_inline)) int out_row(int g, int j) { return 4 * g + j; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __attribute__((always_inline)) v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __attribute__((always_inline)) int out_row(int g, int j) { return 4 * j + g; }
};

constexpr int kMfmaWaves = 8;
template <typename T>
constexpr int kMfmaPrefetch = sizeof(T) == 4 ? 4 : 2;


template <typename T, int NW = kMfmaWaves, int PF = kMfmaPrefetch<T>>
__global__ __launch_bounds__(64 * NW) void k_iface_mfma(IfaceProds<T> ps, int L, int nrhs, int qtiles) {
  using V = typename Mfma<T>::v4;
  __shared__ C<T> red[NW][16][17];
  const int nt = iface_tiles(L);
  const IfaceProd<T> pr = ps.p[blockIdx.z];
  const C<T>* add = pr.add;
  C<T>* y = pr.y;
  const int id = blockIdx.x;
  const int per = 8 * qtiles;  // workgroups per group of 8 row blocks
  const int r = (id / per) * 8 + id % 8, q = (id % per) / 8;
  if (r >= nt) return;  // whole workgroup: the grid is rounded up to 8 row blocks
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g4 = lane >> 4;
  const int Lp = iface_vec_len(L);
  const C<T>* Mr = pr.M + (size_t)r * nt * 256;
  // columns past nrhs read the last one: their outputs are not stored
  const C<T>* Bc = pr.x + (size_t)min(q * 16 + li, nrhs - 1) * Lp;
  // this wave's contraction blocks: an even share [b0, b1)
  const int b0 = wave * nt / NW, b1 = (wave + 1) * nt / NW;
  V p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
  C<T> a[PF][4], bv[PF][4];
  // unconditional whole-vector loads (block index clamped to the tile range)
  auto load = [&](C<T>* ad, C<T>* bd, int b) {
    const int bc = min(b, nt - 1);
    load_m4(Mr + (size_t)bc * 256, lane, ad);
    load_x4(Bc + 16 * bc, g4, bd);
  };
  auto block = [&](const C<T>* ad, const C<T>* bd) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T A = ad[j].x, B = ad[j].y, c = bd[j].x, d = bd[j].y;
      p1 = Mfma<T>::op(A, c + d, p1);
      p2 = Mfma<T>::op(A + B, d, p2);
      p3 = Mfma<T>::op(B - A, c, p3);
    }
  };
  // whole groups of PF blocks with no branch inside, then the remaining
  // blocks, already loaded by the last group (a branch per block measured
  // 9 % slower per chain step: 15.8 against 14.4 us at L = 1047, 64 columns)
  const int full = (b1 - b0) / PF * PF;
#pragma unroll
  for (int s = 0; s < PF; ++s) load(a[s], bv[s], b0 + s);
  for (int i = b0; i < b0 + full; i += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      block(a[s], bv[s]);
      load(a[s], bv[s], i + s + PF);
    }
  }
#pragma unroll
  for (int s = 0; s < PF - 1; ++s)
    if (b0 + full + s < b1) block(a[s], bv[s]);
#pragma unroll
  for (int j = 0; j < 4; ++j) red[wave][Mfma<T>::out_row(g4, j)][li] = mk<T>(p1[j] - p2[j], p1[j] + p3[j]);
  __syncthreads();
  // one output per thread: column t / 16, row t % 16 (consecutive rows of one
  // right-hand side are contiguous in y)
  const int t = threadIdx.x;
  if (t < 256) {
    const int oc = t >> 4, orow = t & 15;
    const int R = r * 16 + orow, Q = q * 16 + oc;
    if (R < L && Q < nrhs) {
      C<T> sum = red[0][orow][oc];
#pragma unroll
      for (int w = 1; w < NW; ++w) sum = cadd<T>(sum, red[w][orow][oc]);
      const size_t o = (size_t)Q * Lp + R;
      y[o] = csub<T>(add[o], sum);
    }
  }
}

// f on the first local line of D_k -= Hm_k lambda_prev; on its last local line
// -= Hp_k mu_next (lambda_next where the next slice's last line is the
// neighbour: the slices next to the two-front middle slice, and that slice).
// f interleaved [L][L][nrhs]. A workgroup takes one slice (blockIdx.y), 64
// positions j along the line and 16 right-hand sides: the three taps of each
// vector are read along j, the sums cross LDS and leave with the right-hand
// side fastest, as f is laid out.
template <typename T>
__global__ __launch_bounds__(256) void k_couple(SliceTables P, int L, int b, const C<T>* __restrict__ Hm,
                                                const C<T>* __restrict__ Hp, const C<T>* __restrict__ lam,
                                                const C<T>* __restrict__ mu, int nrhs, C<T>* f, int k0, int kcount) {
  __shared__ C<T> tm[64][17], tp[64][17];
  const int k = k0 + (int)blockIdx.y;
  if ((int)blockIdx.y >= kcount) return;
  const int j0 = blockIdx.x * 64, q0 = blockIdx.z * 16;
  const int t = threadIdx.x, c = t & 63, sub = t >> 6, j = j0 + c;
  const int Lp = iface_vec_len(L);
  const int prev = P.prev[k], next = P.next[k];
  const bool hasm = prev >= 0, hasp = next >= 0;
  const C<T>* nvec = P.next_lam[k] ? lam : mu;
  // coefficients of this position (zero off the line: those taps are masked)
  C<T> cm[3], cp[3];
  int at[3];
  bool ok[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int jj = j + d - 1;
    ok[d] = j < L && jj >= 0 && jj < L;
    at[d] = min(max(jj, 0), L - 1);
    const size_t co = ((size_t)k * L + min(j, L - 1)) * 3 + d;
    cm[d] = hasm ? Hm[co] : mk<T>(0, 0);
    cp[d] = hasp ? Hp[co] : mk<T>(0, 0);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int rr = q0 + sub + 4 * s, rq = min(rr, nrhs - 1);
    C<T> am = mk<T>(0, 0), ap = mk<T>(0, 0);
    if (hasm) {
      const C<T>* lv = lam + ((size_t)prev * nrhs + rq) * Lp;
      C<T> v[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = lv[at[d]];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (ok[d]) am = cfma<T>(am, cm[d], v[d]);
    }
    if (hasp) {
      const C<T>* mv = nvec + ((size_t)next * nrhs + rq) * Lp;
      C<T> v[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = mv[at[d]];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (ok[d]) ap = cfma<T>(ap, cp[d], v[d]);
    }
    tm[c][sub + 4 * s] = am;
    tp[c][sub + 4 * s] = ap;
  }
  __syncthreads();
  // grid rows (+ b) of D_k's first and last local lines
  const int tw = P.hi[k] - P.lo[k] + 1, naux = P.naux[k];
  const int lo = P.org[k] + P.dir[k] * naux + b, hi = P.org[k] + P.dir[k] * (naux + tw - 1) + b;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int idx = t + 256 * s;
    const int rr = idx & 15, cc = idx >> 4;
    const int e2 = j0 + cc, q = q0 + rr;
    if (e2 < L && q < nrhs) {
      if (hasm) {
        C<T>* o = f + ((size_t)lo * L + e2) * nrhs + q;
        *o = csub<T>(*o, tm[cc][rr]);
      }
      if (hasp) {
        C<T>* o = f + ((size_t)hi * L + e2) * nrhs + q;
        *o = csub<T>(*o, tp[cc][rr]);
      }
    }
  }
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, int W>
size_t lds_for(bool big, size_t stage) {
  const size_t s16 = slice_lds_bytes<T, 16, W>(stage), s32 = slice_lds_bytes<T, 32, W>(stage);
  return big && s32 > s16 ? s32 : s16;
}

template <typename T, int W, bool BIG>
hipError_t launch_one(const SliceSolveArgs<T>& a, int nslices, int ngroups, hipStream_t st) {
  const size_t bytes = lds_for<T, W>(BIG, a.stage);
  hipError_t e = allow_lds(k_slice_solve<T, W, BIG>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_slice_solve<T, W, BIG>), dim3(ngroups, nslices), dim3(slice_threads<T, W>()), bytes, st, a);
  return hipGetLastError();
}

}  // namespace

template <typename T>
size_t slice_scratch_elems(int L, int W) {
  return (size_t)L * 32 * W;
}
template size_t slice_scratch_elems<double>(int, int);
template size_t slice_scratch_elems<float>(int, int);

template <typename T>
size_t slice_stage_elems(int tmax, int fstride_max) {
  const int TP = tmax > 16 ? 32 : 16;
  const int D = TP == 16 ? kDepth<16> : kDepth<32>;
  const int gmax = factor_stride(TP, 0);
  const size_t sb = (size_t)D * (fstride_max > gmax ? fstride_max : gmax);
  const size_t q = 64 * kCpl<T>;  // whole 64-lane copies stay inside the buffer
  return (sb + q - 1) / q * q;
}
template size_t slice_stage_elems<double>(int, int);
template size_t slice_stage_elems<float>(int, int);

template <typename T>
size_t slice_lds(bool big, size_t stage, int W) {
  switch (W) {
    case 1: return lds_for<T, 1>(big, stage);
    case 4: return lds_for<T, 4>(big, stage);
    case 8: return lds_for<T, 8>(big, stage);
    default: return 0;
  }
}
template size_t slice_lds<double>(bool, size_t, int);
template size_t slice_lds<float>(bool, size_t, int);

template <typename T>
hipError_t launch_slice_solves(const SliceSolveArgs<T>& a, int nslices, bool big, int W, int ngroups,
                               hipStream_t st) {
  switch (W) {
    case 1: return big ? launch_one<T, 1, true>(a, nslices, ngroups, st) : launch_one<T, 1, false>(a, nslices, ngroups, st);
    case 4: return big ? launch_one<T, 4, true>(a, nslices, ngroups, st) : launch_one<T, 4, false>(a, nslices, ngroups, st);
    case 8: return big ? launch_one<T, 8, true>(a, nslices, ngroups, st) : launch_one<T, 8, false>(a, nslices, ngroups, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_slice_solves<double>(const SliceSolveArgs<double>&, int, bool, int, int, hipStream_t);
template hipError_t launch_slice_solves<float>(const SliceSolveArgs<float>&, int, bool, int, int, hipStream_t);

int iface_vec_stride(int L) { return iface_vec_len(L); }

template <typename T>
size_t iface_map_stride(int L) {
  const size_t nt = iface_tiles(L);
  return nt * nt * 256;
}
template size_t iface_map_stride<double>(int);
template size_t iface_map_stride<float>(int);

template <typename T>
hipError_t launch_swizzle_maps(const C<T>* src, C<T>* dst, int L, int nslices, hipStream_t st) {
  const size_t total = (size_t)nslices * iface_map_stride<T>(L);
  hipLaunchKernelGGL(k_swizzle_maps<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, dst, L, total);
  return hipGetLastError();
}
template hipError_t launch_swizzle_maps<double>(const double2*, double2*, int, int, hipStream_t);
template hipError_t launch_swizzle_maps<float>(const float2*, float2*, int, int, hipStream_t);

template <typename T>
hipError_t launch_iface_prods(const IfaceProd<T>* prods, int nprods, int L, int nrhs, bool mfma, hipStream_t st) {
  if (nprods <= 0) return hipSuccess;
  if (nprods > kIfaceMaxProds) return hipErrorInvalidValue;
  if (!mfma && nrhs > 4) return hipErrorInvalidValue;  // the vector form holds at most 4 columns
  IfaceProds<T> ps{};
  for (int i = 0; i < nprods; ++i) ps.p[i] = prods[i];
  const int nt = iface_tiles(L);
  if (!mfma) {
    constexpr int NW = 8;
    hipLaunchKernelGGL((k_iface_gemv<T, NW>), dim3(nt, 1, nprods), dim3(64 * NW), 0, st, ps, L, nrhs);
  } else {
    const int qtiles = (nrhs + 15) / 16, groups = (nt + 7) / 8;
    const dim3 grid(groups * 8 * qtiles, 1, nprods), block(64 * kMfmaWaves);
    // more than two column tiles put two workgroups on some compute units,
    // where three blocks of loads in flight per wave measured fastest (9.2
    // against 9.4 ms per C2 interface graph with two, slower with four)
    if (qtiles > 2)
      hipLaunchKernelGGL((k_iface_mfma<T, kMfmaWaves, 3>), grid, block, 0, st, ps, L, nrhs, qtiles);
    else
      hipLaunchKernelGGL((k_iface_mfma<T>), grid, block, 0, st, ps, L, nrhs, qtiles);
  }
  return hipGetLastError();
}
template hipError_t launch_iface_prods<double>(const IfaceProd<double>*, int, int, int, bool, hipStream_t);
template hipError_t launch_iface_prods<float>(const IfaceProd<float>*, int, int, int, bool, hipStream_t);

template <typename T>
hipError_t launch_iface_step(const C<T>* M, const C<T>* add, const C<T>* x, C<T>* y, int L, int nrhs, int kbeg,
                             int kcount, size_t mstride, size_t vstride, int xoff, bool mfma, hipStream_t st,
                             const C<T>* M2, const C<T>* add2, C<T>* y2) {
  if (kcount <= 0) return hipSuccess;
  if (M2 && kcount != 1) return hipErrorInvalidValue;  // a second product only beside a single one
  if (kcount > kIfaceMaxProds) return hipErrorInvalidValue;
  IfaceProd<T> ps[kIfaceMaxProds];
  int np = 0;
  for (int i = 0; i < kcount; ++i) {
    const int k = kbeg + i;
    ps[np++] = {M + (size_t)k * mstride, add + (size_t)k * vstride, x + (size_t)(k + xoff) * vstride,
                y + (size_t)k * vstride};
  }
  if (M2) ps[np++] = {M2 + (size_t)kbeg * mstride, add2 + (size_t)kbeg * vstride, x + (size_t)(kbeg + xoff) * vstride,
                      y2 + (size_t)kbeg * vstride};
  return launch_iface_prods<T>(ps, np, L, nrhs, mfma, st);
}
template hipError_t launch_iface_step<double>(const double2*, const double2*, const double2*, double2*, int, int,
                                              int, int, size_t, size_t, int, bool, hipStream_t, const double2*,
                                              const double2*, double2*);
template hipError_t launch_iface_step<float>(const float2*, const float2*, const float2*, float2*, int, int, int,
                                             int, size_t, size_t, int, bool, hipStream_t, const float2*,
                                             const float2*, float2*);



template <typename T>
hipError_t launch_couple(const SliceTables& P, int L, int b, const C<T>* Hm, const C<T>* Hp, const C<T>* lam,
                         const C<T>* mu, int nrhs, C<T>* f, int k0, int k1, hipStream_t st) {
  if (k1 <= k0) return hipSuccess;
  hipLaunchKernelGGL(k_couple<T>, dim3((L + 63) / 64, k1 - k0, (nrhs + 15) / 16), dim3(256), 0, st, P, L, b, Hm, Hp,
                     lam, mu, nrhs, f, k0, k1 - k0);
  return hipGetLastError();
}
template hipError_t launch_couple<double>(const SliceTables&, int, int, const double2*, const double2*,
                                          const double2*, const double2*, int, double2*, int, int, hipStream_t);
template hipError_t launch_couple<float>(const SliceTables&, int, int, const float2*, const float2*, const float2*,
                                         const float2*, int, float2*, int, int, hipStream_t);

}  // namespace lsw
