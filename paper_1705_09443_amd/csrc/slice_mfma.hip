// Slice solves for batches of right-hand sides on the matrix cores.
//
// The block elimination of a slice subproblem (eq. Hwv_approx, factored at
// setup into W_j = S_j^{-1} B_j, the columns of S_j^{-1} on the lines of D_k,
// and G_j = S_j^{-1} C_j) is, for a batch of right-hand sides, a chain of
// small dense products:
//   forward   Y_j = S_j^{-1}[:, D_k] R_j - W_j Y_{j-1}       (j = 0 .. L-1)
//   backward  X_j = Y_j - G_j X_{j+1}                         (j = L-2 .. 0)
// with Y_j, X_j of t rows and one column per right-hand side. A wave owns 16
// columns and computes each step as 16x16x4 MFMAs (complex = four real
// products), with t padded to 16 or 32 rows.
//
// The dependent operand never moves. An MFMA leaves element i of lane l at
// row rowof(l / 16, i) of its 16-row output; in the i-th MFMA of a 16-wide
// contraction block the same lane supplies contraction index rowof(l / 16, i)
// of the other operand. So Y_{j-1}'s registers are the next step's B operand
// as they stand, and W_j, G_j are stored with their columns in that order
// (negated, so that every product accumulates). One forward or backward step
// is then loads issued PF steps ahead, the MFMAs, and the stores.
#include "kernels.hpp"

namespace lsw {

namespace {

template <typename T>
struct MF;
template <>
struct MF<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __attribute__((always_inline)) v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int rowof(int g, int i) { return 4 * g + i; }
};
template <>
struct MF<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __attribute__((always_inline)) v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int rowof(int g, int i) { return 4 * i + g; }
};

// complex values of one step's forward record (W blocks, then the
// S_j^{-1}[:, D_k] chunks of 4 columns) and backward record (G blocks)
__host__ __device__ inline int mfma_wrec(int rt, int nsd) { return rt * rt * 256 + rt * nsd * 64; }
__host__ __device__ inline int mfma_grec(int rt) { return rt * rt * 256; }

// Re-lay slice k's factors of one precision into operand order.
template <typename T>
__global__ void k_mfma_factors(SliceTables P, int L, int k, int rt, int nsd, const C<T>* __restrict__ FS,
                               const C<T>* __restrict__ FG, C<T>* __restrict__ MW, C<T>* __restrict__ MG) {
  const int wrec = mfma_wrec(rt, nsd), grec = mfma_grec(rt), per = wrec + grec;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)L * per) return;
  const int j = (int)(e / per), w = (int)(e % per);
  const int lo = P.lo[k], hi = P.hi[k], t = P.t[k];
  const int tw = hi - lo + 1;
  const C<T>* fs = FS + P.fs_off[k] + (size_t)j * factor_stride(t, tw);
  const C<T>* fg = FG + P.fg_off[k] + (size_t)j * factor_stride(t, 0);
  if (w < rt * rt * 256 || w >= wrec) {
    const bool isG = w >= wrec;
    const int e2 = isG ? w - wrec : w;
    const int blk = e2 / 256, l = (e2 / 4) % 64, i = e2 % 4;
    const int row = (blk / rt) * 16 + (l & 15), col = (blk % rt) * 16 + MF<T>::rowof(l >> 4, i);
    C<T> v = mk<T>(0, 0);
    if (row < t && col < t) {
      const C<T> f = isG ? fg[row * t + col] : fs[row * t + col];
      v = mk<T>(-f.x, -f.y);
    }
    if (isG)
      MG[(size_t)j * grec + e2] = v;
    else
      MW[(size_t)j * wrec + e2] = v;
  } else {
    const int e2 = w - rt * rt * 256;
    const int r = e2 / (nsd * 64), cc = (e2 / 64) % nsd, l = e2 % 64;
    const int row = r * 16 + (l & 15), col = 4 * cc + (l >> 4);
    MW[(size_t)j * wrec + w] = (row < t && col < tw) ? fs[t * t + row * tw + col] : mk<T>(0, 0);
  }
}

template <typename T>
__device__ __attribute__((always_inline)) inline void ld4(const C<T>* p, C<T>* o) {
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = p[i];
}

// One 16-column tile of slice k: RT row tiles of 16, NSD chunks of 4
// right-hand-side lines, PF steps of loads in flight. UNIT: the right-hand
// sides are columns of J_F Hm_k or J_E Hp_k (setup of the interface maps).
// Source and destination addresses are fixed per lane up front, so a step is
// straight-line code: loads, MFMAs, selects and (masked) stores.
// One complex 16x16x4 block a * x accumulated in Karatsuba's form: with
// a = A + iB and x = c + id, q1 += A (c + d), q2 += (A + B) d, q3 += (B - A) c,
// so that Re = q1 - q2 and Im = q1 + q3 (three real MFMAs instead of four).
// s = c + d is passed in, shared by the blocks that use the same x.
template <typename T>
__device__ __attribute__((always_inline)) inline void cmac(C<T> a, T c, T d, T s, typename MF<T>::v4& q1,
                                                           typename MF<T>::v4& q2, typename MF<T>::v4& q3) {
  q1 = MF<T>::op(a.x, s, q1);
  q2 = MF<T>::op(a.x + a.y, d, q2);
  q3 = MF<T>::op(a.y - a.x, c, q3);
}

template <typename T, int RT, int NSD, int PF, bool UNIT>
__device__ __attribute__((always_inline)) inline void mfma_body(const SliceMfmaArgs<T>& A, int k, int q, int nq) {
  using V = typename MF<T>::v4;
  constexpr int WREC = RT * RT * 256 + RT * NSD * 64, GREC = RT * RT * 256;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int L = A.L, b = A.b;
  const int lo = A.P.lo[k], hi = A.P.hi[k], t = A.P.t[k];
  const int naux = A.P.naux[k], tw = hi - lo + 1, org = A.P.org[k], dir = A.P.dir[k];
  const int n = q * 16 + li;
  const bool valid = n < A.nrhs;
  const int nc = valid ? n : A.nrhs - 1;  // loads of padding columns read a real one
  const C<T>* mw = A.MW + A.mw_off[k];
  const C<T>* mg = A.MG + A.mg_off[k];
  // forward results Y_j as the MFMA leaves them: per row tile and step, a
  // lane's 8 values (Re, then Im) in 16-byte chunks, chunk c of every lane
  // side by side, so that each 16-byte access of the wave covers one
  // contiguous kilobyte (whole cache lines) and not every other 16 bytes
  // of two kilobytes
  T* ys = A.yscr + ((size_t)A.ys_unit[k] * nq + (size_t)q * RT) * (size_t)(L + 1) * 512;
  constexpr int ychw = 16 / (int)sizeof(T);  // values per chunk
  auto ych = [&](int i) { return ((i / ychw) * 64 + lane) * ychw; };

  // right-hand sides: chunk cc of this lane holds line 4 cc + g of column nc
  const C<T>* rp[NSD];
  bool rok[NSD];
  const int col = A.col0 + nc;
  const C<T>* hrow = A.src_kind == kSrcUnitF ? A.Hm : A.Hp;
  const bool uline = UNIT && valid && g == (A.src_kind == kSrcUnitF ? 0 : (tw - 1) % 4);
  const int ucc = UNIT ? (A.src_kind == kSrcUnitF ? 0 : (tw - 1) / 4) : 0;
#pragma unroll
  for (int cc = 0; cc < NSD; ++cc) {
    const int line = 4 * cc + g;
    const int lc = line < tw ? line : tw - 1;
    rok[cc] = valid && line < tw;
    // D_k's local line lc: grid line org + dir (naux + lc); in a slice array
    // (grid order) row lc, or tw - 1 - lc against x1
    rp[cc] = UNIT ? hrow + (size_t)k * L * 3
                  : A.src + (A.src_kind == kSrcGrid ? (size_t)(org + dir * (naux + lc) + b) * L * A.nrhs + nc
                                                    : ((size_t)nc * tw + (dir > 0 ? lc : tw - 1 - lc)) * L);
  }
  // step stride along j of the right-hand sides: the interleaved grid holds
  // nrhs values per point
  const size_t rjs = A.src_kind == kSrcGrid ? (size_t)A.nrhs : 1;
  auto rhs = [&](int cc, int j) -> C<T> {
    if (UNIT) {
      // the unit source column col has 3 coefficients on one line, rows col-1..col+1
      const int dj = col - j;
      const bool ok = uline && cc == ucc && dj >= -1 && dj <= 1;
      const C<T> v = rp[cc][(size_t)j * 3 + (dj < -1 ? 0 : dj > 1 ? 2 : dj + 1)];
      return ok ? v : mk<T>(0, 0);
    }
    const C<T> v = rp[cc][(size_t)j * rjs];
    return rok[cc] ? v : mk<T>(0, 0);
  };

  // outputs: per row held by this lane, the byte offsets of its destination
  // in the E (or only) and F buffers (lines mode may send one row to both)
  // and their step strides. A row with no destination has an offset past the
  // buffers' size and stride 0: the range-checked store drops it, so the
  // steps store with no branch.
  constexpr int kNone = -16;  // 0xfffffff0 as the hardware's unsigned offset
  const int cs = (int)sizeof(C<T>);
  int op[RT][4], oq[RT][4], sp[RT][4], sq[RT][4];
  const C<T>* bp = A.dst;
  const C<T>* bq = A.dst;
  {
    const bool lines = A.dst_kind == kDstLines;
    const size_t ci = UNIT ? (size_t)(A.col0 + n) : (size_t)n;
    // grid mode: offsets from the lowest grid line of D_k
    const int lmin = org + b + (dir > 0 ? naux : dir * (naux + tw - 1));
    if (A.dst_kind == kDstGrid) bp = A.dst + (size_t)lmin * L * A.nrhs;
    if (lines) {
      if (A.dstE) bp = A.dstE + k * A.sk;
      if (A.dstF) bq = A.dstF + k * A.sk;
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = r * 16 + MF<T>::rowof(g, i);
        int o0 = kNone, o1 = kNone, s0 = 0, s1 = 0;
        if (valid && a < t) {
          const bool inD = a >= naux && a < naux + tw;
          if (A.dst_kind == kDstGrid) {
            if (inD) {
              o0 = (((org + dir * a + b) - lmin) * L * A.nrhs + n) * cs;
              s0 = A.nrhs * cs;
            }
          } else if (A.dst_kind == kDstSlice) {
            if (inD) {
              o0 = ((n * tw + (dir > 0 ? a - naux : tw - 1 - (a - naux))) * L) * cs;
              s0 = cs;
            }
          } else {
            if (a == naux + tw - 1 && A.dstE) {
              o0 = (int)(ci * A.sr) * cs;
              s0 = (int)A.sj * cs;
            }
            if (a == naux && A.dstF) {
              o1 = (int)(ci * A.sr) * cs;
              s1 = (int)A.sj * cs;
            }
          }
        }
        op[r][i] = o0;
        oq[r][i] = o1;
        sp[r][i] = s0;
        sq[r][i] = s1;
      }
  }
  const __amdgpu_buffer_rsrc_t rsp = __builtin_amdgcn_make_buffer_rsrc(const_cast<C<T>*>(bp), 0, 0x7fffffff, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsq = __builtin_amdgcn_make_buffer_rsrc(const_cast<C<T>*>(bq), 0, 0x7fffffff, 0x00020000);
  const bool twoq = A.dst_kind == kDstLines && A.dstF;
  auto emit = [&](int j, const V* xR, const V* xI) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const C<T> x = mk<T>(xR[r][i], xI[r][i]);
        store_or_drop<T>(rsp, op[r][i] + j * sp[r][i], x);
        if (twoq) store_or_drop<T>(rsq, oq[r][i] + j * sq[r][i], x);
      }
  };

  V pR[RT], pI[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) pR[r] = pI[r] = V{0, 0, 0, 0};

  // ---------------- forward ----------------
  {
    C<T> wv[PF][RT * RT][4], sv[PF][RT][NSD], rv[PF][NSD];
    auto load = [&](int s, int j) {
      const int jc = j < L ? j : L - 1;
      const C<T>* rec = mw + (size_t)jc * WREC;
#pragma unroll
      for (int blk = 0; blk < RT * RT; ++blk) ld4<T>(rec + blk * 256 + lane * 4, wv[s][blk]);
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int cc = 0; cc < NSD; ++cc) sv[s][r][cc] = rec[RT * RT * 256 + (r * NSD + cc) * 64 + lane];
#pragma unroll
      for (int cc = 0; cc < NSD; ++cc) rv[s][cc] = rhs(cc, jc);
    };
#pragma unroll
    for (int s = 0; s < PF; ++s) load(s, s);
    for (int j0 = 0; j0 < L; j0 += PF) {
#pragma unroll
      for (int s = 0; s < PF; ++s) {
        const int j = j0 + s;
        if (j < L) {
          // complex products in Karatsuba's form (three real MFMAs, see cmac)
          V q1[RT], q2[RT], q3[RT];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            q1[r] = q2[r] = q3[r] = V{0, 0, 0, 0};
#pragma unroll
            for (int cc = 0; cc < NSD; ++cc) {
              const C<T> a = sv[s][r][cc], x = rv[s][cc];
              cmac<T>(a, x.x, x.y, x.x + x.y, q1[r], q2[r], q3[r]);
            }
          }
#pragma unroll
          for (int kt = 0; kt < RT; ++kt) {
            const V ps = pR[kt] + pI[kt];
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
              for (int i = 0; i < 4; ++i)  // stored as -W
                cmac<T>(wv[s][r * RT + kt][i], pR[kt][i], pI[kt][i], ps[i], q1[r], q2[r], q3[r]);
          }
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            V aR = q1[r] - q2[r], aI = q1[r] + q3[r];
            pR[r] = aR;
            pI[r] = aI;
            T* yp = ys + ((size_t)j * RT + r) * 512;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              yp[ych(i) + i % ychw] = aR[i];
              yp[ych(4 + i) + i % ychw] = aI[i];
            }
          }
        }
        load(s, j + PF);
      }
    }
  }

  // ---------------- backward ----------------
  emit(L - 1, pR, pI);
  {
    constexpr int PB = PF;
    C<T> gv[PB][RT * RT][4];
    T yv[PB][RT][8];
    auto load = [&](int s, int j) {
      const int jc = j >= 0 ? j : 0;
      const C<T>* rec = mg + (size_t)jc * GREC;
#pragma unroll
      for (int blk = 0; blk < RT * RT; ++blk) ld4<T>(rec + blk * 256 + lane * 4, gv[s][blk]);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const T* yp = ys + ((size_t)jc * RT + r) * 512;
#pragma unroll
        for (int i = 0; i < 8; ++i) yv[s][r][i] = yp[ych(i) + i % ychw];
      }
    };
    // X_j = Y_j - G_j X_{j+1} from ring slot s
    auto step = [&](int s, int j) {
      // start from Y_j: Re = q1 - q2 = Re Y, Im = q1 + q3 = Im Y
      V q1[RT], q2[RT], q3[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        q1[r] = V{0, 0, 0, 0};
        q2[r] = -V{yv[s][r][0], yv[s][r][1], yv[s][r][2], yv[s][r][3]};
        q3[r] = V{yv[s][r][4], yv[s][r][5], yv[s][r][6], yv[s][r][7]};
      }
#pragma unroll
      for (int kt = 0; kt < RT; ++kt) {
        const V ps = pR[kt] + pI[kt];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i)  // stored as -G
            cmac<T>(gv[s][r * RT + kt][i], pR[kt][i], pI[kt][i], ps[i], q1[r], q2[r], q3[r]);
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        pR[r] = q1[r] - q2[r];
        pI[r] = q1[r] + q3[r];
      }
      emit(j, pR, pI);
    };
    // steps L-2 .. 0: whole groups of PB with no branch inside, then the
    // remaining steps, already loaded by the last group
    const int full = (L - 1) / PB * PB;
#pragma unroll
    for (int s = 0; s < PB; ++s) load(s, L - 2 - s);
    for (int j0 = L - 2; j0 > L - 2 - full; j0 -= PB) {
#pragma unroll
      for (int s = 0; s < PB; ++s) {
        step(s, j0 - s);
        load(s, j0 - s - PB);
      }
    }
#pragma unroll
    for (int s = 0; s < PB - 1; ++s)
      if (L - 2 - full - s >= 0) step(s, L - 2 - full - s);
  }
}

// steps of loads in flight (one wave per SIMD leaves the whole register file)
template <typename T>
constexpr int pf16 = sizeof(T) == 4 ? 8 : 4;
template <typename T>
constexpr int pf32 = sizeof(T) == 4 ? 4 : 2;

// blockIdx.x: group of 4 column tiles (one per wave); blockIdx.y: slice, the
// last of the range first (the 32-line class, the longest solve).
template <typename T, bool UNIT>
__global__ __launch_bounds__(256) void k_slice_mfma(SliceMfmaArgs<T> A) {
  const int nq = (A.nrhs + 15) / 16;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int k = A.slice0 + (int)gridDim.y - 1 - (int)blockIdx.y;
  const int nsd = A.nsd[k];
  if (A.P.t[k] > 16) {
    if (nsd <= 5)
      mfma_body<T, 2, 5, pf32<T>, UNIT>(A, k, q, nq);
    else
      mfma_body<T, 2, 8, pf32<T>, UNIT>(A, k, q, nq);
  } else {
    switch (nsd) {
      case 1: mfma_body<T, 1, 1, pf16<T>, UNIT>(A, k, q, nq); break;
      case 2: mfma_body<T, 1, 2, pf16<T>, UNIT>(A, k, q, nq); break;
      case 3: mfma_body<T, 1, 3, pf16<T>, UNIT>(A, k, q, nq); break;
      default: mfma_body<T, 1, 4, pf16<T>, UNIT>(A, k, q, nq); break;
    }
  }
}

}  // namespace

int mfma_row_tiles(int t) { return t > 16 ? 2 : 1; }
int mfma_chunks(int t, int tw) {
  const int c = (tw + 3) / 4;
  if (t > 16) return c <= 5 ? 5 : 8;
  return c;
}
size_t mfma_wrec_elems(int t, int tw) { return mfma_wrec(mfma_row_tiles(t), mfma_chunks(t, tw)); }
size_t mfma_grec_elems(int t) { return mfma_grec(mfma_row_tiles(t)); }

template <typename T>
hipError_t launch_mfma_factors(const SliceTables& P, int L, int k, int t, int tw, const C<T>* FS, const C<T>* FG,
                               C<T>* MW, C<T>* MG, hipStream_t st) {
  const int rt = mfma_row_tiles(t), nsd = mfma_chunks(t, tw);
  const size_t total = (size_t)L * (mfma_wrec(rt, nsd) + mfma_grec(rt));
  hipLaunchKernelGGL(k_mfma_factors<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, L, k, rt, nsd, FS,
                     FG, MW, MG);
  return hipGetLastError();
}
template hipError_t launch_mfma_factors<double>(const SliceTables&, int, int, int, int, const double2*,
                                                const double2*, double2*, double2*, hipStream_t);
template hipError_t launch_mfma_factors<float>(const SliceTables&, int, int, int, int, const float2*, const float2*,
                                               float2*, float2*, hipStream_t);

template <typename T>
hipError_t launch_slice_mfma(const SliceMfmaArgs<T>& a, int nslices, hipStream_t st) {
  const int nq = (a.nrhs + 15) / 16;
  // the output stores address a slice's lines (at most 32, plus the column
  // and step terms) with 32-bit byte offsets
  if ((size_t)34 * a.L * a.nrhs * sizeof(C<T>) >= ((size_t)1 << 31) - 4096) return hipErrorInvalidValue;
  if (a.src_kind >= kSrcUnitF)
    hipLaunchKernelGGL((k_slice_mfma<T, true>), dim3((nq + 3) / 4, nslices), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_slice_mfma<T, false>), dim3((nq + 3) / 4, nslices), dim3(256), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_slice_mfma<double>(const SliceMfmaArgs<double>&, int, hipStream_t);
template hipError_t launch_slice_mfma<float>(const SliceMfmaArgs<float>&, int, hipStream_t);

}  // namespace lsw
