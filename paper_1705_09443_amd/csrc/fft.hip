// FFT convolution with the Green's-function table (Sec. 2.1: the uniform
// grid lets the Nystrom sum of eq. LS_d be evaluated by FFT).
//
// y = a x + c * crop_I IFFT2( khat .* FFT2( pad_P(s .* x) ) ),   P = 2^k >= 2(n+1),
// with s = m (A-apply and incident right-hand side) or 1 (K-apply).
// khat = FFT2 of the table wrapped to P x P; the table is even in each axis,
// so only the (P/2+1)^2 quadrant of khat is stored.
//
// Three passes over HBM, each an LDS-resident Stockham FFT of S sequences:
//   row pass      S input rows of length n -> zero-padded length-P FFTs ->
//                 tiled buffer X[P/S][n][S] (an S x S block per tile is contiguous)
//   column pass   one tile: S columns of n rows, zero-padded, FFT, times khat,
//                 inverse FFT, first n rows written back in place
//   inverse rows  S rows gathered from the tiles, inverse FFT, first n entries,
//                 epilogue a x + c/P^2 (.) written to y
// Only the n nonzero input rows are transformed by the row pass and only the
// n needed output rows leave the column pass.
#include "kernels.hpp"

namespace lsw {

namespace {

// In-place Stockham FFT of nseq interleaved sequences in LDS: element k of
// sequence s lives at buf[k * nseq + s]. Radix-16 passes while 16 divides the
// remaining length, then one radix-8, -4 or -2 pass; each butterfly's DFT is
// done in registers. twl (LDS) holds w^k = exp(-2 pi i k / P), k < P; the
// inverse uses the conjugate (unnormalised).
// complex values a thread holds per pass (16: one radix-16 butterfly)
template <typename T>
constexpr int kVals = 16;
constexpr int kFftMaxThreads = 512;

// x * (-i) forward, x * (+i) inverse
template <typename T>
__device__ __attribute__((always_inline)) inline C<T> rot90(C<T> x, bool inv) {
  return inv ? mk<T>(-x.y, x.x) : mk<T>(x.y, -x.x);
}
template <typename T>
__device__ __attribute__((always_inline)) inline void dft2(C<T>& a, C<T>& b) {
  const C<T> t = a;
  a = cadd<T>(t, b);
  b = csub<T>(t, b);
}
// in-place 4-point DFT of x[0], x[s], x[2s], x[3s]
template <typename T>
__device__ __attribute__((always_inline)) inline void dft4(C<T>* x, int s, bool inv) {
  const C<T> a0 = cadd<T>(x[0], x[2 * s]), a1 = csub<T>(x[0], x[2 * s]);
  const C<T> a2 = cadd<T>(x[s], x[3 * s]), a3 = rot90<T>(csub<T>(x[s], x[3 * s]), inv);
  x[0] = cadd<T>(a0, a2);
  x[2 * s] = csub<T>(a0, a2);
  x[s] = cadd<T>(a1, a3);
  x[3 * s] = csub<T>(a1, a3);
}
// exp(-+ 2 pi i m / 16), m = 0..15, for the internal twiddles of the
// radix-8/16 DFTs (cos and sin of m pi / 8 from cos(pi/8), sin(pi/8), 1/sqrt 2)
template <typename T>
__device__ __attribute__((always_inline)) inline C<T> w16(int m, bool inv) {
  constexpr double a = 0.92387953251128675613, b = 0.38268343236508977173, h = 0.70710678118654752440;
  constexpr double cs[16] = {1, a, h, b, 0, -b, -h, -a, -1, -a, -h, -b, 0, b, h, a};
  constexpr double sn[16] = {0, b, h, a, 1, a, h, b, 0, -b, -h, -a, -1, -a, -h, -b};
  return mk<T>((T)cs[m & 15], inv ? (T)sn[m & 15] : (T)-sn[m & 15]);
}
// in-place R-point DFT of x[0..R) in natural order (R = 2, 4, 8, 16)
template <typename T, int R>
__device__ __attribute__((always_inline)) inline void dft(C<T>* x, bool inv) {
  if constexpr (R == 2) {
    dft2<T>(x[0], x[1]);
  } else if constexpr (R == 4) {
    dft4<T>(x, 1, inv);
  } else if constexpr (R == 8) {
    // n = 2a + b: 4-point DFTs over a, twiddles w8^(b c), 2-point DFTs over b
    dft4<T>(x, 2, inv);
    dft4<T>(x + 1, 2, inv);
#pragma unroll
    for (int c = 1; c < 4; ++c) x[2 * c + 1] = cmul<T>(x[2 * c + 1], w16<T>(2 * c, inv));
    C<T> y[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      C<T> a = x[2 * c], b = x[2 * c + 1];
      dft2<T>(a, b);
      y[c] = a;
      y[c + 4] = b;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = y[k];
  } else {
    // n = 4a + b: 4-point DFTs over a, twiddles w16^(b c), 4-point DFTs over b
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4<T>(x + b, 4, inv);
#pragma unroll
    for (int b = 1; b < 4; ++b)
#pragma unroll
      for (int c = 1; c < 4; ++c) x[4 * c + b] = cmul<T>(x[4 * c + b], w16<T>(b * c, inv));
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4<T>(x + 4 * c, 1, inv);
    // element (c, d) sits at 4 c + d and is output c + 4 d: transpose
    C<T> y[16];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int d = 0; d < 4; ++d) y[c + 4 * d] = x[4 * c + d];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = y[k];
  }
}

// log2 of a power of two
__device__ __attribute__((always_inline)) inline int ilog2(int v) { return __builtin_ctz((unsigned)v); }
template <int R>
constexpr int kLog2 = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;

// P, nseq and Ns are powers of two: the index arithmetic is shifts and masks
template <typename T, int R, bool inv>
__device__ __attribute__((always_inline)) inline void lds_fft_pass(C<T>* buf, int P, int nseq, int Ns,
                                                                   const C<T>* twl) {
  constexpr int NB = kVals<T> / R;  // butterflies per thread
  constexpr int LR = kLog2<R>;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ls = ilog2(nseq), ln = ilog2(Ns), lstep = ilog2(P) - ln - LR;
  const int nbf = P >> LR;
  const int total = nbf << ls;
  C<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bidx = tid + q * nt;
    if (bidx < total) {
      const int s = bidx & (nseq - 1), j = bidx >> ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[((j + r * nbf) << ls) + s];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bidx = tid + q * nt;
    if (bidx >= total) continue;
    const int s = bidx & (nseq - 1), j = bidx >> ls;
    const int k = j & (Ns - 1);
    const int step = k << lstep;  // k P / (Ns R)
    C<T>* x = v[q];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      C<T> w = twl[r * step];
      if (inv) w.y = -w.y;
      x[r] = cmul<T>(x[r], w);
    }
    dft<T, R>(x, inv);
    const int idxD = ((j >> ln) << (ln + LR)) + k;  // (j / Ns) Ns R + k
#pragma unroll
    for (int r = 0; r < R; ++r) buf[((idxD + r * Ns) << ls) + s] = x[r];
  }
  __syncthreads();
}

// In-place FFT of nseq interleaved length-P sequences (P a power of two);
// twl: the length-P twiddle table in LDS. Needs blockDim.x >= nseq * P / kVals<T>.
template <typename T, bool inv>
__device__ __attribute__((always_inline)) inline void lds_fft(C<T>* buf, int P, int nseq, const C<T>* twl) {
  int Ns = 1;
  for (; P / Ns >= 16; Ns *= 16) lds_fft_pass<T, 16, inv>(buf, P, nseq, Ns, twl);
  const int rem = P / Ns;
  if (rem == 8) lds_fft_pass<T, 8, inv>(buf, P, nseq, Ns, twl);
  else if (rem == 4) lds_fft_pass<T, 4, inv>(buf, P, nseq, Ns, twl);
  else if (rem == 2) lds_fft_pass<T, 2, inv>(buf, P, nseq, Ns, twl);
}

// the twiddle table into LDS (no barrier: the caller's next one covers it);
// P <= kVals * blockDim.x, all of a thread's loads in flight at once
template <typename T>
__device__ inline void load_twiddles(C<T>* twl, const C<T>* __restrict__ tw, int P) {
  constexpr int V = kVals<T>;
  C<T> v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    v[q] = tw[i < P ? i : 0];
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    if (i < P) twl[i] = v[q];
  }
}

// Element i of a complex grid in device memory, read or written through a
// global-address-space pointer: grids named by pointer tables would otherwise
// be reached with flat loads and stores.
template <typename T>
__device__ __attribute__((always_inline)) inline C<T> gld(const C<T>* p, size_t i) {
  using G = const __attribute__((address_space(1))) T;
  const G* q = (const G*)p;
  return mk<T>(q[2 * i], q[2 * i + 1]);
}
template <typename T>
__device__ __attribute__((always_inline)) inline void gst(C<T>* p, size_t i, C<T> v) {
  using G = __attribute__((address_space(1))) T;
  G* q = (G*)p;
  q[2 * i] = v.x;
  q[2 * i + 1] = v.y;
}

// Global <-> LDS copies: every thread moves at most kVals elements; the
// loops are unrolled with clamped, unconditional loads (values masked after)
// so that all of a thread's loads are in flight before the first is used.

// S rows of (s .* x) [+ zero padding to P] into buf (k * S + s)
template <typename T, bool HASM>
__device__ __attribute__((always_inline)) inline void load_rows(C<T>* buf, const C<T>* __restrict__ xr,
                                                                const T* __restrict__ m, int n, int P, int S,
                                                                int i0) {
  constexpr int V = kVals<T>;
  const int total = S * P, lP = ilog2(P);
  C<T> v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx >> lP, k = idx & (P - 1), row = i0 + sq;
    const bool ok = idx < total && k < n && row < n;
    const size_t o = (size_t)(row < n ? row : n - 1) * n + (k < n ? k : n - 1);
    C<T> w = gld<T>(xr, o);
    if (HASM) w = cscale<T>(w, m[o]);
    v[q] = ok ? w : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) buf[(idx & (P - 1)) * S + (idx >> lP)] = v[q];
  }
}

// ---- pass 1: rows of (s .* x), zero-padded to P -----------------------------
// xp: right-hand side r read from the grid xp[r] instead of x
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k_row_forward(const C<T>* __restrict__ x, const T* __restrict__ m, int n, int P,
                              int S, const C<T>* __restrict__ tw, C<T>* __restrict__ X,
                              const C<T>* const* __restrict__ xp) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int rhs = blockIdx.y;
  const int i0 = blockIdx.x * S;
  const size_t nn = (size_t)n * n;
  const C<T>* xr = xp ? xp[rhs] : x + rhs * nn;
  if (m)
    load_rows<T, true>(buf, xr, m, n, P, S, i0);
  else
    load_rows<T, false>(buf, xr, m, n, P, S, i0);
  __syncthreads();
  lds_fft<T, false>(buf, P, S, twl);
  const int ntile = P / S;
  C<T>* Xr = X + (size_t)rhs * ntile * n * S;
  const int lS = ilog2(S);
#pragma unroll
  for (int q = 0; q < kVals<T>; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int tile = idx >> (2 * lS), within = idx & (S * S - 1);
    const int sq = within >> lS, kk = within & (S - 1);
    const int row = i0 + sq;
    if (idx < S * P && row < n) Xr[((size_t)tile * n + row) * S + kk] = buf[(tile * S + kk) * S + sq];
  }
}

// ---- pass 2: columns, times khat, inverse columns ------------------------
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k_col_convolve(C<T>* __restrict__ X, const C<T>* __restrict__ khat, int n, int P,
                               int S, const C<T>* __restrict__ tw) {
  constexpr int V = kVals<T>;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int tile = blockIdx.x, rhs = blockIdx.y;
  const int ntile = P / S;
  const int total = S * P, live = S * n;
  C<T>* Xt = X + ((size_t)rhs * ntile + tile) * n * S;
  {
    C<T> v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      const C<T> w = Xt[idx < live ? idx : 0];
      v[q] = idx < live ? w : mk<T>(0, 0);
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      if (idx < total) buf[idx] = v[q];
    }
  }
  __syncthreads();
  lds_fft<T, false>(buf, P, S, twl);
  // times khat: k depends on |delta| only, so khat is symmetric and column c
  // of the quadrant is its row c; consecutive threads walk along it
  {
    const int half = P / 2 + 1, lP = ilog2(P);
    C<T> kv[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      const int sq = idx >> lP, r = idx & (P - 1);
      const int col = tile * S + (idx < total ? sq : 0);
      const int kr = r <= P - r ? r : P - r;
      const int kc = col <= P - col ? col : P - col;
      kv[q] = khat[(size_t)kc * half + kr];
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      if (idx < total) {
        const int sq = idx >> lP, r = idx & (P - 1);
        buf[r * S + sq] = cmul<T>(buf[r * S + sq], kv[q]);
      }
    }
  }
  __syncthreads();
  lds_fft<T, true>(buf, P, S, twl);
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < live) Xt[idx] = buf[idx];
  }
}

// ---- pass 3: inverse rows and epilogue y = a x + coef * conv --------------
// W64: right-hand side r written, widened, to y64[r] instead of y
// xp: right-hand side r of x read from the grid xp[r]
template <typename T, bool W64>
__global__ __launch_bounds__(kFftMaxThreads) void k_row_inverse(const C<T>* __restrict__ X, const C<T>* __restrict__ x, int n, int P,
                              int S, const C<T>* __restrict__ tw, T a, T coef,
                              C<T>* __restrict__ y, double2* const* __restrict__ y64,
                              const C<T>* const* __restrict__ xp) {
  constexpr int V = kVals<T>;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int rhs = blockIdx.y;
  const int i0 = blockIdx.x * S;
  const int ntile = P / S;
  const int total = S * P;
  const C<T>* Xr = X + (size_t)rhs * ntile * n * S;
  const int lS = ilog2(S);
  {
    C<T> v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      const int tl = idx >> (2 * lS), within = idx & (S * S - 1);
      const int sq = within >> lS, kk = within & (S - 1);
      const int row = i0 + sq;
      const bool ok = idx < total && row < n;
      const C<T> w = Xr[ok ? ((size_t)tl * n + row) * S + kk : 0];
      v[q] = ok ? w : mk<T>(0, 0);
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      if (idx < total) {
        const int tl = idx >> (2 * lS), within = idx & (S * S - 1);
        buf[(tl * S + (within & (S - 1))) * S + (within >> lS)] = v[q];
      }
    }
  }
  __syncthreads();
  lds_fft<T, true>(buf, P, S, twl);
  const size_t nn = (size_t)n * n;
  const int live = S * n;
  const C<T>* xr = xp ? xp[rhs] : x + rhs * nn;
  C<T> xv[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / n, k = idx % n, row = i0 + sq;
    const bool ok = idx < live && row < n;
    xv[q] = a != T(0) ? gld<T>(xr, ok ? (size_t)row * n + k : 0) : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / n, k = idx % n, row = i0 + sq;
    if (idx < live && row < n) {
      const C<T> v = cadd<T>(cscale<T>(buf[k * S + sq], coef), cscale<T>(xv[q], a));
      if (W64)
        gst<double>(y64[rhs], (size_t)row * n + k, make_double2((double)v.x, (double)v.y));
      else
        y[rhs * nn + (size_t)row * n + k] = v;
    }
  }
}

// ---- transforms of a compile-time length ------------------------------------
// For P = 128 ... 4096 the passes are instantiated per length: the plan, the
// LDS offsets and the lane maps are constants, so the only index arithmetic
// left is a base address per butterfly. A thread owns butterfly j of
// sequence s in every pass (bidx = tid + q NT, s = bidx mod S, j = bidx / S),
// which gives two register-resident steps:
//  * the first pass (radix 16, stride P/16) takes its inputs straight from
//    device memory; with zero padding beyond n < P/2 its upper eight inputs
//    are zero and its first 4-point stage is halved;
//  * in the last pass (stride P/R) a thread's NB = 16/R butterflies are
//    j0 + q P/16, so it holds elements j0 + r' P/16, r' < 16: exactly the
//    inputs of the inverse transform's first pass. The column pass multiplies
//    them by the spectrum in registers and goes on without an LDS exchange.
// The twiddles of the pass with stride NS and radix R sit contiguously in
// LDS at NS - 1 + k (R - 1) + r - 1 (w^(r k P / (NS R)), k < NS, 1 <= r < R):
// P - 1 values for the whole plan.

constexpr int ct_radix(int P, int NS) { return P / NS >= 16 ? 16 : P / NS; }
constexpr int ct_log2(int v) { return v <= 1 ? 0 : 1 + ct_log2(v / 2); }
// rows per tile of the row transforms [P/S][ct_rows(n)][S]: n rounded up to
// a multiple of 8, so that every S x S block (S <= 8) starts a cache line
// (with n odd, half the tiles would otherwise straddle two lines per block)
__host__ __device__ constexpr int ct_rows(int n) { return (n + 7) & ~7; }

// the twiddles of every pass into LDS (the caller's next barrier covers them)
template <typename T, int P, int S>
__device__ __attribute__((always_inline)) inline void ct_twiddles(C<T>* twl, const C<T>* __restrict__ tw) {
  constexpr int NT = S * P / 16;
  constexpr int R2 = ct_radix(P, 16), R3 = P > 256 ? ct_radix(P, 256) : 2;
  for (int e = threadIdx.x; e < P - 1; e += NT) {
    int m = 0;  // entries of the first pass (stride 1) are never read
    if (e >= 15 && e < 16 * R2 - 1) {
      const int l = e - 15, k = l / (R2 - 1), r = l - k * (R2 - 1) + 1;
      m = r * k * (P / (16 * R2));
    }
    if constexpr (P > 256) {
      if (e >= 255) {
        const int l = e - 255, k = l / (R3 - 1), r = l - k * (R3 - 1) + 1;
        m = r * k * (P / (256 * R3));
      }
    }
    twl[e] = tw[m];
  }
}

// 16-point DFT (natural order) whose inputs 8..15 are zero: the first
// 4-point stage of the 4 x 4 decomposition has two inputs per transform
template <typename T, bool INV>
__device__ __attribute__((always_inline)) inline void dft16_low(C<T>* x) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const C<T> a0 = x[b], a1 = x[b + 4], ra = rot90<T>(a1, INV);
    x[b] = cadd<T>(a0, a1);
    x[b + 8] = csub<T>(a0, a1);
    x[b + 4] = cadd<T>(a0, ra);
    x[b + 12] = csub<T>(a0, ra);
  }
#pragma unroll
  for (int b = 1; b < 4; ++b)
#pragma unroll
    for (int c = 1; c < 4; ++c) x[4 * c + b] = cmul<T>(x[4 * c + b], w16<T>(b * c, INV));
#pragma unroll
  for (int c = 0; c < 4; ++c) dft4<T>(x + 4 * c, 1, INV);
  C<T> y[16];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = 0; d < 4; ++d) y[c + 4 * d] = x[4 * c + d];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = y[k];
}

// inputs of the pass of stride NS from LDS: butterfly (s, j) reads element
// j + r P/R of sequence s at (j + r P/R) S + s = bidx + r (P/R) S
template <typename T, int P, int S, int NS>
__device__ __attribute__((always_inline)) inline void ct_read(const C<T>* buf, C<T> (&v)[16]) {
  constexpr int R = ct_radix(P, NS), NB = 16 / R, NT = S * P / 16;
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) v[q * R + r] = buf[threadIdx.x + q * NT + r * (P / R) * S];
}

// twiddles and R-point DFTs of the pass of stride NS
template <typename T, int P, int S, int NS, bool INV>
__device__ __attribute__((always_inline)) inline void ct_bfly(const C<T>* twl, C<T> (&v)[16]) {
  constexpr int R = ct_radix(P, NS), NB = 16 / R, NT = S * P / 16, LS = ct_log2(S);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if constexpr (NS > 1) {
      const int k = ((threadIdx.x + q * NT) >> LS) & (NS - 1);
      const C<T>* w = twl + (NS - 1) + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) v[q * R + r] = INV ? cmulc<T>(v[q * R + r], w[r - 1]) : cmul<T>(v[q * R + r], w[r - 1]);
    }
    dft<T, R>(&v[q * R], INV);
  }
}

// outputs of the pass of stride NS to LDS: element (j / NS) NS R + k + r NS
template <typename T, int P, int S, int NS>
__device__ __attribute__((always_inline)) inline void ct_write(C<T>* buf, const C<T> (&v)[16]) {
  constexpr int R = ct_radix(P, NS), NB = 16 / R, NT = S * P / 16, LS = ct_log2(S);
  constexpr int LN = ct_log2(NS), LR = ct_log2(R);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bidx = threadIdx.x + q * NT, s = bidx & (S - 1), j = bidx >> LS;
    const int base = ((((j >> LN) << (LN + LR)) + (j & (NS - 1))) << LS) + s;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[base + r * NS * S] = v[q * R + r];
  }
}

// the passes after the first, from the LDS written by the first pass: every
// pass but the last writes LDS back; the last leaves its outputs in v
template <typename T, int P, int S, bool INV, int NS = 16>
__device__ __attribute__((always_inline)) inline void ct_rest(C<T>* buf, const C<T>* twl, C<T> (&v)[16]) {
  __syncthreads();
  ct_read<T, P, S, NS>(buf, v);
  ct_bfly<T, P, S, NS, INV>(twl, v);
  if constexpr (NS * ct_radix(P, NS) < P) {
    __syncthreads();
    ct_write<T, P, S, NS>(buf, v);
    ct_rest<T, P, S, INV, NS * 16>(buf, twl, v);
  }
}

// stride of the last pass and its radix
template <int P>
constexpr int ct_last_ns() { return P > 256 ? 256 : 16; }
template <int P>
constexpr int ct_last_radix() { return ct_radix(P, ct_last_ns<P>()); }

// last-pass registers (butterfly q, output r) -> first-pass registers of the
// next transform (element j0 + r' P/16 at r' = q + r NB)
template <typename T, int P>
__device__ __attribute__((always_inline)) inline void ct_regroup(C<T> (&v)[16]) {
  constexpr int R = ct_last_radix<P>(), NB = 16 / R;
  C<T> u[16];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) u[q + r * NB] = v[q * R + r];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = u[i];
}

// pass 1, rows: S rows of (s .* x) zero-padded to P, transformed, written as
// the tiles [P/S][n][S]
template <typename T, int P, int S, bool HASM>
__global__ __launch_bounds__(S * P / 16) void k_row_forward_ct(const C<T>* __restrict__ x, const T* __restrict__ m,
                                                              int n, const C<T>* __restrict__ tw,
                                                              C<T>* __restrict__ X, const C<T>* const* __restrict__ xp) {
  constexpr int LS = ct_log2(S), RL = ct_last_radix<P>(), NBL = 16 / RL;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  ct_twiddles<T, P, S>(twl, tw);
  const int rhs = blockIdx.y, i0 = blockIdx.x * S;
  const int s = threadIdx.x & (S - 1), j0 = threadIdx.x >> LS, row = i0 + s;
  const size_t nn = (size_t)n * n;
  const C<T>* xr = xp ? xp[rhs] : x + rhs * nn;
  C<T> v[16];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int c = j0 + r * (P / 16);
    const bool ok = row < n && c < n;
    const size_t o = ok ? (size_t)row * n + c : 0;
    C<T> w = gld<T>(xr, o);
    if (HASM) w = cscale<T>(w, m[o]);
    v[r] = ok ? w : mk<T>(0, 0);
  }
  dft16_low<T, false>(v);
  ct_write<T, P, S, 1>(buf, v);
  ct_rest<T, P, S, false>(buf, twl, v);
  // the last pass's outputs: frequency f = j0 + q P/16 + r P/RL of row i0 + s
  if (row < n) {
    const int np = ct_rows(n);
    C<T>* Xr = X + (size_t)rhs * (P / S) * np * S;
#pragma unroll
    for (int q = 0; q < NBL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int f = j0 + q * (P / 16) + r * (P / RL);
        Xr[((size_t)(f >> LS) * np + row) * S + (f & (S - 1))] = v[q * RL + r];
      }
  }
}

// pass 2, one tile of S columns (blockIdx.y) of right-hand side blockIdx.x:
// column FFT of the n live rows, times the spectrum, inverse column FFT, the
// n live rows written back in place
template <typename T, int P, int S>
__global__ __launch_bounds__(S * P / 16) void k_col_convolve_ct(C<T>* __restrict__ X, const C<T>* __restrict__ khat,
                                                               int n, const C<T>* __restrict__ tw) {
  constexpr int LS = ct_log2(S), RL = ct_last_radix<P>(), NBL = 16 / RL;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  ct_twiddles<T, P, S>(twl, tw);
  const int rhs = blockIdx.x, tile = blockIdx.y;
  const int s = threadIdx.x & (S - 1), j0 = threadIdx.x >> LS;
  C<T>* Xt = X + ((size_t)rhs * (P / S) + tile) * ct_rows(n) * S;
  const int live = n * S;
  // the spectrum values this thread multiplies by, loaded before the forward
  // transform so that their latency hides behind it: row frequency
  // f = j0 + r P/16; the spectrum is even in both indices, and its stored
  // quadrant is symmetric (column c is row c)
  C<T> kv[16];
  {
    constexpr int half = P / 2 + 1;
    const int c = tile * S + s, kc = c <= P - c ? c : P - c;
    const C<T>* kr = khat + (size_t)kc * half;
#pragma unroll
    for (int r = 0; r < 16; ++r) kv[r] = r < 8 ? kr[j0 + r * (P / 16)] : kr[P - j0 - r * (P / 16)];
  }
  C<T> v[16];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int idx = threadIdx.x + r * (P / 16) * S;  // row j0 + r P/16, column s
    const C<T> w = Xt[idx < live ? idx : 0];
    v[r] = idx < live ? w : mk<T>(0, 0);
  }
  dft16_low<T, false>(v);
  ct_write<T, P, S, 1>(buf, v);
  ct_rest<T, P, S, false>(buf, twl, v);
  ct_regroup<T, P>(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = cmul<T>(v[r], kv[r]);
  dft<T, 16>(v, true);
  __syncthreads();  // every read of the forward transform's last pass is done
  ct_write<T, P, S, 1>(buf, v);
  ct_rest<T, P, S, true>(buf, twl, v);
  // rows j0 + q P/16 + r P/RL; only r < RL/2 can be below n < P/2
#pragma unroll
  for (int q = 0; q < NBL; ++q)
#pragma unroll
    for (int r = 0; r < RL / 2; ++r) {
      const int idx = threadIdx.x + (q * (P / 16) + r * (P / RL)) * S;
      if (idx < live) Xt[idx] = v[q * RL + r];
    }
}

// pass 3: S rows gathered from the tiles, inverse FFT, first n entries,
// epilogue a x + coef (.) to y (or, widened, to y64[rhs])
template <typename T, int P, int S, bool W64>
__global__ __launch_bounds__(S * P / 16) void k_row_inverse_ct(const C<T>* __restrict__ X, const C<T>* __restrict__ x,
                                                              int n, const C<T>* __restrict__ tw, T a, T coef,
                                                              C<T>* __restrict__ y, double2* const* __restrict__ y64,
                                                              const C<T>* const* __restrict__ xp) {
  constexpr int LS = ct_log2(S), RL = ct_last_radix<P>(), NBL = 16 / RL;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  ct_twiddles<T, P, S>(twl, tw);
  const int rhs = blockIdx.y, i0 = blockIdx.x * S;
  const int s = threadIdx.x & (S - 1), j0 = threadIdx.x >> LS, row = i0 + s;
  const bool live = row < n;
  const int np = ct_rows(n);
  const C<T>* Xr = X + (size_t)rhs * (P / S) * np * S;
  C<T> v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int f = j0 + r * (P / 16);
    const C<T> w = Xr[live ? ((size_t)(f >> LS) * np + row) * S + (f & (S - 1)) : 0];
    v[r] = live ? w : mk<T>(0, 0);
  }
  // x at this thread's outputs, loaded before the transform: columns
  // j0 + q P/16 + r P/RL; only r < RL/2 can be below n < P/2
  const size_t nn = (size_t)n * n;
  const C<T>* xr = xp ? xp[rhs] : x + rhs * nn;
  C<T> xv[NBL][RL / 2];
#pragma unroll
  for (int q = 0; q < NBL; ++q)
#pragma unroll
    for (int r = 0; r < RL / 2; ++r) {
      const int c = j0 + q * (P / 16) + r * (P / RL);
      const bool ok = live && c < n && a != T(0);
      const C<T> w = gld<T>(xr, ok ? (size_t)row * n + c : 0);
      xv[q][r] = ok ? w : mk<T>(0, 0);
    }
  dft<T, 16>(v, true);
  ct_write<T, P, S, 1>(buf, v);
  ct_rest<T, P, S, true>(buf, twl, v);
  if (!live) return;
#pragma unroll
  for (int q = 0; q < NBL; ++q)
#pragma unroll
    for (int r = 0; r < RL / 2; ++r) {
      const int c = j0 + q * (P / 16) + r * (P / RL);
      if (c < n) {
        const size_t o = (size_t)row * n + c;
        C<T> w = cscale<T>(v[q * RL + r], coef);
        if (a != T(0)) w = cadd<T>(w, cscale<T>(xv[q][r], a));
        if (W64)
          gst<double>(y64[rhs], o, make_double2((double)w.x, (double)w.y));
        else
          y[rhs * nn + o] = w;
      }
    }
}

// ---- setup: khat = FFT2 of the wrapped table, quadrant kept ---------------
__global__ void k_wrap_table(const double2* __restrict__ kq, int n, int P, double2* __restrict__ W) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)P * P) return;
  const int q1 = (int)(idx / P), q2 = (int)(idx % P);
  const int d1 = q1 <= P / 2 ? q1 : P - q1;
  const int d2 = q2 <= P / 2 ? q2 : P - q2;
  // offsets beyond n+1 never reach the interior product; they are zero
  W[idx] = (d1 <= n + 1 && d2 <= n + 1) ? kq[(size_t)d1 * (n + 2) + d2] : make_double2(0.0, 0.0);
}

// In-place FFT of S full rows (stride P) of a P x P array.
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_rows_full(double2* __restrict__ W, int P, int S, const double2* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  double2* buf = reinterpret_cast<double2*>(smem_raw);
  double2* twl = buf + S * P;
  load_twiddles<double>(twl, tw, P);
  const int r0 = blockIdx.x * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int s = idx / P, k = idx % P;
    buf[k * S + s] = W[(size_t)(r0 + s) * P + k];
  }
  __syncthreads();
  lds_fft<double, false>(buf, P, S, twl);
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int s = idx / P, k = idx % P;
    W[(size_t)(r0 + s) * P + k] = buf[k * S + s];
  }
}

// In-place FFT of S full columns of a P x P array; quadrant written to khat.
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_cols_full(double2* __restrict__ W, int P, int S, const double2* __restrict__ tw,
                                double2* __restrict__ khat, float2* __restrict__ khat32) {
  extern __shared__ unsigned char smem_raw[];
  double2* buf = reinterpret_cast<double2*>(smem_raw);
  double2* twl = buf + S * P;
  load_twiddles<double>(twl, tw, P);
  const int c0 = blockIdx.x * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int r = idx / S, s = idx % S;
    buf[idx] = W[(size_t)r * P + c0 + s];
  }
  __syncthreads();
  lds_fft<double, false>(buf, P, S, twl);
  const int half = P / 2 + 1;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int r = idx / S, s = idx % S;
    const int c = c0 + s;
    if (r < half && c < half) {
      khat[(size_t)r * half + c] = buf[idx];
      khat32[(size_t)r * half + c] = make_float2((float)buf[idx].x, (float)buf[idx].y);
    }
  }
}

// ---- 3D convolution: five passes of length-P transforms -------------------
// Every pass loads S sequences into LDS as buf[t * S + s] (element t of
// sequence s), transforms them with lds_fft and stores them back. Pass 1 and
// 5 take S rows (contiguous); passes 2-4 take S consecutive k3 (contiguous in
// memory) of sequences along axis 2 or 1, so every global access moves S
// consecutive values.
//   x  [n][n][n] --1--> w1 [n][n][P] --2--> w2 [n][P][P] --3 (axis 1, khat,
//   inverse)--> w2 --4 (inverse axis 2)--> w1 --5 (inverse axis 3)--> y

// pass 1: S rows rho = i1 n + i2 of (s .* x), zero-padded to P, transformed
template <typename T, bool HASM>
__global__ __launch_bounds__(kFftMaxThreads) void k3_rows_fwd(const C<T>* __restrict__ x, const T* __restrict__ m,
                                                              int n, int P, int S, const C<T>* __restrict__ tw,
                                                              C<T>* __restrict__ w1) {
  constexpr int V = kVals<T>;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int rhs = blockIdx.y, r0 = blockIdx.x * S, rows = n * n;
  const size_t n3 = (size_t)rows * n;
  const C<T>* xr = x + rhs * n3;
  C<T> v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / P, k = idx % P, row = r0 + sq;
    const bool ok = idx < S * P && k < n && row < rows;
    const size_t o = (size_t)(row < rows ? row : rows - 1) * n + (k < n ? k : n - 1);
    C<T> w = xr[o];
    if (HASM) w = cscale<T>(w, m[o]);
    v[q] = ok ? w : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < S * P) buf[(idx % P) * S + idx / P] = v[q];
  }
  __syncthreads();
  lds_fft<T, false>(buf, P, S, twl);
  C<T>* out = w1 + (size_t)rhs * rows * P;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / P, k = idx % P, row = r0 + sq;
    if (idx < S * P && row < rows) out[(size_t)row * P + k] = buf[k * S + sq];
  }
}

// Where element t of sequence s of a workgroup lives: base + rhs * rhs_stride
// + blockIdx.y * oth + (blockIdx.x * S + s) * sst + t * st.
struct Seq3 {
  size_t st, sst, oth, rhs;
};

// passes 2-4: S sequences of nin inputs (the rest zero); MODE 0 forward, 1
// forward, times khat, inverse (axis 1), 2 inverse; nout outputs stored
// through out. blockIdx.x: chunk of S sequences, blockIdx.y: the other index
// (i1 for axis 2, k2 for axis 1), blockIdx.z: right-hand side.
template <typename T, int MODE>
__global__ __launch_bounds__(kFftMaxThreads) void k3_axis(const C<T>* __restrict__ src, C<T>* __restrict__ dst,
                                                          const C<T>* __restrict__ khat, int P, int S, int nin,
                                                          int nout, Seq3 si, Seq3 so, const C<T>* __restrict__ tw) {
  constexpr int V = kVals<T>;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int c0 = blockIdx.x * S, o = blockIdx.y, rhs = blockIdx.z;
  const C<T>* in = src + rhs * si.rhs + (size_t)o * si.oth + (size_t)c0 * si.sst;
  C<T> v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int t = idx / S, sq = idx % S;
    const bool ok = idx < S * P && t < nin;
    const C<T> w = in[ok ? (size_t)t * si.st + (size_t)sq * si.sst : 0];
    v[q] = ok ? w : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < S * P) buf[idx] = v[q];
  }
  __syncthreads();
  lds_fft<T, (MODE == 2)>(buf, P, S, twl);
  if (MODE == 1) {
    // times khat(k1 = t, k2 = o, k3 = c0 + sq), the table even in every axis
    const int H = P / 2 + 1;
    const int k2 = o <= P - o ? o : P - o;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      if (idx < S * P) {
        const int t = idx / S, c = c0 + idx % S;
        const int k1 = t <= P - t ? t : P - t, k3 = c <= P - c ? c : P - c;
        buf[idx] = cmul<T>(buf[idx], khat[((size_t)k1 * H + k2) * H + k3]);
      }
    }
    __syncthreads();
    lds_fft<T, true>(buf, P, S, twl);
  }
  C<T>* out = dst + rhs * so.rhs + (size_t)o * so.oth + (size_t)c0 * so.sst;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int t = idx / S, sq = idx % S;
    if (idx < S * P && t < nout) out[(size_t)t * so.st + (size_t)sq * so.sst] = buf[idx];
  }
}

// pass 5: S rows of w1, inverse transform, first n entries, epilogue
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k3_rows_inv(const C<T>* __restrict__ w1,
                                                              const C<T>* __restrict__ x, int n, int P, int S,
                                                              const C<T>* __restrict__ tw, T a, T coef,
                                                              C<T>* __restrict__ y) {
  constexpr int V = kVals<T>;
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  C<T>* twl = buf + S * P;
  load_twiddles<T>(twl, tw, P);
  const int rhs = blockIdx.y, r0 = blockIdx.x * S, rows = n * n;
  const C<T>* in = w1 + (size_t)rhs * rows * P;
  C<T> v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / P, k = idx % P, row = r0 + sq;
    const bool ok = idx < S * P && row < rows;
    const C<T> w = in[(size_t)(ok ? row : 0) * P + k];
    v[q] = ok ? w : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < S * P) buf[(idx % P) * S + idx / P] = v[q];
  }
  __syncthreads();
  lds_fft<T, true>(buf, P, S, twl);
  const size_t n3 = (size_t)rows * n;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    const int sq = idx / n, k = idx % n, row = r0 + sq;
    if (idx < S * n && row < rows) {
      const size_t o = rhs * n3 + (size_t)row * n + k;
      const C<T> xv = a != T(0) ? x[o] : mk<T>(0, 0);
      y[o] = cadd<T>(cscale<T>(buf[k * S + sq], coef), cscale<T>(xv, a));
    }
  }
}

// setup: the table octant wrapped to P^3 (zero beyond offset n+1)
__global__ void k3_wrap_table(const double2* __restrict__ kq, int n, int P, double2* __restrict__ W) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)P * P * P) return;
  const int q1 = (int)(idx / ((size_t)P * P)), q2 = (int)((idx / P) % P), q3 = (int)(idx % P);
  const int d1 = q1 <= P / 2 ? q1 : P - q1, d2 = q2 <= P / 2 ? q2 : P - q2, d3 = q3 <= P / 2 ? q3 : P - q3;
  const int Q = n + 2;
  W[idx] = (d1 < Q && d2 < Q && d3 < Q) ? kq[((size_t)d1 * Q + d2) * Q + d3] : make_double2(0.0, 0.0);
}

// setup: the octant of the transformed P^3 array
__global__ void k3_octant(const double2* __restrict__ W, int P, double2* __restrict__ khat,
                          float2* __restrict__ khat32) {
  const int H = P / 2 + 1;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)H * H * H) return;
  const int a = (int)(idx / ((size_t)H * H)), b = (int)((idx / H) % H), c = (int)(idx % H);
  const double2 v = W[((size_t)a * P + b) * P + c];
  khat[idx] = v;
  khat32[idx] = make_float2((float)v.x, (float)v.y);
}

template <typename T>
constexpr int seq_per_block(int P) {
  int S = (163840 - P * (int)sizeof(C<T>)) / (P * (int)sizeof(C<T>));
  if (S > 8) S = 8;
  if (S * P > kVals<T> * kFftMaxThreads) S = kVals<T> * kFftMaxThreads / P;
  if (S > P) S = P;
  if (S < 1) S = 1;
  return S;
}

template <typename T>
int threads_for(int S, int P) {
  int nt = S * P / kVals<T>;
  if (nt < 64) nt = 64;
  if (nt > kFftMaxThreads) nt = kFftMaxThreads;
  return nt;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

template <typename T>
size_t fft_work_elems(int n, int nrhs) {
  const int P = fft_len(n);
  return (size_t)nrhs * P * ct_rows(n);
}
template size_t fft_work_elems<double>(int, int);
template size_t fft_work_elems<float>(int, int);

template <typename T, int P>
hipError_t launch_convolve_ct(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat, const C<T>* tw, T a,
                              T coef, C<T>* work, C<T>* y, hipStream_t st, double2* const* y64,
                              const C<T>* const* xp) {
  constexpr int S = seq_per_block<T>(P), NT = S * P / 16;
  static_assert((S & (S - 1)) == 0 && NT >= 64 && NT <= kFftMaxThreads, "compile-time plan");
  const size_t lds = (size_t)(S + 1) * P * sizeof(C<T>);
  hipError_t e;
  if ((e = allow_lds(k_row_forward_ct<T, P, S, true>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_forward_ct<T, P, S, false>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_col_convolve_ct<T, P, S>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_inverse_ct<T, P, S, false>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_inverse_ct<T, P, S, true>, lds)) != hipSuccess) return e;
  // the column pass takes right-hand sides fastest: consecutive workgroups
  // read the same spectrum columns
  const dim3 grow((n + S - 1) / S, nrhs), gcol(nrhs, P / S);
  if (m)
    hipLaunchKernelGGL((k_row_forward_ct<T, P, S, true>), grow, dim3(NT), lds, st, x, m, n, tw, work, xp);
  else
    hipLaunchKernelGGL((k_row_forward_ct<T, P, S, false>), grow, dim3(NT), lds, st, x, m, n, tw, work, xp);
  hipLaunchKernelGGL((k_col_convolve_ct<T, P, S>), gcol, dim3(NT), lds, st, work, khat, n, tw);
  if (y64)
    hipLaunchKernelGGL((k_row_inverse_ct<T, P, S, true>), grow, dim3(NT), lds, st, work, x, n, tw, a, coef, y, y64,
                       xp);
  else
    hipLaunchKernelGGL((k_row_inverse_ct<T, P, S, false>), grow, dim3(NT), lds, st, work, x, n, tw, a, coef, y, y64,
                       xp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convolve(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat,
                           const C<T>* tw, T a, T c, C<T>* work, C<T>* y, hipStream_t st, double2* const* y64,
                           const C<T>* const* xp) {
  const int P = fft_len(n);
  const T coef_ct = c / ((T)P * (T)P);
  switch (P) {
    case 128: return launch_convolve_ct<T, 128>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    case 256: return launch_convolve_ct<T, 256>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    case 512: return launch_convolve_ct<T, 512>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    case 1024: return launch_convolve_ct<T, 1024>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    case 2048: return launch_convolve_ct<T, 2048>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    case 4096: return launch_convolve_ct<T, 4096>(x, m, n, nrhs, khat, tw, a, coef_ct, work, y, st, y64, xp);
    default: break;  // shorter lengths: the runtime-length passes below
  }
  const int S = seq_per_block<T>(P);
  const int nt = threads_for<T>(S, P);
  const size_t lds = (size_t)(S + 1) * P * sizeof(C<T>);
  if (S & (S - 1)) return hipErrorInvalidValue;  // the passes index by shifts
  hipError_t e;
  if ((e = allow_lds(k_row_forward<T>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_col_convolve<T>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_inverse<T, false>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_inverse<T, true>, lds)) != hipSuccess) return e;
  const T coef = c / ((T)P * (T)P);
  dim3 grow((n + S - 1) / S, nrhs), gcol(P / S, nrhs);
  hipLaunchKernelGGL(k_row_forward<T>, grow, dim3(nt), lds, st, x, m, n, P, S, tw, work, xp);
  hipLaunchKernelGGL(k_col_convolve<T>, gcol, dim3(nt), lds, st, work, khat, n, P, S, tw);
  if (y64)
    hipLaunchKernelGGL((k_row_inverse<T, true>), grow, dim3(nt), lds, st, work, x, n, P, S, tw, a, coef, y, y64, xp);
  else
    hipLaunchKernelGGL((k_row_inverse<T, false>), grow, dim3(nt), lds, st, work, x, n, P, S, tw, a, coef, y, y64, xp);
  return hipGetLastError();
}
template hipError_t launch_convolve<double>(const double2*, const double*, int, int, const double2*,
                                            const double2*, double, double, double2*, double2*,
                                            hipStream_t, double2* const*, const double2* const*);
template hipError_t launch_convolve<float>(const float2*, const float*, int, int, const float2*,
                                           const float2*, float, float, float2*, float2*, hipStream_t,
                                           double2* const*, const float2* const*);

hipError_t launch_green_spectrum(const double2* kq, int n, const double2* tw, double2* scratch,
                                 double2* khat, float2* khat32, hipStream_t st) {
  const int P = fft_len(n);
  const int S = seq_per_block<double>(P);
  const int nt = threads_for<double>(S, P);
  const size_t lds = (size_t)(S + 1) * P * sizeof(double2);
  if (S & (S - 1)) return hipErrorInvalidValue;  // the passes index by shifts
  hipError_t e;
  if ((e = allow_lds(k_fft_rows_full, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_fft_cols_full, lds)) != hipSuccess) return e;
  const size_t tot = (size_t)P * P;
  hipLaunchKernelGGL(k_wrap_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, kq, n, P, scratch);
  hipLaunchKernelGGL(k_fft_rows_full, dim3(P / S), dim3(nt), lds, st, scratch, P, S, tw);
  hipLaunchKernelGGL(k_fft_cols_full, dim3(P / S), dim3(nt), lds, st, scratch, P, S, tw, khat, khat32);
  return hipGetLastError();
}


size_t fft3_w1_elems(int n) { return (size_t)n * n * fft_len(n); }
size_t fft3_w2_elems(int n) {
  const size_t P = fft_len(n);
  return (size_t)n * P * P;
}

namespace {
// sequences per workgroup of the 3D passes: at most 16, S * P <= kVals * 512
template <typename T>
int seq3(int P) {
  int S = 16;
  while (S > 1 && (S * P > kVals<T> * kFftMaxThreads || (size_t)(S + 1) * P * sizeof(C<T>) > 163840)) S >>= 1;
  return S > P ? P : S;
}
}  // namespace

template <typename T>
hipError_t launch_convolve3(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat, const C<T>* tw, T a,
                            T c, C<T>* w1, C<T>* w2, C<T>* y, hipStream_t st) {
  const int P = fft_len(n);
  const int S = seq3<T>(P);
  const int nt = threads_for<T>(S, P);
  const size_t lds = (size_t)(S + 1) * P * sizeof(C<T>);
  if (S & (S - 1)) return hipErrorInvalidValue;  // the passes index by shifts
  hipError_t e;
  if ((e = allow_lds(k3_rows_fwd<T, true>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k3_rows_fwd<T, false>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k3_axis<T, 0>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k3_axis<T, 1>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k3_axis<T, 2>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k3_rows_inv<T>, lds)) != hipSuccess) return e;
  const int rows = n * n;
  const size_t PP = (size_t)P * P;
  const size_t r1 = fft3_w1_elems(n), r2 = fft3_w2_elems(n);
  const T coef = c / ((T)P * (T)P * (T)P);
  const dim3 grow((rows + S - 1) / S, nrhs);
  if (m)
    hipLaunchKernelGGL((k3_rows_fwd<T, true>), grow, dim3(nt), lds, st, x, m, n, P, S, tw, w1);
  else
    hipLaunchKernelGGL((k3_rows_fwd<T, false>), grow, dim3(nt), lds, st, x, m, n, P, S, tw, w1);
  // sequences: element t at stride st, S consecutive k3 (stride 1) per group
  const Seq3 a1{(size_t)P, 1, (size_t)n * P, r1};  // w1 along i2, groups by i1
  const Seq3 a2{(size_t)P, 1, PP, r2};             // w2 along k2, groups by i1
  const Seq3 a3{PP, 1, (size_t)P, r2};             // w2 along i1, groups by k2
  // axis 2: w1[i1][i2][k3] (i2 < n) -> w2[i1][k2][k3]
  hipLaunchKernelGGL((k3_axis<T, 0>), dim3(P / S, n, nrhs), dim3(nt), lds, st, w1, w2, khat, P, S, n, P, a1, a2,
                     tw);
  // axis 1 with khat: w2[i1][k2][k3] (i1 < n), in place
  hipLaunchKernelGGL((k3_axis<T, 1>), dim3(P / S, P, nrhs), dim3(nt), lds, st, w2, w2, khat, P, S, n, n, a3, a3,
                     tw);
  // inverse axis 2: w2[i1][k2][k3] -> w1[i1][i2][k3] (i2 < n)
  hipLaunchKernelGGL((k3_axis<T, 2>), dim3(P / S, n, nrhs), dim3(nt), lds, st, w2, w1, khat, P, S, P, n, a2, a1,
                     tw);
  hipLaunchKernelGGL(k3_rows_inv<T>, grow, dim3(nt), lds, st, w1, x, n, P, S, tw, a, coef, y);
  return hipGetLastError();
}
template hipError_t launch_convolve3<double>(const double2*, const double*, int, int, const double2*,
                                             const double2*, double, double, double2*, double2*, double2*,
                                             hipStream_t);
template hipError_t launch_convolve3<float>(const float2*, const float*, int, int, const float2*, const float2*,
                                            float, float, float2*, float2*, float2*, hipStream_t);

hipError_t launch_green_spectrum3(const double2* kq, int n, const double2* tw, double2* scratch, double2* khat,
                                  float2* khat32, hipStream_t st) {
  const int P = fft_len(n);
  const int S = seq3<double>(P);
  const int nt = threads_for<double>(S, P);
  const size_t lds = (size_t)(S + 1) * P * sizeof(double2);
  if (S & (S - 1)) return hipErrorInvalidValue;  // the passes index by shifts
  hipError_t e;
  if ((e = allow_lds(k3_axis<double, 0>, lds)) != hipSuccess) return e;
  const size_t P3 = (size_t)P * P * P, PP = (size_t)P * P;
  hipLaunchKernelGGL(k3_wrap_table, dim3((unsigned)((P3 + 255) / 256)), dim3(256), 0, st, kq, n, P, scratch);
  // forward transforms along each axis in place, all P inputs and outputs:
  // axis 3 (S rows as sequences: stride 1 within, P between rows), axis 2, axis 1
  // axis 3: the P^2 rows (contiguous sequences, P apart) in groups of S rows
  const Seq3 r3{1, (size_t)P, (size_t)S * P, 0};
  hipLaunchKernelGGL((k3_axis<double, 0>), dim3(1, (unsigned)(PP / S), 1), dim3(nt), lds, st, scratch, scratch,
                     (const double2*)nullptr, P, S, P, P, r3, r3, tw);
  // axis 2 (groups by k1) and axis 1 (groups by k2), S consecutive k3 each
  const Seq3 r2{(size_t)P, 1, PP, 0}, r1{PP, 1, (size_t)P, 0};
  hipLaunchKernelGGL((k3_axis<double, 0>), dim3(P / S, P, 1), dim3(nt), lds, st, scratch, scratch,
                     (const double2*)nullptr, P, S, P, P, r2, r2, tw);
  hipLaunchKernelGGL((k3_axis<double, 0>), dim3(P / S, P, 1), dim3(nt), lds, st, scratch, scratch,
                     (const double2*)nullptr, P, S, P, P, r1, r1, tw);
  const int H = P / 2 + 1;
  const size_t H3 = (size_t)H * H * H;
  hipLaunchKernelGGL(k3_octant, dim3((unsigned)((H3 + 255) / 256)), dim3(256), 0, st, scratch, P, khat, khat32);
  return hipGetLastError();
}

}  // namespace lsw
