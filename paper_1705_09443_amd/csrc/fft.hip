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

// In-place Stockham FFT (radix 4, a final radix 2 when log2 P is odd) of nseq
// interleaved sequences: element k of sequence s lives at buf[k * nseq + s].
// tw[k] = exp(-2 pi i k / P); the inverse uses the conjugate (unnormalised).
// complex values a thread holds per pass (16: no register spills at 512 threads)
template <typename T>
constexpr int kVals = 16;
constexpr int kFftMaxThreads = 512;

template <typename T, int R>
__device__ inline void lds_fft_pass(C<T>* buf, int P, int nseq, int Ns, const C<T>* __restrict__ tw, bool inv) {
  constexpr int NB = kVals<T> / R;  // butterflies per thread
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nbf = P / R;
  const int total = nbf * nseq;
  C<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bidx = tid + q * nt;
    if (bidx < total) {
      const int s = bidx % nseq, j = bidx / nseq;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[(j + r * nbf) * nseq + s];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int bidx = tid + q * nt;
    if (bidx >= total) continue;
    const int s = bidx % nseq, j = bidx / nseq;
    const int k = j % Ns;
    const int step = k * (P / (Ns * R));
    C<T>* x = v[q];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      C<T> w = tw[r * step];
      if (inv) w.y = -w.y;
      x[r] = cmul<T>(x[r], w);
    }
    if (R == 4) {
      const C<T> a0 = cadd<T>(x[0], x[2]), a1 = csub<T>(x[0], x[2]);
      const C<T> a2 = cadd<T>(x[1], x[3]);
      const C<T> d = csub<T>(x[1], x[3]);
      // times -i (forward) or +i (inverse)
      const C<T> a3 = inv ? mk<T>(-d.y, d.x) : mk<T>(d.y, -d.x);
      x[0] = cadd<T>(a0, a2);
      x[2] = csub<T>(a0, a2);
      x[1] = cadd<T>(a1, a3);
      x[3] = csub<T>(a1, a3);
    } else {
      const C<T> a0 = cadd<T>(x[0], x[1]), a1 = csub<T>(x[0], x[1]);
      x[0] = a0;
      x[1] = a1;
    }
    const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(idxD + r * Ns) * nseq + s] = x[r];
  }
  __syncthreads();
}

// In-place Stockham FFT (radix 4, a final radix 2 when log2 P is odd) of nseq
// interleaved sequences: element k of sequence s lives at buf[k * nseq + s].
// tw[k] = exp(-2 pi i k / P); the inverse uses the conjugate (unnormalised).
// Needs blockDim.x >= nseq * P / kVals<T>.
template <typename T>
__device__ void lds_fft(C<T>* buf, int P, int nseq, const C<T>* __restrict__ tw, bool inv) {
  int Ns = 1;
  for (; P / Ns >= 4; Ns *= 4) lds_fft_pass<T, 4>(buf, P, nseq, Ns, tw, inv);
  if (Ns < P) lds_fft_pass<T, 2>(buf, P, nseq, Ns, tw, inv);
}

// ---- pass 1: rows of (s .* x), zero-padded to P -----------------------------
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k_row_forward(const C<T>* __restrict__ x, const T* __restrict__ m, int n, int P,
                              int S, const C<T>* __restrict__ tw, C<T>* __restrict__ X) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  const int rhs = blockIdx.y;
  const int i0 = blockIdx.x * S;
  const size_t nn = (size_t)n * n;
  const C<T>* xr = x + rhs * nn;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int s = idx / P, k = idx % P;
    const int row = i0 + s;
    C<T> v = mk<T>(0, 0);
    if (k < n && row < n) {
      v = xr[(size_t)row * n + k];
      if (m) v = cscale<T>(v, m[(size_t)row * n + k]);
    }
    buf[k * S + s] = v;
  }
  __syncthreads();
  lds_fft<T>(buf, P, S, tw, false);
  const int ntile = P / S;
  C<T>* Xr = X + (size_t)rhs * ntile * n * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int tile = idx / (S * S), within = idx % (S * S);
    const int s = within / S, kk = within % S;
    const int row = i0 + s;
    if (row < n) Xr[((size_t)tile * n + row) * S + kk] = buf[(tile * S + kk) * S + s];
  }
}

// ---- pass 2: columns, times khat, inverse columns ------------------------
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k_col_convolve(C<T>* __restrict__ X, const C<T>* __restrict__ khat, int n, int P,
                               int S, const C<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  const int tile = blockIdx.x, rhs = blockIdx.y;
  const int ntile = P / S;
  C<T>* Xt = X + ((size_t)rhs * ntile + tile) * n * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int row = idx / S;
    buf[idx] = row < n ? Xt[idx] : mk<T>(0, 0);
  }
  __syncthreads();
  lds_fft<T>(buf, P, S, tw, false);
  const int half = P / 2 + 1;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int r = idx / S, s = idx % S;
    const int col = tile * S + s;
    const int kr = r <= P - r ? r : P - r;
    const int kc = col <= P - col ? col : P - col;
    buf[idx] = cmul<T>(buf[idx], khat[(size_t)kr * half + kc]);
  }
  __syncthreads();
  lds_fft<T>(buf, P, S, tw, true);
  for (int idx = threadIdx.x; idx < S * n; idx += blockDim.x) Xt[idx] = buf[idx];
}

// ---- pass 3: inverse rows and epilogue y = a x + coef * conv --------------
template <typename T>
__global__ __launch_bounds__(kFftMaxThreads) void k_row_inverse(const C<T>* __restrict__ X, const C<T>* __restrict__ x, int n, int P,
                              int S, const C<T>* __restrict__ tw, T a, T coef,
                              C<T>* __restrict__ y) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
  const int rhs = blockIdx.y;
  const int i0 = blockIdx.x * S;
  const int ntile = P / S;
  const C<T>* Xr = X + (size_t)rhs * ntile * n * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int tile = idx / (S * S), within = idx % (S * S);
    const int s = within / S, kk = within % S;
    const int row = i0 + s;
    buf[(tile * S + kk) * S + s] = row < n ? Xr[((size_t)tile * n + row) * S + kk] : mk<T>(0, 0);
  }
  __syncthreads();
  lds_fft<T>(buf, P, S, tw, true);
  const size_t nn = (size_t)n * n;
  for (int idx = threadIdx.x; idx < S * n; idx += blockDim.x) {
    const int s = idx / n, k = idx % n;
    const int row = i0 + s;
    if (row >= n) continue;
    const size_t o = rhs * nn + (size_t)row * n + k;
    C<T> v = cscale<T>(buf[k * S + s], coef);
    if (a != T(0)) v = cadd<T>(v, cscale<T>(x[o], a));
    y[o] = v;
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
  const int r0 = blockIdx.x * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int s = idx / P, k = idx % P;
    buf[k * S + s] = W[(size_t)(r0 + s) * P + k];
  }
  __syncthreads();
  lds_fft<double>(buf, P, S, tw, false);
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
  const int c0 = blockIdx.x * S;
  for (int idx = threadIdx.x; idx < S * P; idx += blockDim.x) {
    const int r = idx / S, s = idx % S;
    buf[idx] = W[(size_t)r * P + c0 + s];
  }
  __syncthreads();
  lds_fft<double>(buf, P, S, tw, false);
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

template <typename T>
int seq_per_block(int P) {
  int S = 131072 / (P * (int)sizeof(C<T>));
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
  return (size_t)nrhs * P * n;
}
template size_t fft_work_elems<double>(int, int);
template size_t fft_work_elems<float>(int, int);

template <typename T>
hipError_t launch_convolve(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat,
                           const C<T>* tw, T a, T c, C<T>* work, C<T>* y, hipStream_t st) {
  const int P = fft_len(n);
  const int S = seq_per_block<T>(P);
  const int nt = threads_for<T>(S, P);
  const size_t lds = (size_t)S * P * sizeof(C<T>);
  hipError_t e;
  if ((e = allow_lds(k_row_forward<T>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_col_convolve<T>, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_row_inverse<T>, lds)) != hipSuccess) return e;
  const T coef = c / ((T)P * (T)P);
  dim3 grow((n + S - 1) / S, nrhs), gcol(P / S, nrhs);
  hipLaunchKernelGGL(k_row_forward<T>, grow, dim3(nt), lds, st, x, m, n, P, S, tw, work);
  hipLaunchKernelGGL(k_col_convolve<T>, gcol, dim3(nt), lds, st, work, khat, n, P, S, tw);
  hipLaunchKernelGGL(k_row_inverse<T>, grow, dim3(nt), lds, st, work, x, n, P, S, tw, a, coef, y);
  return hipGetLastError();
}
template hipError_t launch_convolve<double>(const double2*, const double*, int, int, const double2*,
                                            const double2*, double, double, double2*, double2*,
                                            hipStream_t);
template hipError_t launch_convolve<float>(const float2*, const float*, int, int, const float2*,
                                           const float2*, float, float, float2*, float2*, hipStream_t);

hipError_t launch_green_spectrum(const double2* kq, int n, const double2* tw, double2* scratch,
                                 double2* khat, float2* khat32, hipStream_t st) {
  const int P = fft_len(n);
  const int S = seq_per_block<double>(P);
  const int nt = threads_for<double>(S, P);
  const size_t lds = (size_t)S * P * sizeof(double2);
  hipError_t e;
  if ((e = allow_lds(k_fft_rows_full, lds)) != hipSuccess) return e;
  if ((e = allow_lds(k_fft_cols_full, lds)) != hipSuccess) return e;
  const size_t tot = (size_t)P * P;
  hipLaunchKernelGGL(k_wrap_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, kq, n, P, scratch);
  hipLaunchKernelGGL(k_fft_rows_full, dim3(P / S), dim3(nt), lds, st, scratch, P, S, tw);
  hipLaunchKernelGGL(k_fft_cols_full, dim3(P / S), dim3(nt), lds, st, scratch, P, S, tw, khat, khat32);
  return hipGetLastError();
}

}  // namespace lsw
