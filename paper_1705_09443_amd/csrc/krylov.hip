// Krylov-loop helpers for the float64 (flexible) GMRES: batched dot products
// with fixed-order reductions (bitwise reproducible, no float atomics),
// multi-term axpy updates, precision casts and the adjoint's pointwise
// product.
#include <algorithm>

#include "kernels.hpp"

namespace lsw {

namespace {

constexpr int kThreads = 256;

__device__ inline double2 wave_sum(double2 v) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

// partials[p][blk] = sum over the blk-th chunk of conj(x_p) y_p
__global__ __launch_bounds__(kThreads) void k_dot_partials(const DotPair* __restrict__ pairs, size_t N,
                                                           double2* __restrict__ partials) {
  const int p = blockIdx.y, blk = blockIdx.x;
  const DotPair pr = pairs[p];
  const size_t chunk = (N + kDotBlocks - 1) / kDotBlocks;
  const size_t beg = blk * chunk;
  const size_t end = beg + chunk < N ? beg + chunk : N;
  double2 acc = make_double2(0.0, 0.0);
  for (size_t i = beg + threadIdx.x; i < end; i += kThreads) {
    const double2 a = pr.x[i], c = pr.y[i];
    acc.x += a.x * c.x + a.y * c.y;
    acc.y += a.x * c.y - a.y * c.x;
  }
  acc = wave_sum(acc);
  __shared__ double2 ws[kThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 s = ws[0];
    for (int w = 1; w < kThreads / 64; ++w) {
      s.x += ws[w].x;
      s.y += ws[w].y;
    }
    partials[(size_t)p * kDotBlocks + blk] = s;
  }
}

// The dot products of one group (shared y) per blockIdx.y: the same per-pair
// arithmetic and order as k_dot_partials, with y read once.
__global__ __launch_bounds__(kThreads) void k_mdot_partials(const DotGroup* __restrict__ groups, size_t N,
                                                            double2* __restrict__ partials) {
  const int blk = blockIdx.x;
  const DotGroup& gr = groups[blockIdx.y];
  const int cnt = gr.count;
  const size_t chunk = (N + kDotBlocks - 1) / kDotBlocks;
  const size_t beg = blk * chunk;
  const size_t end = beg + chunk < N ? beg + chunk : N;
  const double2* xs[kDotGroup];
#pragma unroll
  for (int k = 0; k < kDotGroup; ++k) xs[k] = gr.x[k < cnt ? k : 0];
  double2 acc[kDotGroup];
#pragma unroll
  for (int k = 0; k < kDotGroup; ++k) acc[k] = make_double2(0.0, 0.0);
  for (size_t i = beg + threadIdx.x; i < end; i += kThreads) {
    const double2 c = gr.y[i];
#pragma unroll
    for (int k = 0; k < kDotGroup; ++k) {
      if (k < cnt) {
        const double2 a = xs[k][i];
        acc[k].x += a.x * c.x + a.y * c.y;
        acc[k].y += a.x * c.y - a.y * c.x;
      }
    }
  }
  __shared__ double2 ws[kDotGroup][kThreads / 64];
#pragma unroll
  for (int k = 0; k < kDotGroup; ++k) {
    if (k < cnt) {
      const double2 v = wave_sum(acc[k]);
      if ((threadIdx.x & 63) == 0) ws[k][threadIdx.x >> 6] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    const int k = threadIdx.x;
    double2 s = ws[k][0];
    for (int w = 1; w < kThreads / 64; ++w) {
      s.x += ws[k][w].x;
      s.y += ws[k][w].y;
    }
    partials[(size_t)(gr.pbase + k) * kDotBlocks + blk] = s;
  }
}

__global__ void k_dot_reduce(const double2* __restrict__ partials, int npairs, double2* __restrict__ out,
                             int nparts = kDotBlocks) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  double2 s = make_double2(0.0, 0.0);
  for (int b = 0; b < nparts; ++b) {
    s.x += partials[(size_t)p * nparts + b].x;
    s.y += partials[(size_t)p * nparts + b].y;
  }
  out[p] = s;
}

// blocks (and partial sums) per output of the updates that also form norms
constexpr int kNormBlocks = 256;

// norm_partials (optional): ||y_o||^2 of this block's share of the updated
// output, at norm_partials[o * gridDim.x + blockIdx.x]
template <typename TX>
__global__ __launch_bounds__(kThreads) void k_axpys(const AxpyOut* __restrict__ outs,
                                                    const AxpyTerm<TX>* __restrict__ terms,
                                                    const double2* __restrict__ coefs, size_t N,
                                                    double2* __restrict__ norm_partials) {
  const AxpyOut o = outs[blockIdx.y];
  double nrm = 0.0;
  double sc = 1.0;
  if (o.scale_coef >= 0) {
    const double v = coefs[o.scale_coef].x;
    sc = 1.0 / (o.sqrt_scale ? sqrt(v) : v);
  }
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < N; i += (size_t)gridDim.x * kThreads) {
    double2 acc = make_double2(0.0, 0.0);
    for (int t = o.tbeg; t < o.tend; ++t) {
      const AxpyTerm<TX> tm = terms[t];
      double2 c = coefs[tm.coef];
      if (tm.negate) {
        c.x = -c.x;
        c.y = -c.y;
      }
      const C<TX> xv = tm.x[i];
      acc.x += c.x * (double)xv.x - c.y * (double)xv.y;
      acc.y += c.x * (double)xv.y + c.y * (double)xv.x;
    }
    double2 y = o.zero_first ? make_double2(0.0, 0.0) : o.y[i];
    y.x = (y.x + acc.x) * sc;
    y.y = (y.y + acc.y) * sc;
    o.y[i] = y;
    nrm += y.x * y.x + y.y * y.y;
  }
  if (norm_partials) {
    const double2 v = wave_sum(make_double2(nrm, 0.0));
    __shared__ double ws[kThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v.x;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = ws[0];
      for (int w = 1; w < kThreads / 64; ++w) s += ws[w];
      norm_partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(s, 0.0);
    }
  }
}

template <typename TD, typename TS>
__global__ void k_copy_cast(C<TD>* const* __restrict__ dst, const C<TS>* const* __restrict__ src, size_t N) {
  const int p = blockIdx.y;
  C<TD>* d = dst[p];
  const C<TS>* s = src[p];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
    d[i] = ccast<TD, TS>(s[i]);
}

template <typename TD, typename TS>
__global__ void k_cast_flat(C<TD>* __restrict__ dst, const C<TS>* __restrict__ src, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = ccast<TD, TS>(src[i]);
}

// partials[c][blk] = the blk-th chunk of ||x_c||^2 for the columns of a
// [ncols][N] block (fixed chunks and order: reproducible)
__global__ __launch_bounds__(kThreads) void k_colnorm2(const double2* __restrict__ x, size_t N,
                                                       double* __restrict__ partials) {
  const int c = blockIdx.y, blk = blockIdx.x;
  const double2* xc = x + (size_t)c * N;
  const size_t chunk = (N + kDotBlocks - 1) / kDotBlocks;
  const size_t beg = blk * chunk;
  const size_t end = beg + chunk < N ? beg + chunk : N;
  double acc = 0.0;
  for (size_t i = beg + threadIdx.x; i < end; i += kThreads) {
    const double2 a = xc[i];
    acc += a.x * a.x + a.y * a.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  __shared__ double ws[kThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = ws[0];
    for (int w = 1; w < kThreads / 64; ++w) s += ws[w];
    partials[(size_t)c * kDotBlocks + blk] = s;
  }
}

__global__ void k_adjoint_product(const double2* __restrict__ psi, const double2* __restrict__ nu, int nrhs,
                                  size_t N, double omega2, double* __restrict__ grad) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nrhs; ++j) {
      const double2 a = psi[(size_t)j * N + i], c = nu[(size_t)j * N + i];
      s += a.x * c.x - a.y * c.y;
    }
    grad[i] = -omega2 * s;
  }
}

// out[t] = in[t] * s[t] for n complex coefficients and real factors
__global__ void k_scale_coefs(const double2* __restrict__ in, const double* __restrict__ s, double2* __restrict__ out,
                              int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = make_double2(in[t].x * s[t], in[t].y * s[t]);
}

// u = x and psi = x + y (y may be null: psi = x), one pass over x and y;
// each element of y is read before u is written, so u may be y itself
__global__ void k_solution_out(double2* u, double2* __restrict__ psi, const double2* __restrict__ x,
                               const double2* y, size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = x[i];
    const double2 w = y ? y[i] : make_double2(0.0, 0.0);
    u[i] = v;
    psi[i] = make_double2(v.x + w.x, v.y + w.y);
  }
}

// k plane waves exp(i omega (cos t_j x1 + sin t_j x2)), t_j = 2 pi j / k, at the
// interior points x = (i + 1) h: [k][n][n]
__global__ void k_plane_waves(double2* __restrict__ out, int n, double omega, int k) {
  const size_t N = (size_t)n * n, total = N * k;
  const double h = 1.0 / (n + 1);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / N);
    const size_t p = e % N;
    const double x1 = (double)(p / n + 1) * h, x2 = (double)(p % n + 1) * h;
    const double t = 2.0 * M_PI * j / k;
    const double ph = omega * (cos(t) * x1 + sin(t) * x2);
    out[e] = make_double2(cos(ph), sin(ph));
  }
}

__global__ void k_conj(double2* __restrict__ d, const double2* __restrict__ s, size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
    d[i] = make_double2(s[i].x, -s[i].y);
}

unsigned grid_for(size_t N) {
  size_t g = (N + kThreads - 1) / kThreads;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_dots(const DotPair* pairs, int npairs, size_t N, double2* partials, double2* out,
                       hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dot_partials, dim3(kDotBlocks, npairs), dim3(kThreads), 0, st, pairs, N, partials);
  hipLaunchKernelGGL(k_dot_reduce, dim3((npairs + 127) / 128), dim3(128), 0, st, partials, npairs, out, kDotBlocks);
  return hipGetLastError();
}

hipError_t launch_mdots(const DotGroup* groups, int ngroups, int npairs, size_t N, double2* partials, double2* out,
                        hipStream_t st) {
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mdot_partials, dim3(kDotBlocks, ngroups), dim3(kThreads), 0, st, groups, N, partials);
  hipLaunchKernelGGL(k_dot_reduce, dim3((npairs + 127) / 128), dim3(128), 0, st, partials, npairs, out, kDotBlocks);
  return hipGetLastError();
}

template <typename TX>
hipError_t launch_axpys(const AxpyOut* outs, int nout, const AxpyTerm<TX>* terms, const double2* coefs,
                        size_t N, hipStream_t st) {
  if (nout <= 0) return hipSuccess;
  unsigned g = grid_for(N);
  if (g > 512) g = 512;
  hipLaunchKernelGGL(k_axpys<TX>, dim3(g, nout), dim3(kThreads), 0, st, outs, terms, coefs, N, (double2*)nullptr);
  return hipGetLastError();
}

hipError_t launch_axpys_norms(const AxpyOut* outs, int nout, const AxpyTerm<double>* terms, const double2* coefs,
                              size_t N, double2* partials, double2* norm2, hipStream_t st) {
  if (nout <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpys<double>, dim3(kNormBlocks, nout), dim3(kThreads), 0, st, outs, terms, coefs, N,
                     partials);
  hipLaunchKernelGGL(k_dot_reduce, dim3((nout + 127) / 128), dim3(128), 0, st, partials, nout, norm2, kNormBlocks);
  return hipGetLastError();
}
template hipError_t launch_axpys<double>(const AxpyOut*, int, const AxpyTerm<double>*, const double2*,
                                         size_t, hipStream_t);
template hipError_t launch_axpys<float>(const AxpyOut*, int, const AxpyTerm<float>*, const double2*,
                                        size_t, hipStream_t);

template <typename TD, typename TS>
hipError_t launch_copy_cast(C<TD>* const* dst, const C<TS>* const* src, int npairs, size_t N, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  unsigned g = grid_for(N);
  if (g > 512) g = 512;
  hipLaunchKernelGGL((k_copy_cast<TD, TS>), dim3(g, npairs), dim3(kThreads), 0, st, dst, src, N);
  return hipGetLastError();
}
template hipError_t launch_copy_cast<double, double>(double2* const*, const double2* const*, int, size_t,
                                                     hipStream_t);
template hipError_t launch_copy_cast<float, double>(float2* const*, const double2* const*, int, size_t,
                                                    hipStream_t);
template hipError_t launch_copy_cast<double, float>(double2* const*, const float2* const*, int, size_t,
                                                    hipStream_t);
template hipError_t launch_copy_cast<float, float>(float2* const*, const float2* const*, int, size_t,
                                                   hipStream_t);

template <typename TD, typename TS>
hipError_t launch_cast_flat(C<TD>* dst, const C<TS>* src, size_t count, hipStream_t st) {
  hipLaunchKernelGGL((k_cast_flat<TD, TS>), dim3(2048), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}
template hipError_t launch_cast_flat<double, float>(double2*, const float2*, size_t, hipStream_t);
template hipError_t launch_cast_flat<float, double>(float2*, const double2*, size_t, hipStream_t);
template hipError_t launch_cast_flat<double, double>(double2*, const double2*, size_t, hipStream_t);
template hipError_t launch_cast_flat<float, float>(float2*, const float2*, size_t, hipStream_t);

// out[i] = sum over c < nparts of parts[c * count + i] (fixed order)
__global__ void k_sum_parts(const double2* __restrict__ parts, int nparts, size_t count, double2* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    double2 acc = parts[i];
    for (int c = 1; c < nparts; ++c) {
      const double2 v = parts[(size_t)c * count + i];
      acc.x += v.x;
      acc.y += v.y;
    }
    out[i] = acc;
  }
}

hipError_t launch_sum_parts(const double2* parts, int nparts, size_t count, double2* out, hipStream_t st) {
  const int blocks = (int)std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sum_parts, dim3(std::max(blocks, 1)), dim3(256), 0, st, parts, nparts, count, out);
  return hipGetLastError();
}

hipError_t launch_colnorm2(const double2* x, int ncols, size_t N, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_colnorm2, dim3(kDotBlocks, ncols), dim3(kThreads), 0, st, x, N, partials);
  return hipGetLastError();
}

hipError_t launch_adjoint_product(const double2* psi, const double2* nu, int nrhs, size_t N, double omega2,
                                  double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_product, dim3(grid_for(N)), dim3(kThreads), 0, st, psi, nu, nrhs, N, omega2, grad);
  return hipGetLastError();
}

hipError_t launch_conj(double2* dst, const double2* src, size_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_conj, dim3(grid_for(N)), dim3(kThreads), 0, st, dst, src, N);
  return hipGetLastError();
}

hipError_t launch_plane_waves(double2* out, int n, double omega, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_plane_waves, dim3(grid_for((size_t)n * n * k)), dim3(kThreads), 0, st, out, n, omega, k);
  return hipGetLastError();
}

hipError_t launch_scale_coefs(const double2* in, const double* s, double2* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_coefs, dim3((n + 127) / 128), dim3(128), 0, st, in, s, out, n);
  return hipGetLastError();
}
hipError_t launch_solution_out(double2* u, double2* psi, const double2* x, const double2* y, size_t N,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_solution_out, dim3(grid_for(N)), dim3(kThreads), 0, st, u, psi, x, y, N);
  return hipGetLastError();
}

}  // namespace lsw
