// Device kernels of the sparsify-and-sweep solver and their launchers.
#pragma once

#include "common.hpp"

namespace lsw {

// ---- FFT convolution with the Green's table (fft.hip) ----
// FFT length for n interior points: the power of two >= 2(n+1).
inline int fft_len(int n) {
  int P = 1;
  while (P < 2 * (n + 1)) P <<= 1;
  return P;
}
template <typename T>
size_t fft_work_elems(int n, int nrhs);
// y = a x + c * K (s .* x) on [nrhs][n][n]; s = m or 1 (m == nullptr).
template <typename T>
hipError_t launch_convolve(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat,
                           const C<T>* tw, T a, T c, C<T>* work, C<T>* y, hipStream_t st);
// khat (quadrant (P/2+1)^2) from the table quadrant kq [(n+2)][(n+2)].
hipError_t launch_green_spectrum(const double2* kq, int n, const double2* tw, double2* scratch,
                                 double2* khat, float2* khat32, hipStream_t st);

// ---- stencils, slices and sweep (sweep.hip) ----
struct StencilTables {
  const double2* alpha;  // 9
  const double2* beta;   // 9
  const double2* gglob;  // (2b+1)^2 x 9
  const double2* gaux;   // b x (2b+1) x ns x 9
  const int* kmap;       // L x L
  const double* m;       // n x n
  int n, b, L, ns;
  double omega2;
};

struct SliceTables {
  const int* lo;     // per slice: first grid line of D_k
  const int* hi;     // last grid line of D_k
  const int* first;  // first line of the subproblem
  const int* t;      // lines of the subproblem
  const size_t* fs_off;  // offset (complex elements) of slice k in FS: L x (t^2 + 3t)
  const size_t* fg_off;  // offset of slice k in FG: L x t^2
  int nslices;
};

template <typename T>
hipError_t launch_apply_Q(const StencilTables& S, const C<T>* r, int nrhs, C<T>* f, hipStream_t st);
template <typename T>
hipError_t launch_apply_H(const StencilTables& S, const C<T>* u, int nrhs, C<T>* y, hipStream_t st);
template <typename T>
hipError_t launch_extract(int n, int b, const C<T>* uext, int nrhs, C<T>* z, hipStream_t st);
// Assemble and factor every slice subproblem (one workgroup per slice);
// writes FS, FG, the coupling rows Hm, Hp ([nslices][L][3]) and status
// (nonzero: a zero pivot was met).
template <typename T>
hipError_t launch_factor_slices(const StencilTables& S, const SliceTables& P, C<T>* FS, C<T>* FG,
                                C<T>* Hm, C<T>* Hp, int* status, hipStream_t st);

enum SweepMode { kSweepFull = 0, kSliceOnly = 1 };
// Full sweep (Algorithm 2, steps 3-8) of f -> u on [nrhs][L][L], or one slice
// solve of v -> w on [nrhs][lines][L] (mode kSliceOnly, slice k).
template <typename T>
hipError_t launch_sweep(const SliceTables& P, int L, int b, const C<T>* FS, const C<T>* FG,
                        const C<T>* Hm, const C<T>* Hp, const C<T>* f, C<T>* u, C<T>* yscratch,
                        int nrhs, int mode, int slice, hipStream_t st);

// ---- Krylov helpers (krylov.hip) ----
struct DotPair {
  const double2* x;
  const double2* y;
};
// out[p] = sum conj(x_p) y_p over N complex entries; partials has room for
// npairs * kDotBlocks entries. Deterministic (fixed-order reductions).
constexpr int kDotBlocks = 64;
hipError_t launch_dots(const DotPair* pairs, int npairs, size_t N, double2* partials, double2* out,
                       hipStream_t st);
// y_o = beta_o * y_o + sum_t c_t x_t. Terms of output o are [tbeg[o], tbeg[o+1]).
template <typename TX>
struct AxpyTerm {
  const C<TX>* x;
  int coef;     // index into coefs
  int negate;   // 1: use -coef
};
struct AxpyOut {
  double2* y;
  int tbeg, tend;
  int zero_first;  // 1: y starts from 0
  int scale_coef;  // >= 0: multiply the sum of terms by 1/coefs[scale_coef].x (after sqrt if sqrt_scale)
  int sqrt_scale;
};
template <typename TX>
hipError_t launch_axpys(const AxpyOut* outs, int nout, const AxpyTerm<TX>* terms,
                        const double2* coefs, size_t N, hipStream_t st);
// dst[p] = cast(src[p]) for npairs contiguous batches of N entries.
template <typename TD, typename TS>
hipError_t launch_copy_cast(C<TD>* const* dst, const C<TS>* const* src, int npairs, size_t N,
                            hipStream_t st);
// grad = -omega^2 Re sum_j psi_j * nu_j (psi, nu: [nrhs][N])
hipError_t launch_adjoint_product(const double2* psi, const double2* nu, int nrhs, size_t N,
                                  double omega2, double* grad, hipStream_t st);
// dst = conj(src) over N entries (float64)
hipError_t launch_conj(double2* dst, const double2* src, size_t N, hipStream_t st);
// x (+)= s * y elementwise over N with real s, float64 (incident total field etc.)
hipError_t launch_add_scaled(double2* x, const double2* y, double s, size_t N, hipStream_t st);

}  // namespace lsw
