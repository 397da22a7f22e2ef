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
// With y64 (a device array of nrhs pointers to n x n float64 grids), right-hand
// side r goes to y64[r] instead, formed in T and then widened (y unused). With
// xp (nrhs pointers to n x n grids), right-hand side r is read from xp[r]
// instead of x.
template <typename T>
hipError_t launch_convolve(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat,
                           const C<T>* tw, T a, T c, C<T>* work, C<T>* y, hipStream_t st,
                           double2* const* y64 = nullptr, const C<T>* const* xp = nullptr);
// khat (quadrant (P/2+1)^2) from the table quadrant kq [(n+2)][(n+2)].
hipError_t launch_green_spectrum(const double2* kq, int n, const double2* tw, double2* scratch,
                                 double2* khat, float2* khat32, hipStream_t st);

// ---- 3D: the same convolution on [nrhs][n][n][n], P^3 zero padding ----
// Work per right-hand side: w1 n^2 P and w2 n P^2 complex values.
size_t fft3_w1_elems(int n);
size_t fft3_w2_elems(int n);
template <typename T>
hipError_t launch_convolve3(const C<T>* x, const T* m, int n, int nrhs, const C<T>* khat, const C<T>* tw, T a,
                            T c, C<T>* w1, C<T>* w2, C<T>* y, hipStream_t st);
// khat (octant (P/2+1)^3, float64 and a float32 copy) from the table octant kq
// [(n+2)]^3; scratch holds P^3 values.
hipError_t launch_green_spectrum3(const double2* kq, int n, const double2* tw, double2* scratch, double2* khat,
                                  float2* khat32, hipStream_t st);

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

// Complex values per block step of a slice factor: t^2 (+ t * tw for the
// forward factors), rounded up to an even count so every block starts on a
// 16-byte boundary.
__host__ __device__ inline int factor_stride(int t, int tw) { return (t * t + t * tw + 1) & ~1; }

// Per slice, in table order. A subproblem's t lines are numbered locally in
// the order of its front, a = 0..t-1 at grid line org + dir a: naux auxiliary
// lines, the tw = hi - lo + 1 lines of D_k, then t - naux - tw auxiliary lines
// (the two-front middle slice only). Every slice kernel works in these local
// coordinates: the stencil offset d1 along local lines is dir d1 in the grid.
struct SliceTables {
  const int* lo;     // per slice: first grid line of D_k
  const int* hi;     // last grid line of D_k
  const int* first;  // lowest grid line of the subproblem
  const int* t;      // lines of the subproblem
  const int* naux;   // auxiliary lines before D_k, locally
  const int* org;    // grid line of local line 0
  const int* dir;    // +1 (along x1) or -1
  const int* prev;   // slice coupled to D_k's first local line (eliminated earlier), -1: none
  const int* next;   // slice coupled to D_k's last local line, -1: none
  const int* next_lam;  // 1: that coupling reads the next slice's lambda, 0: its mu
  const size_t* fs_off;  // offset (complex elements) of slice k in FS: L x factor_stride(t, tw)
  const size_t* fg_off;  // offset of slice k in FG: L x factor_stride(t, 0)
  int nslices;
};

// Extended-grid fields come in two layouts: [nrhs][L][L] (right-hand side
// slowest: the C ABI's, and the sequential sweep's) and the interleaved
// [L][L][nrhs] of the interface schedule, where a 16-column tile of the
// matrix-core slice solves reads one 128-byte run per grid point.
// With r64 (interleaved only: a device array of nrhs pointers to n x n
// float64 grids), right-hand side q is read from r64[q], narrowed to T on
// load (r unused).
template <typename T>
hipError_t launch_apply_Q(const StencilTables& S, const C<T>* r, int nrhs, C<T>* f, bool interleaved,
                          hipStream_t st, const double2* const* r64 = nullptr);
template <typename T>
hipError_t launch_apply_H(const StencilTables& S, const C<T>* u, int nrhs, C<T>* y, hipStream_t st);
template <typename T>
// With zp (interleaved only: a device array of nrhs pointers to n x n grids),
// right-hand side q is written to zp[q] instead of z.
hipError_t launch_extract(int n, int b, const C<T>* uext, int nrhs, C<T>* z, bool interleaved, hipStream_t st,
                          C<T>* const* zp = nullptr);
// Between the [nb][E] layout of extended-grid batches and the interleaved
// [E][nb] one (to_il: the former into the latter; else back).
template <typename T>
hipError_t launch_interleave(const C<T>* in, int nb, size_t E, C<T>* out, bool to_il, hipStream_t st);
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

// ---- interface form of the sweep (interface.hip) ----
// kSrcGrid / kDstGrid: the interleaved extended grid [L][L][nrhs]
enum SliceSrc { kSrcGrid = 0, kSrcSlice = 1, kSrcUnitF = 2, kSrcUnitE = 3 };
enum SliceDst { kDstGrid = 0, kDstSlice = 1, kDstLines = 2 };
template <typename T>
struct SliceSolveArgs {
  SliceTables P;
  int L, b;
  const C<T>* FS;
  const C<T>* FG;
  const C<T>* Hm;
  const C<T>* Hp;
  int slice0;      // first slice of the launch
  int nrhs;        // right-hand sides (columns) of this launch
  int src_kind;    // SliceSrc
  const C<T>* src; // [nrhs][L][L] (grid) or [nrhs][lines][L] (slice)
  int col0;        // first column for the unit sources (columns of J_F Hm or J_E Hp)
  int dst_kind;    // SliceDst
  C<T>* dst;       // grid or slice array
  C<T>* dstE;      // lines: last line of D_k  at dstE[k sk + col sr + j sj]
  C<T>* dstF;      // lines: first line of D_k at dstF[k sk + col sr + j sj]
  size_t sk, sr, sj;
  C<T>* yscr;      // nslices * ngroups * slice_scratch_elems(L, W)
  size_t stage;    // LDS stage buffer length (slice_stage_elems)
  T* mfma_scr;     // scratch of the matrix-core path (batches of more than 8)
};
// Scratch (complex elements) of one workgroup of W waves.
template <typename T>
size_t slice_scratch_elems(int L, int W);
// LDS stage buffer length for slices with at most tmax lines and factor stride fstride_max.
template <typename T>
size_t slice_stage_elems(int tmax, int fstride_max);
// Dynamic LDS bytes of one workgroup (0 for an unsupported W); big: the
// launch holds a slice of more than 16 lines.
template <typename T>
size_t slice_lds(bool big, size_t stage, int W);
// One workgroup per (group of W right-hand sides, slice), one wave per
// right-hand side; W in {1, 4, 8}; slices of up to 32 lines, more than 16
// only if big.
template <typename T>
hipError_t launch_slice_solves(const SliceSolveArgs<T>& a, int nslices, bool big, int W, int ngroups,
                               hipStream_t st);
// Interface maps in operand order: complex elements per slice, and the
// re-layout of row-major [nslices][L][L] maps into that order.
template <typename T>
size_t iface_map_stride(int L);
// Row length of the interface vectors lambda, mu ([nslices][nrhs][Lp], zero
// past L): L rounded up to a multiple of 16.
int iface_vec_stride(int L);
template <typename T>
hipError_t launch_swizzle_maps(const C<T>* src, C<T>* dst, int L, int nslices, hipStream_t st);
// ---- slice solves for batches on the matrix cores (slice_mfma.hip) ----
// Factors in operand order: per slice k and step j a forward record of
// mfma_wrec_elems(t, tw) complex values (W_j, then the D_k columns of
// S_j^{-1}) and a backward record of mfma_grec_elems(t) (G_j).
int mfma_row_tiles(int t);
int mfma_chunks(int t, int tw);
size_t mfma_wrec_elems(int t, int tw);
size_t mfma_grec_elems(int t);
template <typename T>
hipError_t launch_mfma_factors(const SliceTables& P, int L, int k, int t, int tw, const C<T>* FS, const C<T>* FG,
                               C<T>* MW, C<T>* MG, hipStream_t st);
template <typename T>
struct SliceMfmaArgs {
  SliceTables P;
  int L, b;
  const C<T>* MW;
  const C<T>* MG;
  const size_t* mw_off;  // per slice, complex elements
  const size_t* mg_off;
  const int* nsd;        // per slice: chunks of 4 right-hand-side lines
  const int* ys_unit;    // per slice: sum of the row tiles of the slices before it
  const C<T>* Hm;
  const C<T>* Hp;
  int slice0, nrhs;
  int src_kind;
  const C<T>* src;
  int col0;
  int dst_kind;
  C<T>* dst;
  C<T>* dstE;
  C<T>* dstF;
  size_t sk, sr, sj;
  T* yscr;               // (sum of row tiles) x ceil(nrhs/16) x (L+1) x 512 scalars
};
// Slices [slice0, slice0 + nslices) for a batch, one wave per 16 columns.
template <typename T>
hipError_t launch_slice_mfma(const SliceMfmaArgs<T>& a, int nslices, hipStream_t st);

// One product of an interface step, y = add - M x, every pointer already at
// its slice: M one L x L map in operand order, x, add, y [nrhs][Lp] (in place
// allowed, y == add).
template <typename T>
struct IfaceProd {
  const C<T>* M;
  const C<T>* add;
  const C<T>* x;
  C<T>* y;
};
constexpr int kIfaceMaxProds = 4;
template <typename T>
struct IfaceProds {
  IfaceProd<T> p[kIfaceMaxProds];
};
// Up to kIfaceMaxProds independent products in one launch (blockIdx.z picks
// one; none may write what another reads). mfma: on the matrix cores, one
// workgroup per 16 x 16 output tile; else vector dot products (nrhs <= 4,
// hipErrorInvalidValue above).
template <typename T>
hipError_t launch_iface_prods(const IfaceProd<T>* prods, int nprods, int L, int nrhs, bool mfma, hipStream_t st);
// y_k = add_k - M_k x_{k+xoff} for k = kbeg .. kbeg+kcount-1, maps mstride
// apart (iface_map_stride(L)), vectors vstride apart; with M2 (kcount = 1)
// the same launch also forms y2_k = add2_k - M2_k x_{k+xoff}.
template <typename T>
hipError_t launch_iface_step(const C<T>* M, const C<T>* add, const C<T>* x, C<T>* y, int L, int nrhs, int kbeg,
                             int kcount, size_t mstride, size_t vstride, int xoff, bool mfma, hipStream_t st,
                             const C<T>* M2 = nullptr, const C<T>* add2 = nullptr, C<T>* y2 = nullptr);
// f -= J_F Hm_k lambda_{k-1} + J_E Hp_k mu_{k+1} on slices [k0, k1)
template <typename T>
hipError_t launch_couple(const SliceTables& P, int L, int b, const C<T>* Hm, const C<T>* Hp, const C<T>* lam,
                         const C<T>* mu, int nrhs, C<T>* f, int k0, int k1, hipStream_t st);

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
// The same dot products grouped by a shared y: group g forms
// out[pbase_g + k] = sum conj(x_{g,k}) y_g for k < count_g <= kDotGroup, reading
// y_g once for all of them; every product is summed in the same order as
// launch_dots would (bitwise the same results). npairs: the number of out
// entries the groups cover, each once.
constexpr int kDotGroup = 8;
struct DotGroup {
  const double2* y;
  const double2* x[kDotGroup];
  int count;
  int pbase;
};
hipError_t launch_mdots(const DotGroup* groups, int ngroups, int npairs, size_t N, double2* partials, double2* out,
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
hipError_t launch_axpys(const AxpyOut* outs, int nout, const AxpyTerm<TX>* terms, const double2* coefs,
                        size_t N, hipStream_t st);
// launch_axpys that also forms norm2[o] = ||y_o||^2 of every updated output
// (in the pass that writes it; fixed-order reduction through partials, which
// needs nout * 256 entries)
hipError_t launch_axpys_norms(const AxpyOut* outs, int nout, const AxpyTerm<double>* terms, const double2* coefs,
                              size_t N, double2* partials, double2* norm2, hipStream_t st);
// dst[p] = cast(src[p]) for npairs contiguous batches of N entries.
template <typename TD, typename TS>
hipError_t launch_copy_cast(C<TD>* const* dst, const C<TS>* const* src, int npairs, size_t N,
                            hipStream_t st);
// grad = -omega^2 Re sum_j psi_j * nu_j (psi, nu: [nrhs][N])
hipError_t launch_adjoint_product(const double2* psi, const double2* nu, int nrhs, size_t N,
                                  double omega2, double* grad, hipStream_t st);
// dst = conj(src) over N entries (float64)
hipError_t launch_conj(double2* dst, const double2* src, size_t N, hipStream_t st);
// out[t] = in[t] * s[t], t < n (complex coefficients, real factors)
hipError_t launch_scale_coefs(const double2* in, const double* s, double2* out, int n, hipStream_t st);
// u = x and psi = x + y (y null: psi = x) elementwise over N, float64: a
// solve's output and the total field kept for the adjoint, in one pass
hipError_t launch_solution_out(double2* u, double2* psi, const double2* x, const double2* y, size_t N,
                               hipStream_t st);
// dst[i] = src[i] over count values, converting the precision
template <typename TD, typename TS>
hipError_t launch_cast_flat(C<TD>* dst, const C<TS>* src, size_t count, hipStream_t st);
// partials[c][0..kDotBlocks) of ||x_c||^2 for the ncols columns of [ncols][N]
hipError_t launch_colnorm2(const double2* x, int ncols, size_t N, double* partials, hipStream_t st);
// out[i] = sum of parts[c][i] over c < nparts, for i < count (fixed order)
hipError_t launch_sum_parts(const double2* parts, int nparts, size_t count, double2* out, hipStream_t st);
// k plane waves exp(i omega (cos t_j x1 + sin t_j x2)), t_j = 2 pi j / k, on the interior grid: [k][n][n]
hipError_t launch_plane_waves(double2* out, int n, double omega, int k, hipStream_t st);

// ---- 3D sparsified system and sweep (slab3.hip) ----
// Float64 stencil tables of the 3D method on the device.
struct Stencil3 {
  const double2* alpha;  // 27
  const double2* beta;   // 27
  const double2* gglob;  // [(2b+1)^3][27]
  const double2* gaux;   // [b][2b+1][2b+1][ns][27]
  const int* kmap;       // [L]^3
  const double* m;       // [n]^3
  int n, b, L, ns;
  double omega2;
};
// A slab: lines [first, hi], D = [lo, hi], t lines, naux = lo - first, nb = t L.
struct Slab3 {
  int first, lo, hi, t, naux, nb;
};
// Largest block (slab lines x L) the slab factorization takes: a two-column
// sub-panel of this many rows fills the LDS of one workgroup.
constexpr int kSlab3MaxBlock = 4800;
// Float64 work arrays of a slab's factorization.
struct Slab3Work {
  double2* S;   // [nb][nb] block being inverted
  double2* W;   // [nb][nb] S_{j-1}^{-1} C_{j-1}
  double2* Sp;  // [nb][nb] S_{j-1}^{-1}
  double2* Xr;  // [32][nb] pivot rows of a panel
  double2* cf;  // [3][nb][9] block coefficients A_j, B_j, C_{j-1}
  int* piv;     // [nb] row interchanges
  int* perm;    // [nb] column order of the inverse
  int dir;      // +1: the slab's top chain (blocks 0 .. m-1), -1: its bottom chain (L-1 .. m+1)
};
// The blocks one launch of a slab solve works on (the two chains' current
// blocks, or the middle block alone) and the coupling terms each takes.
struct Slab3Step {
  int nt;
  int j[2];
  int terms[2];
};
// One slab solve: factors, coefficients, work vectors, and where its
// right-hand side comes from and its D part goes to.
template <typename T>
struct Slab3Apply {
  Slab3 p;
  int L, nrhs;
  const C<T>* F;    // [L][nb][nb] S_j^{-1}
  const C<T>* cbc;  // [L][2][nb][9] B_j, C_j
  const C<T>* cm;   // [L][L][9] coupling of line lo to lo - 1
  const C<T>* cp;   // [L][L][9] coupling of line hi to hi + 1
  C<T>* Y;          // [nrhs][L][nb]
  C<T>* z;          // [2][nrhs][nb], one per block of a step
  const C<T>* src;  // D part of the right-hand side, (rhs, aD, e2, e3) at rhs*src_rs + (aD L + e2) L + e3; may be null
  size_t src_rs;
  const C<T>* cu;   // line lo - 1 (cmode 1) or hi + 1 (cmode 2) of the sweep field, rhs stride cu_rs
  size_t cu_rs;
  int cmode;        // 0 none, 1: minus coupling on the first line of D, 2: plus coupling on the last line
  C<T>* dst;        // D part of the result, same layout as src with dst_rs
  size_t dst_rs;
  int dop;          // 0 store, 1 subtract
};
template <typename T>
hipError_t launch3_apply_Q(const Stencil3& S, const C<T>* r, int nrhs, C<T>* f, hipStream_t st);
template <typename T>
hipError_t launch3_apply_H(const Stencil3& S, const C<T>* u, int nrhs, C<T>* y, hipStream_t st);
template <typename T>
hipError_t launch3_extract(const C<T>* u, int n, int b, int nrhs, C<T>* z, hipStream_t st);
// S_j^{-1} of every block of every slab by two-ended elimination (top and
// bottom chain per slab toward the middle block L/2). nentries = 2 x slabs:
// entry 2k is slab k's top chain, 2k+1 its bottom chain (device arrays slabs,
// works, factors: the slab's descriptor, work and factor base per entry);
// status > 0: zero pivot in slab status-1
template <typename T>
hipError_t launch3_factor(const Stencil3& S, const Slab3* slabs, const Slab3Work* works, int nentries, int maxnb,
                          C<T>* const* factors, int* status, hipStream_t st);
template <typename T>
hipError_t launch3_apply_coefs(const Stencil3& S, const Slab3* slabs, int nslab, int maxnb, C<T>* const* cbc,
                               C<T>* const* cm, C<T>* const* cpl, hipStream_t st);
template <typename T>
hipError_t launch3_slab_solve(const Slab3Apply<T>& A, hipStream_t st);

}  // namespace lsw
