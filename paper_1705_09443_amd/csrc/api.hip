// C ABI of the solver: setup (Algorithm 1), the right-preconditioned
// flexible GMRES loop in float64 around the applies (Sec. 2.5), the adjoint
// gradient, and the per-operator entry points.
#include <algorithm>
#include <chrono>
#include <limits>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocblas/rocblas.h>

#include "../../include/lsweep.h"
#include "kernels.hpp"
#include "setup_host.hpp"

namespace lsw {

namespace {
thread_local std::string g_error;
}
void set_error(const std::string& msg) { g_error = msg; }
const char* get_error() { return g_error.c_str(); }

namespace {

// Device buffer owned by the handle.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      std::swap(p, o.p);
      std::swap(bytes, o.bytes);
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t nbytes) {
    if (nbytes <= bytes && p) return hipSuccess;
    release();
    if (nbytes == 0) nbytes = 16;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e == hipSuccess) bytes = nbytes;
    else p = nullptr;
    return e;
  }
  void swap(DBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
  template <typename X>
  X* as() const { return static_cast<X*>(p); }
};

// Descriptor tables of one phase of an iteration, written into pinned host
// memory and sent to the device with one asynchronous copy, so that the host
// never waits for the device to drain just to upload them. The caller
// rewrites a stage only once the copy and every launch that reads its device
// copy have completed (after a later synchronisation).
struct Stage {
  char* host = nullptr;
  DBuf dev;
  size_t cap = 0, used = 0;
  Stage() = default;
  Stage(const Stage&) = delete;
  Stage& operator=(const Stage&) = delete;
  ~Stage() {
    if (host) (void)hipHostFree(host);
  }
  hipError_t alloc(size_t bytes) {
    if (bytes <= cap && host) return hipSuccess;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host), bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = dev.alloc(bytes);
    if (e != hipSuccess) return e;
    cap = bytes;
    return hipSuccess;
  }
  void reset() { used = 0; }
  // appends the table (256-byte aligned) and returns its device address
  template <typename X>
  X* put(const X* data, size_t count) {
    const size_t off = (used + 255) & ~size_t(255), bytes = count * sizeof(X);
    if (off + bytes > cap) return nullptr;
    if (bytes) std::memcpy(host + off, data, bytes);
    used = off + bytes;
    return reinterpret_cast<X*>(dev.as<char>() + off);
  }
  template <typename X>
  X* put(const std::vector<X>& v) {
    return put(v.data(), v.size());
  }
  hipError_t flush(hipStream_t st) {
    if (!used) return hipSuccess;
    return hipMemcpyAsync(dev.p, host, used, hipMemcpyHostToDevice, st);
  }
};

#define LSW_ALLOC(buf, nbytes)                                                      \
  do {                                                                              \
    if ((buf).alloc(nbytes) != hipSuccess) {                                        \
      (void)hipGetLastError();                                                      \
      lsw::set_error("device allocation of " + std::to_string((size_t)(nbytes)) +   \
                     " bytes failed");                                              \
      return LS_E_NOMEM;                                                            \
    }                                                                               \
  } while (0)

// Kernel choice for a batch of right-hand sides: slice solves on the vector
// ALUs with 1, 4 or 8 right-hand sides per workgroup, or (16) on the matrix
// cores in 16-column tiles; interface products as vector dot products (0, at
// most 4 columns) or on the matrix cores (1).
struct KernelChoice {
  int slice;
  int iface;
};
// batch sizes with an entry of their own; larger batches follow the last
constexpr int kChoiceMax = 256;
// lines of a 3D slab subproblem at most (its dense blocks have t L rows)
constexpr int kSlab3MaxLines = 32;

}  // namespace
}  // namespace lsw

using namespace lsw;

// 3D state of a handle (grid dim 3): host tables, the Green's spectrum
// octant, the stencil tables, and per slab the factors S_j^{-1}, the
// apply-time block coefficients and the couplings to the neighbouring slabs.
struct Sweep3 {
  HostSetup3 H;
  std::vector<Slab3> slabs;
  int maxnb = 0;
  DBuf alpha, beta, gglob, gaux, kmap, khat, khat32, w1, w2, Y, z;
  std::vector<DBuf> F, cbc, cm, cp;
};

struct ls_handle {
  int device = 0;
  int dim = 2;
  std::unique_ptr<Sweep3> s3;
  hipStream_t st = nullptr;
  ls_options opt{};
  HostSetup H;
  int n = 0, b = 0, w = 0, L = 0, P = 0, ns = 0, nslices = 0, prec = LS_FP64;
  double omega = 0;
  size_t N = 0, E = 0;
  // tables
  DBuf m, m32, khat, khat32, tw, tw32, alpha, beta, gglob, gaux, kmap;
  DBuf s_lo, s_hi, s_first, s_t, s_naux, s_org, s_dir, s_prev, s_next, s_nlam, fs_off, fg_off, FS, FG, Hm, Hp,
      status;
  // interface maps M_k, P_k, N_k ([nslices][L][L]); two fronts: also
  // Q = E T_mid J_E Hp_mid of the middle slice (one map)
  DBuf IM, IP, IN, IQ;
  // grid order -> table index of every slice (the two-front table order differs)
  std::vector<int> tbl_of_grid;
  // per slice on the host: line count t and forward factor stride
  std::vector<int> t_host, fstride_host, tw_host;
  // kernel choice per batch size [0, kChoiceMax], and what the autotuner measured
  std::vector<KernelChoice> choice;
  std::vector<ls_tune_layer> tune_w;
  std::vector<ls_tune_kernels> tune_k;
  // factors in matrix-core operand order (slice_mfma.hip), per-slice offsets,
  // chunk counts and scratch units; total scratch units over all slices
  DBuf MW, MG, mw_off, mg_off, mnsd, mys_unit;
  int mys_units = 0;
  // workspaces
  int cap = 0;  // right-hand sides the workspaces hold
  DBuf fftw64, fftw32, fext, uext, yscr, vin, zout, aout, lam, mu, sscr, mscr;
  DBuf V, Z, W, X, G, R, T1, T2;
  DBuf pairs, groups, partials, coefs, outs, terms64, terms32, ptrs_a, ptrs_b;
  // descriptor stages of the Arnoldi step: before and after its readback
  Stage stage_main;
  // the Krylov loop's operator: false, the Lippmann-Schwinger operator A on
  // the interior grid with P = extract(sweep(Q .)); true, the sparse system H
  // on the extended grid with the sweep alone (ls_solve_H)
  bool hmode = false;
  // block flexible GMRES (ls_options.block_size > 1): library GEMM handle
  // on st and the small coefficient matrices of every block
  rocblas_handle blas = nullptr;
  DBuf bcoef, gpart;
  // adjoint state
  int last_nrhs = 0;
  DBuf psi;
  // captured interface recurrences, one graph per (batch size, precision)
  hipStream_t cst = nullptr;
  // two fronts: the right front's recurrences run on st3, ordered by these
  hipStream_t st3 = nullptr;
  hipEvent_t evPA = nullptr, evR = nullptr, evM = nullptr, evR2 = nullptr;
  // second stream for the last slice's solves, and the events that order it
  hipStream_t st2 = nullptr;
  hipEvent_t evQ = nullptr, evA = nullptr, evL = nullptr, evC = nullptr;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  // kernel timing
  bool profiling = false;
  struct Rec {
    int kind;
    int cols;  // right-hand-side columns the launch processed
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  ~ls_handle() {
    drop_graphs();
    if (blas) (void)rocblas_destroy_handle(blas);
    if (cst) (void)hipStreamDestroy(cst);
    if (st3) (void)hipStreamDestroy(st3);
    if (st2) (void)hipStreamDestroy(st2);
    for (hipEvent_t e : {evQ, evA, evL, evC, evPA, evR, evM, evR2})
      if (e) (void)hipEventDestroy(e);
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }

  StencilTables stencils() const {
    StencilTables s;
    s.alpha = alpha.as<double2>();
    s.beta = beta.as<double2>();
    s.gglob = gglob.as<double2>();
    s.gaux = gaux.as<double2>();
    s.kmap = kmap.as<int>();
    s.m = m.as<double>();
    s.n = n;
    s.b = b;
    s.L = L;
    s.ns = ns;
    s.omega2 = omega * omega;
    return s;
  }
  SliceTables slices() const {
    SliceTables t;
    t.lo = s_lo.as<int>();
    t.hi = s_hi.as<int>();
    t.first = s_first.as<int>();
    t.t = s_t.as<int>();
    t.naux = s_naux.as<int>();
    t.org = s_org.as<int>();
    t.dir = s_dir.as<int>();
    t.prev = s_prev.as<int>();
    t.next = s_next.as<int>();
    t.next_lam = s_nlam.as<int>();
    t.fs_off = fs_off.as<size_t>();
    t.fg_off = fg_off.as<size_t>();
    t.nslices = nslices;
    return t;
  }
};

// The 3D operator alone: Green's spectrum octant, medium and work arrays.
struct ls_op3 {
  int device = 0;
  hipStream_t st = nullptr;
  int n = 0, P = 0;
  double omega = 0;
  DBuf m, m32, khat, khat32, tw, tw32, w1, w2;
  int cap = 0;  // right-hand sides the work arrays hold
};

namespace {

enum KernelKind {
  kKSweep = 0,
  kKFft,
  kKQ,
  kKExtract,
  kKFactor,
  kKSlices,
  kKIface,
  kKSlicesLast,
  kKGram,
  kKGramUpd,
  kKFft64,
  kKNumKinds
};
const char* kKindNames[kKNumKinds] = {"sweep",        "fft_convolve",      "stencil_Q",  "extract",
                                      "factor",       "slice_solves",      "interface",  "slice_solves_last",
                                      "block_gram",   "block_update",      "fft_convolve_c128"};

hipEvent_t take_event(ls_handle* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Brackets one launch with events on the handle's stream when profiling.
struct Timed {
  ls_handle* h;
  int kind, cols;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timed(ls_handle* hh, int k, int c, hipStream_t stream = nullptr) : h(hh), kind(k), cols(c), s(stream ? stream : hh->st) {
    if (h->profiling) {
      a = take_event(h);
      (void)hipEventRecord(a, s);
    }
  }
  ~Timed() {
    if (a) {
      hipEvent_t b = take_event(h);
      (void)hipEventRecord(b, s);
      h->recs.push_back({kind, cols, a, b});
    }
  }
};

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static const double2* khat(const ls_handle* h) { return h->khat.as<double2>(); }
  static const double2* tw(const ls_handle* h) { return h->tw.as<double2>(); }
  static const double* m(const ls_handle* h) { return h->m.as<double>(); }
  static double2* fftw(ls_handle* h) { return h->fftw64.as<double2>(); }
  static const double2* khat3(const ls_handle* h) { return h->s3->khat.as<double2>(); }
};
template <>
struct Prec<float> {
  static const float2* khat(const ls_handle* h) { return h->khat32.as<float2>(); }
  static const float2* tw(const ls_handle* h) { return h->tw32.as<float2>(); }
  static const float* m(const ls_handle* h) { return h->m32.as<float>(); }
  static float2* fftw(ls_handle* h) { return h->fftw32.as<float2>(); }
  static const float2* khat3(const ls_handle* h) { return h->s3->khat32.as<float2>(); }
};

ls_status check_handle(const ls_handle* h) {
  if (!h) {
    set_error("null handle");
    return LS_E_INVALID;
  }
  return LS_OK;
}

// Right-hand sides per workgroup of the slice solves.
int rhs_group(int nrhs) { return nrhs == 1 ? 1 : (nrhs <= 4 ? 4 : 8); }

// Batches above this many columns take the matrix-core slice solves.
constexpr int kMfmaMinCols = 8;

// Default kernel choice: the fastest measured on MI355X for the 1023^2 grid
// (b = 12, w = 4). complex64: vector slice solves up to 4 right-hand sides
// (one per workgroup up to 2), matrix-core interface products from one;
// complex128: the vector forms for one right-hand side, matrix-core slice
// solves from 3 and interface products from 2.
KernelChoice default_choice(int nb, bool fp64) {
  if (fp64) return {nb == 1 ? 1 : nb == 2 ? 4 : 16, nb == 1 ? 0 : 1};
  return {nb <= 2 ? 1 : nb <= 4 ? 4 : 16, 1};
}

void set_default_choices(ls_handle* h) {
  h->choice.resize(kChoiceMax + 1);
  for (int nb = 0; nb <= kChoiceMax; ++nb) h->choice[nb] = default_choice(std::max(nb, 1), h->prec == LS_FP64);
}

KernelChoice choice_for(const ls_handle* h, int nb) { return h->choice[std::min(std::max(nb, 1), kChoiceMax)]; }

// Scratch of the matrix-core slice solves for ncols columns: the forward
// results of every slice, (L+1) x 512 scalars per row tile and 16 columns.
size_t mfma_scratch_bytes(const ls_handle* h, int ncols, size_t cs) {
  return (size_t)h->mys_units * ((ncols + 15) / 16) * (size_t)(h->L + 1) * 512 * (cs / 2);
}

// Workspaces sized for nrhs right-hand sides.
ls_status ensure_workspace(ls_handle* h, int nrhs) {
  if (nrhs <= h->cap) return LS_OK;
  h->drop_graphs();  // captured launches refer to the old buffers
  const size_t N = h->N, E = h->E;
  const int rs = h->opt.restart;
  const size_t cs = h->prec == LS_FP64 ? sizeof(double2) : sizeof(float2);
  if (h->dim == 3) {
    Sweep3& s3 = *h->s3;
    // FFT work sized for complex128 so that both precisions fit
    LSW_ALLOC(s3.w1, (size_t)nrhs * fft3_w1_elems(h->n) * sizeof(double2));
    LSW_ALLOC(s3.w2, (size_t)nrhs * fft3_w2_elems(h->n) * sizeof(double2));
    LSW_ALLOC(h->fext, (size_t)nrhs * E * cs);
    LSW_ALLOC(h->uext, (size_t)nrhs * E * cs);
    LSW_ALLOC(s3.Y, (size_t)nrhs * h->L * s3.maxnb * cs);
    LSW_ALLOC(s3.z, (size_t)2 * nrhs * s3.maxnb * cs);
  } else {
    LSW_ALLOC(h->fftw64, fft_work_elems<double>(h->n, nrhs) * sizeof(double2));
    LSW_ALLOC(h->fftw32, fft_work_elems<float>(h->n, nrhs) * sizeof(float2));
    LSW_ALLOC(h->fext, (size_t)nrhs * E * cs);
    LSW_ALLOC(h->uext, (size_t)nrhs * E * cs);
    LSW_ALLOC(h->yscr, (size_t)nrhs * h->L * 32 * cs);
    // interface vectors: rows padded to whole 16-blocks; the padding stays zero
    const size_t vbytes = (size_t)h->nslices * nrhs * iface_vec_stride(h->L) * cs;
    LSW_ALLOC(h->lam, vbytes);
    LSW_ALLOC(h->mu, vbytes);
    LSW_HIP_TRY(hipMemsetAsync(h->lam.p, 0, vbytes, h->st));
    LSW_HIP_TRY(hipMemsetAsync(h->mu.p, 0, vbytes, h->st));
    // slice-solve scratch: groups of up to 8 waves, one per right-hand side
    LSW_ALLOC(h->sscr, (size_t)h->nslices * std::max(4, nrhs + 7) * slice_scratch_elems<double>(h->L, 1) * cs);
  }
  LSW_ALLOC(h->vin, (size_t)nrhs * N * cs);
  LSW_ALLOC(h->zout, (size_t)nrhs * N * cs);
  LSW_ALLOC(h->aout, (size_t)nrhs * N * cs);
  LSW_ALLOC(h->V, (size_t)nrhs * (rs + 1) * N * sizeof(double2));
  // the block method keeps its directions in complex128 (X += Z Y is one GEMM)
  LSW_ALLOC(h->Z, (size_t)nrhs * rs * N * (h->opt.block_size > 1 ? sizeof(double2) : cs));
  LSW_ALLOC(h->W, (size_t)nrhs * N * sizeof(double2));
  LSW_ALLOC(h->X, (size_t)nrhs * N * sizeof(double2));
  LSW_ALLOC(h->G, (size_t)nrhs * N * sizeof(double2));
  LSW_ALLOC(h->R, (size_t)nrhs * N * sizeof(double2));
  LSW_ALLOC(h->T1, (size_t)nrhs * N * sizeof(double2));
  LSW_ALLOC(h->T2, (size_t)nrhs * N * sizeof(double2));
  const size_t maxpairs = (size_t)nrhs * (rs + 2);
  LSW_ALLOC(h->pairs, maxpairs * sizeof(DotPair));
  LSW_ALLOC(h->groups, maxpairs * sizeof(DotGroup));
  // dot-product partials: kDotBlocks per pair, or 256 per norm of an update
  LSW_ALLOC(h->partials, std::max(maxpairs * (size_t)kDotBlocks, (size_t)nrhs * 256) * sizeof(double2));
  LSW_ALLOC(h->coefs, (4 * maxpairs + 16) * sizeof(double2));
  LSW_ALLOC(h->outs, (size_t)nrhs * 2 * sizeof(AxpyOut));
  // the terms of one step's update and normalisation, and of the solution
  // and residual updates at a cycle's end
  LSW_ALLOC(h->terms64, (2 * maxpairs + 2 * nrhs) * sizeof(AxpyTerm<double>));
  LSW_ALLOC(h->terms32, (2 * maxpairs + 2 * nrhs) * sizeof(AxpyTerm<float>));
  LSW_ALLOC(h->ptrs_a, (size_t)nrhs * sizeof(void*));
  LSW_ALLOC(h->ptrs_b, (size_t)nrhs * sizeof(void*));
  {
    // 3 pointer pairs per right-hand side, dot groups, update terms and
    // coefficient factors of up to maxpairs products, outputs and one unit
    // term per right-hand side, alignment slack (terms and outputs with room
    // to spare)
    const size_t main_bytes = (size_t)nrhs * 6 * sizeof(void*) +
                              maxpairs * (sizeof(DotGroup) + 2 * sizeof(AxpyTerm<double>) + sizeof(double)) +
                              (size_t)nrhs * (2 * sizeof(AxpyOut) + sizeof(AxpyTerm<double>)) +
                              (size_t)(nrhs + 1) * sizeof(int) + sizeof(double2) + 16 * 256;
    if (h->stage_main.alloc(main_bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation for the descriptor stages failed");
      return LS_E_NOMEM;
    }
  }
  h->cap = nrhs;
  return LS_OK;
}

// Scratch of the matrix-core slice solves, sized for the workspace's batch
// (at least ncols columns); grown on first use.
ls_status ensure_mscr(ls_handle* h, int ncols) {
  const size_t cs = h->prec == LS_FP64 ? sizeof(double2) : sizeof(float2);
  const size_t need = mfma_scratch_bytes(h, std::max(ncols, h->cap), cs);
  if (h->mscr.p && h->mscr.bytes >= need) return LS_OK;
  // launches in flight may still read the old buffer
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  if (h->st2) LSW_HIP_TRY(hipStreamSynchronize(h->st2));
  LSW_ALLOC(h->mscr, need);
  return LS_OK;
}

// Host -> device copy of a small descriptor table. Synchronous, so the host
// vector may be reused as soon as this returns.
template <typename X>
ls_status upload(const ls_handle* h, DBuf& dst, const std::vector<X>& src) {
  if (src.empty()) return LS_OK;
  if (src.size() * sizeof(X) > dst.bytes) {
    set_error("internal: descriptor table larger than its device buffer");
    return LS_E_INVALID;
  }
  LSW_HIP_TRY(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice, h->st));
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

// ---- the applies, on contiguous batches ------------------------------------
template <typename T>
// y64, xp (2D only): per-right-hand-side output (float64) and input grids
ls_status apply_A(ls_handle* h, const C<T>* x, int nb, C<T>* y, double2* const* y64 = nullptr,
                  const C<T>* const* xp = nullptr) {
  Timed tm(h, sizeof(T) == sizeof(float) ? kKFft : kKFft64, nb);
  if (h->dim == 3) {
    if (y64 || xp) {
      set_error("internal: per-right-hand-side grids in a 3D operator apply");
      return LS_E_STATE;
    }
    LSW_HIP_TRY(launch_convolve3<T>(x, Prec<T>::m(h), h->n, nb, Prec<T>::khat3(h), Prec<T>::tw(h), (T)1,
                                    (T)(h->omega * h->omega), h->s3->w1.as<C<T>>(), h->s3->w2.as<C<T>>(), y, h->st));
    return LS_OK;
  }
  LSW_HIP_TRY(launch_convolve<T>(x, Prec<T>::m(h), h->n, nb, Prec<T>::khat(h), Prec<T>::tw(h), (T)1,
                                 (T)(h->omega * h->omega), Prec<T>::fftw(h), y, h->st, y64, xp));
  return LS_OK;
}

template <typename T>
SliceSolveArgs<T> slice_args(ls_handle* h) {
  SliceSolveArgs<T> a{};
  a.P = h->slices();
  a.L = h->L;
  a.b = h->b;
  a.FS = h->FS.as<C<T>>();
  a.FG = h->FG.as<C<T>>();
  a.Hm = h->Hm.as<C<T>>();
  a.Hp = h->Hp.as<C<T>>();
  return a;
}

// All slices of [k0, k1) solved in one launch: kernel 16 on the matrix cores,
// else on the vector ALUs with at most kernel (1, 4 or 8) right-hand sides
// (waves) per workgroup, fewer if the LDS would not fit.
template <typename T>
ls_status solve_slices(ls_handle* h, SliceSolveArgs<T> a, int k0, int k1, int kernel, hipStream_t st = nullptr) {
  if (k0 >= k1) return LS_OK;
  if (!st) st = h->st;
  if (kernel == 16) {
    if (!a.mfma_scr) {
      set_error("internal: no scratch for the matrix-core slice solves");
      return LS_E_STATE;
    }
    SliceMfmaArgs<T> m{};
    m.P = a.P;
    m.L = a.L;
    m.b = a.b;
    m.MW = h->MW.as<C<T>>();
    m.MG = h->MG.as<C<T>>();
    m.mw_off = h->mw_off.as<size_t>();
    m.mg_off = h->mg_off.as<size_t>();
    m.nsd = h->mnsd.as<int>();
    m.ys_unit = h->mys_unit.as<int>();
    m.Hm = a.Hm;
    m.Hp = a.Hp;
    m.slice0 = k0;
    m.nrhs = a.nrhs;
    m.src_kind = a.src_kind;
    m.src = a.src;
    m.col0 = a.col0;
    m.dst_kind = a.dst_kind;
    m.dst = a.dst;
    m.dstE = a.dstE;
    m.dstF = a.dstF;
    m.sk = a.sk;
    m.sr = a.sr;
    m.sj = a.sj;
    m.yscr = a.mfma_scr;
    LSW_HIP_TRY(launch_slice_mfma<T>(m, k1 - k0, st));
    return LS_OK;
  }
  int f16 = 0, f32 = 0;
  for (int k = k0; k < k1; ++k) {
    int& f = h->t_host[k] > 16 ? f32 : f16;
    f = std::max(f, h->fstride_host[k]);
  }
  const bool big = f32 > 0;
  a.slice0 = k0;
  a.stage = std::max(f16 ? slice_stage_elems<T>(16, f16) : 0, big ? slice_stage_elems<T>(32, f32) : 0);
  int W = kernel;
  while (W > 1 && slice_lds<T>(big, a.stage, W) > 163840) W = W == 8 ? 4 : 1;
  if (slice_lds<T>(big, a.stage, W) > 163840) {
    set_error("slice subproblem too large for the LDS of one workgroup");
    return LS_E_INVALID;
  }
  LSW_HIP_TRY(launch_slice_solves<T>(a, k1 - k0, big, W, (a.nrhs + W - 1) / W, st));
  return LS_OK;
}

Stencil3 stencil3(const ls_handle* h) {
  const Sweep3& s = *h->s3;
  Stencil3 S;
  S.alpha = s.alpha.as<double2>();
  S.beta = s.beta.as<double2>();
  S.gglob = s.gglob.as<double2>();
  S.gaux = s.gaux.as<double2>();
  S.kmap = s.kmap.as<int>();
  S.m = h->m.as<double>();
  S.n = h->n;
  S.b = h->b;
  S.L = h->L;
  S.ns = h->ns;
  S.omega2 = h->omega * h->omega;
  return S;
}

// Solve of slab k's subproblem for nb right-hand sides: factors and work
// vectors filled in; source, couplings and destination left to the caller.
template <typename T>
Slab3Apply<T> slab3_args(ls_handle* h, int k, int nb) {
  Sweep3& s = *h->s3;
  Slab3Apply<T> a{};
  a.p = s.slabs[k];
  a.L = h->L;
  a.nrhs = nb;
  a.F = s.F[k].as<C<T>>();
  a.cbc = s.cbc[k].as<C<T>>();
  a.cm = s.cm[k].as<C<T>>();
  a.cp = s.cp[k].as<C<T>>();
  a.Y = s.Y.as<C<T>>();
  a.z = s.z.as<C<T>>();
  return a;
}

// z = P r in 3D (Algorithm 2 slab by slab): f = Q r, forward sweep
// u_k = T_k (f_k - H_[k,k-1] u_{k-1}), backward sweep u_k -= T_k H_[k,k+1] u_{k+1},
// z = u on I.
template <typename T>
ls_status apply_P3(ls_handle* h, const C<T>* r, int nb, C<T>* z) {
  const Stencil3 S = stencil3(h);
  Sweep3& s = *h->s3;
  const int L = h->L, b = h->b, nl = (int)s.slabs.size();
  const size_t LL = (size_t)L * L, E = LL * L;
  C<T>* f = h->fext.as<C<T>>();
  C<T>* u = h->uext.as<C<T>>();
  {
    Timed tm(h, kKQ, nb);
    LSW_HIP_TRY(launch3_apply_Q<T>(S, r, nb, f, h->st));
  }
  // the sweep (f -> u on handle-owned buffers) as one graph per batch size
  // and precision: several thousand dependent launches per apply
  const std::pair<int, int> key(-(nb + 1), (int)sizeof(T));
  auto it = h->graphs.find(key);
  hipGraphExec_t ge = nullptr;
  if (it != h->graphs.end()) {
    ge = it->second;
  } else {
    if (!h->cst) LSW_HIP_TRY(hipStreamCreateWithFlags(&h->cst, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    LSW_HIP_TRY(hipStreamBeginCapture(h->cst, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int k = 0; k < nl && ce == hipSuccess; ++k) {
      const Slab3& p = s.slabs[k];
      Slab3Apply<T> a = slab3_args<T>(h, k, nb);
      a.src = f + (size_t)(p.lo + b) * LL;
      a.src_rs = E;
      if (k > 0) {
        a.cu = u + (size_t)(p.lo - 1 + b) * LL;
        a.cu_rs = E;
        a.cmode = 1;
      }
      a.dst = u + (size_t)(p.lo + b) * LL;
      a.dst_rs = E;
      a.dop = 0;
      ce = launch3_slab_solve<T>(a, h->cst);
    }
    for (int k = nl - 2; k >= 0 && ce == hipSuccess; --k) {
      const Slab3& p = s.slabs[k];
      Slab3Apply<T> a = slab3_args<T>(h, k, nb);
      a.cu = u + (size_t)(p.hi + 1 + b) * LL;
      a.cu_rs = E;
      a.cmode = 2;
      a.dst = u + (size_t)(p.lo + b) * LL;
      a.dst_rs = E;
      a.dop = 1;
      ce = launch3_slab_solve<T>(a, h->cst);
    }
    const hipError_t ee = hipStreamEndCapture(h->cst, &g);
    LSW_HIP_TRY(ce);
    LSW_HIP_TRY(ee);
    const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    LSW_HIP_TRY(ie);
    h->graphs.emplace(key, ge);
  }
  {
    Timed tm(h, kKSlices, nb);
    LSW_HIP_TRY(hipGraphLaunch(ge, h->st));
  }
  {
    Timed tm(h, kKExtract, nb);
    LSW_HIP_TRY(launch3_extract<T>(u, h->n, b, nb, z, h->st));
  }
  return LS_OK;
}

// z = P r (Algorithm 2), interface schedule or slice by slice.
// r64 (2D interface schedule only): right-hand side q read from the float64
// grid r64[q] (a device pointer array), narrowed by the Q stencil (r unused);
// zp (same condition): right-hand side q of z written to the grid zp[q]
template <typename T>
ls_status sweep_core(ls_handle* h, int nb, C<T>* f, C<T>* u);

template <typename T>
ls_status apply_P(ls_handle* h, const C<T>* r, int nb, C<T>* z, const double2* const* r64 = nullptr,
                  C<T>* const* zp = nullptr) {
  if (h->dim == 3) return apply_P3<T>(h, r, nb, z);
  const StencilTables S = h->stencils();
  C<T>* f = h->fext.as<C<T>>();
  C<T>* u = h->uext.as<C<T>>();
  // the interface schedule keeps f and u interleaved ([L][L][nb]); the
  // sequential sweep takes them right-hand side by right-hand side
  const bool il = h->opt.sweep_schedule != LS_SWEEP_SEQUENTIAL;
  {
    Timed tm(h, kKQ, nb);
    LSW_HIP_TRY(launch_apply_Q<T>(S, r, nb, f, il, h->st, r64));
  }
  const ls_status e = sweep_core<T>(h, nb, f, u);
  if (e != LS_OK) return e;
  {
    Timed tm(h, kKExtract, nb);
    LSW_HIP_TRY(launch_extract<T>(h->n, h->b, u, nb, z, il, h->st, zp));
  }
  return LS_OK;
}

// z = the sweep applied to v (Algorithm 2, steps 3-8), both on the extended
// grid [nb][L][L]: the preconditioner of the sparse system H itself (the
// direct Helmholtz scheme's solve); the interface schedule works on the
// interleaved copies in the handle's buffers.
template <typename T>
ls_status apply_sweep_ext(ls_handle* h, const C<T>* v, int nb, C<T>* z) {
  if (h->opt.sweep_schedule == LS_SWEEP_SEQUENTIAL) return sweep_core<T>(h, nb, const_cast<C<T>*>(v), z);
  C<T>* f = h->fext.as<C<T>>();
  C<T>* u = h->uext.as<C<T>>();
  LSW_HIP_TRY(launch_interleave<T>(v, nb, h->E, f, true, h->st));
  const ls_status e = sweep_core<T>(h, nb, f, u);
  if (e != LS_OK) return e;
  LSW_HIP_TRY(launch_interleave<T>(u, nb, h->E, z, false, h->st));
  return LS_OK;
}

// The sweep on the handle's layout: f -> u, [nb][L][L] for the sequential
// schedule, interleaved [L][L][nb] for the interface schedule.
template <typename T>
ls_status sweep_core(ls_handle* h, int nb, C<T>* f, C<T>* u) {
  if (h->opt.sweep_schedule == LS_SWEEP_SEQUENTIAL) {
    Timed tm(h, kKSweep, nb);
    LSW_HIP_TRY(launch_sweep<T>(h->slices(), h->L, h->b, h->FS.as<C<T>>(), h->FG.as<C<T>>(), h->Hm.as<C<T>>(),
                                h->Hp.as<C<T>>(), f, u, h->yscr.as<C<T>>(), nb, kSweepFull, 0, h->st));
  } else {
    const int nl = h->nslices, L = h->L;
    const KernelChoice kc = choice_for(h, nb);
    const int R = kc.slice;
    const bool imf = kc.iface != 0 || nb > 4;
    if (R == 16) {
      const ls_status me = ensure_mscr(h, nb);
      if (me != LS_OK) return me;
    }
    C<T>* lam = h->lam.as<C<T>>();
    C<T>* mu = h->mu.as<C<T>>();
    const int Lp = iface_vec_stride(L);
    const size_t MS = iface_map_stride<T>(L), vs = (size_t)nb * Lp;
    SliceSolveArgs<T> a = slice_args<T>(h);
    a.nrhs = nb;
    a.yscr = h->sscr.as<C<T>>();
    a.mfma_scr = h->mscr.as<T>();
    // The last slice in table order (one front: the 32-line class with the far
    // PML, the longest solve; two fronts: the middle slice, the only one with
    // auxiliary lines on both sides) runs on a second stream: its phase A is
    // first needed after the whole lambda recurrence (one front: its P term;
    // two fronts: the middle step), and its phase C only needs the lambda of
    // its neighbours, so both overlap the recurrences on the main stream.
    const bool split = nl > 2;
    const int kmain = split ? nl - 1 : nl;
    // two fronts: p slices per front in table order, the middle slice last
    const bool two = h->H.fronts == 2;
    const int p = (nl - 1) / 2;
    auto phaseA = [&](int k0, int k1, hipStream_t s) -> ls_status {
      SliceSolveArgs<T> p = a;
      p.src_kind = kSrcGrid;
      p.src = f;
      p.dst_kind = kDstLines;
      p.dstE = lam;
      p.dstF = mu;
      p.sk = vs;  // lines into lambda / mu: [slice][nb][Lp]
      p.sr = Lp;
      p.sj = 1;
      return solve_slices<T>(h, p, k0, k1, R, s);
    };
    auto phaseC = [&](int k0, int k1, hipStream_t s) -> ls_status {
      SliceSolveArgs<T> p = a;
      p.src_kind = kSrcGrid;
      p.src = f;
      p.dst_kind = kDstGrid;
      p.dst = u;
      p.dstE = p.dstF = nullptr;
      return solve_slices<T>(h, p, k0, k1, R, s);
    };
    // graphs: part 0 the lambda recurrence (with the P terms of slices 1 ..
    // l-2), part 1 the last P term, the mu recurrence and the coupling of the
    // slices on the main stream. The last
    // slice's coupling (lambda term only) runs on the second stream after its
    // own phase A, which reads the line it changes.
    // Two fronts: the recurrences of the two fronts are independent until the
    // middle slice; they are launched directly (not captured), step by step
    // alternately on the main stream (left front) and a third stream (right
    // front), so that both hardware queues hold their front's chain at once.
    // (A captured graph's launch returns to the host only as its last
    // launches run, so two graphs on two streams ran one after the other; one
    // launch holding both fronts' products doubled its duration.)
    auto graph = [&](int part, hipGraphExec_t& out) -> ls_status {
      const std::pair<int, int> key((2 * nb + (int)imf) * 8 + part, (int)sizeof(T));
      auto it = h->graphs.find(key);
      if (it != h->graphs.end()) {
        out = it->second;
        return LS_OK;
      }
      const C<T>* IM = h->IM.as<C<T>>();
      const C<T>* IP = h->IP.as<C<T>>();
      const C<T>* IN = h->IN.as<C<T>>();
      const C<T>* Hm = h->Hm.as<C<T>>();
      const C<T>* Hp = h->Hp.as<C<T>>();
      hipGraph_t g = nullptr;
      LSW_HIP_TRY(hipStreamBeginCapture(h->cst, hipStreamCaptureModeThreadLocal));
      hipError_t ce = hipSuccess;
      if (part == 0) {
        // lambda_k = lambda_k - M_k lambda_{k-1}, and in the same launch the P
        // term of slice k, mu_k -= P_k lambda_{k-1}, which reads the same vector
        for (int k = 1; k <= nl - 2 && ce == hipSuccess; ++k)
          ce = launch_iface_step<T>(IM, lam, lam, lam, L, nb, k, 1, MS, vs, -1, imf, h->cst, IP, mu, mu);
      } else if (part == 1) {
        // the P term of the last slice (all of them when there are two slices)
        const int kp = nl > 2 ? nl - 1 : 1;
        ce = launch_iface_step<T>(IP, mu, lam, mu, L, nb, kp, nl - kp, MS, vs, -1, imf, h->cst);
        for (int k = nl - 2; k >= 1 && ce == hipSuccess; --k)
          ce = launch_iface_step<T>(IN, mu, mu, mu, L, nb, k, 1, MS, vs, +1, imf, h->cst);
        if (ce == hipSuccess) ce = launch_couple<T>(h->slices(), L, h->b, Hm, Hp, lam, mu, nb, f, 0, kmain, h->cst);
      }
      const hipError_t ee = hipStreamEndCapture(h->cst, &g);
      LSW_HIP_TRY(ce);
      LSW_HIP_TRY(ee);
      const hipError_t ie = hipGraphInstantiate(&out, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      LSW_HIP_TRY(ie);
      h->graphs.emplace(key, out);
      return LS_OK;
    };
    if (nl > 1) {
      // the executing streams before the capture stream (each takes a
      // hardware queue when created)
      if (split && !h->st2) {
        LSW_HIP_TRY(hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking));
        for (hipEvent_t* ev : {&h->evQ, &h->evA, &h->evL, &h->evC})
          LSW_HIP_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming));
      }
      if (two && !h->st3) {
        LSW_HIP_TRY(hipStreamCreateWithFlags(&h->st3, hipStreamNonBlocking));
        for (hipEvent_t* ev : {&h->evPA, &h->evR, &h->evM, &h->evR2})
          LSW_HIP_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming));
      }
      if (!h->cst) LSW_HIP_TRY(hipStreamCreateWithFlags(&h->cst, hipStreamNonBlocking));
      ls_status e = LS_OK;
      if (split) {
        LSW_HIP_TRY(hipEventRecord(h->evQ, h->st));
        LSW_HIP_TRY(hipStreamWaitEvent(h->st2, h->evQ, 0));
        {
          Timed tm(h, kKSlicesLast, nb, h->st2);
          if ((e = phaseA(kmain, nl, h->st2)) != LS_OK) return e;
        }
        LSW_HIP_TRY(hipEventRecord(h->evA, h->st2));
      }
      {
        Timed tm(h, kKSlices, nb);
        if ((e = phaseA(0, kmain, h->st)) != LS_OK) return e;
      }
      if (two) {
        Timed tm(h, kKIface, nb);
        const C<T>* IM = h->IM.as<C<T>>();
        const C<T>* IP = h->IP.as<C<T>>();
        const C<T>* IN = h->IN.as<C<T>>();
        const C<T>* Hm = h->Hm.as<C<T>>();
        const C<T>* Hp = h->Hp.as<C<T>>();
        const int m = nl - 1;
        auto V = [&](C<T>* base, int k) { return base + (size_t)k * vs; };
        // lambda_k -= M_k lambda_{k-1}, mu_k -= P_k lambda_{k-1}: step i of the
        // left front (slice i) on st, of the right front (slice p + i) on st3
        LSW_HIP_TRY(hipEventRecord(h->evPA, h->st));
        LSW_HIP_TRY(hipStreamWaitEvent(h->st3, h->evPA, 0));
        for (int i = 1; i <= p - 1; ++i)
          for (const int k : {i, p + i}) {
            IfaceProd<T> pr[2] = {{IM + (size_t)k * MS, V(lam, k), V(lam, k - 1), V(lam, k)},
                                  {IP + (size_t)k * MS, V(mu, k), V(lam, k - 1), V(mu, k)}};
            LSW_HIP_TRY(launch_iface_prods<T>(pr, 2, L, nb, imf, k == i ? h->st : h->st3));
          }
        LSW_HIP_TRY(hipEventRecord(h->evR, h->st3));
        LSW_HIP_TRY(hipStreamWaitEvent(h->st, h->evR, 0));
        LSW_HIP_TRY(hipEventRecord(h->evL, h->st));  // both lambda recurrences done
        LSW_HIP_TRY(hipStreamWaitEvent(h->st, h->evA, 0));
        // the middle slice m: its first (mu) and last (lambda) lines take the
        // lambda of both fronts' last slices, p - 1 and 2p - 1
        {
          IfaceProd<T> a[2] = {{IM + (size_t)m * MS, V(lam, m), V(lam, p - 1), V(lam, m)},
                               {IP + (size_t)m * MS, V(mu, m), V(lam, p - 1), V(mu, m)}};
          IfaceProd<T> c[2] = {{h->IQ.as<C<T>>(), V(lam, m), V(lam, 2 * p - 1), V(lam, m)},
                               {IN + (size_t)m * MS, V(mu, m), V(lam, 2 * p - 1), V(mu, m)}};
          LSW_HIP_TRY(launch_iface_prods<T>(a, 2, L, nb, imf, h->st));
          LSW_HIP_TRY(launch_iface_prods<T>(c, 2, L, nb, imf, h->st));
        }
        LSW_HIP_TRY(hipEventRecord(h->evM, h->st));
        LSW_HIP_TRY(hipStreamWaitEvent(h->st3, h->evM, 0));
        // mu_k -= N_k mu_next outward; next to the middle slice the left front
        // reads its mu (first line), the right front its lambda (last line)
        for (int i = p - 1; i >= 1; --i)
          for (const int k : {i, p + i}) {
            const C<T>* x = i < p - 1 ? V(mu, k + 1) : (k == i ? V(mu, m) : V(lam, m));
            IfaceProd<T> pr[1] = {{IN + (size_t)k * MS, V(mu, k), x, V(mu, k)}};
            LSW_HIP_TRY(launch_iface_prods<T>(pr, 1, L, nb, imf, k == i ? h->st : h->st3));
          }
        // each front's couplings on its own stream
        LSW_HIP_TRY(launch_couple<T>(h->slices(), L, h->b, Hm, Hp, lam, mu, nb, f, p, 2 * p, h->st3));
        LSW_HIP_TRY(hipEventRecord(h->evR2, h->st3));
        LSW_HIP_TRY(launch_couple<T>(h->slices(), L, h->b, Hm, Hp, lam, mu, nb, f, 0, p, h->st));
        LSW_HIP_TRY(hipStreamWaitEvent(h->st, h->evR2, 0));
      } else {
        hipGraphExec_t g0 = nullptr, g1 = nullptr;
        if (nl > 2 && (e = graph(0, g0)) != LS_OK) return e;  // part 0 is empty for two slices
        if ((e = graph(1, g1)) != LS_OK) return e;
        Timed tm(h, kKIface, nb);
        if (g0) LSW_HIP_TRY(hipGraphLaunch(g0, h->st));
        if (split) {
          LSW_HIP_TRY(hipEventRecord(h->evL, h->st));
          LSW_HIP_TRY(hipStreamWaitEvent(h->st, h->evA, 0));
        }
        LSW_HIP_TRY(hipGraphLaunch(g1, h->st));
      }
      if (split) {
        // the last slice in table order: its coupling (to its neighbours'
        // lambda, final after evL) and phase C on the second stream
        LSW_HIP_TRY(hipStreamWaitEvent(h->st2, h->evL, 0));
        {
          Timed tm(h, kKSlicesLast, nb, h->st2);
          LSW_HIP_TRY(launch_couple<T>(h->slices(), L, h->b, h->Hm.as<C<T>>(), h->Hp.as<C<T>>(), lam, mu, nb, f,
                                       kmain, nl, h->st2));
          if ((e = phaseC(kmain, nl, h->st2)) != LS_OK) return e;
        }
        LSW_HIP_TRY(hipEventRecord(h->evC, h->st2));
      }
      {
        Timed tm(h, kKSlices, nb);
        if ((e = phaseC(0, kmain, h->st)) != LS_OK) return e;
      }
      if (split) LSW_HIP_TRY(hipStreamWaitEvent(h->st, h->evC, 0));
    } else {
      Timed tm(h, kKSlices, nb);
      ls_status e = phaseC(0, nl, h->st);
      if (e != LS_OK) return e;
    }
  }
  return LS_OK;
}

// The slice factors again in the operand order of the matrix-core slice
// solves, with the per-slice offsets, chunk counts and scratch units.
template <typename T>
ls_status build_mfma_factors(ls_handle* h) {
  const int nl = h->nslices, L = h->L;
  const size_t cs = sizeof(C<T>);
  std::vector<size_t> mwo(nl), mgo(nl);
  std::vector<int> nsd(nl), ysu(nl);
  size_t w = 0, g = 0;
  int units = 0;
  for (int k = 0; k < nl; ++k) {
    const int t = h->t_host[k], tw = h->tw_host[k];
    mwo[k] = w;
    mgo[k] = g;
    w += (size_t)L * mfma_wrec_elems(t, tw);
    g += (size_t)L * mfma_grec_elems(t);
    nsd[k] = mfma_chunks(t, tw);
    ysu[k] = units;
    units += mfma_row_tiles(t);
  }
  LSW_ALLOC(h->MW, w * cs);
  LSW_ALLOC(h->MG, g * cs);
  LSW_ALLOC(h->mw_off, nl * sizeof(size_t));
  LSW_ALLOC(h->mg_off, nl * sizeof(size_t));
  LSW_ALLOC(h->mnsd, nl * sizeof(int));
  LSW_ALLOC(h->mys_unit, nl * sizeof(int));
  if (upload(h, h->mw_off, mwo) != LS_OK || upload(h, h->mg_off, mgo) != LS_OK || upload(h, h->mnsd, nsd) != LS_OK ||
      upload(h, h->mys_unit, ysu) != LS_OK)
    return LS_E_DEVICE;
  for (int k = 0; k < nl; ++k)
    LSW_HIP_TRY(launch_mfma_factors<T>(h->slices(), L, k, h->t_host[k], h->tw_host[k], h->FS.as<C<T>>(),
                                       h->FG.as<C<T>>(), h->MW.as<C<T>>() + mwo[k], h->MG.as<C<T>>() + mgo[k],
                                       h->st));
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  h->mys_units = units;
  return LS_OK;
}

// Interface maps M_k = E T_k J_F Hm_k, P_k = F T_k J_F Hm_k (k >= 1) and
// N_k = F T_k J_E Hp_k (1 <= k <= l-2): slice solves whose right-hand sides
// are the L columns of J_F Hm_k or J_E Hp_k, 32 columns per workgroup.
// Two fronts (table order: left front, right front, middle slice m = l-1):
// M_k and P_k for the slices with a predecessor in their front and for the
// middle slice (whose predecessor is the left front's last slice), N_k for
// the slices with a successor whose mu is needed (not the outermost ones), and
// for the middle slice, whose successor is the right front's last slice, also
// Q_m = E T_m J_E Hp_m: its last line from that neighbour.
template <typename T>
ls_status build_interface(ls_handle* h) {
  const int nl = h->nslices, L = h->L;
  if (nl < 2) return LS_OK;
  const bool two = h->H.fronts == 2;
  const int p = (nl - 1) / 2;  // two fronts: slices per front
  const size_t cs = sizeof(C<T>);
  const size_t LL = (size_t)L * L;
  LSW_ALLOC(h->IM, (size_t)nl * LL * cs);
  LSW_ALLOC(h->IP, (size_t)nl * LL * cs);
  LSW_ALLOC(h->IN, (size_t)nl * LL * cs);
  if (two) LSW_ALLOC(h->IQ, LL * cs);
  constexpr int W = 8;  // waves per workgroup of the vector-ALU path
  // columns per launch: whole 16-column tiles of the matrix-core path, as many
  // as an ~8 GB scratch allows; a short last launch of at most 8 columns takes
  // the vector-ALU path with its own small scratch
  const size_t tile_bytes = mfma_scratch_bytes(h, 16, cs);
  const int tiles = (int)std::max<size_t>(1, std::min<size_t>((L + 15) / 16, (size_t)8e9 / tile_bytes));
  const int cols = tiles * 16;
  DBuf mscr, vscr;
  LSW_ALLOC(mscr, tile_bytes * tiles);
  LSW_ALLOC(vscr, (size_t)nl * slice_scratch_elems<double>(L, W) * cs);
  SliceSolveArgs<T> a = slice_args<T>(h);
  a.yscr = vscr.as<C<T>>();
  a.mfma_scr = mscr.as<T>();
  a.dst_kind = kDstLines;
  a.sk = LL;
  a.sr = 1;
  a.sj = L;
  for (int col0 = 0; col0 < L; col0 += cols) {
    a.col0 = col0;
    a.nrhs = std::min(cols, L - col0);
    a.src_kind = kSrcUnitF;
    a.dstE = h->IM.as<C<T>>();
    a.dstF = h->IP.as<C<T>>();
    const int kern = a.nrhs > kMfmaMinCols ? 16 : W;
    ls_status e = two ? solve_slices<T>(h, a, 1, p, kern) : solve_slices<T>(h, a, 1, nl, kern);
    if (e == LS_OK && two) e = solve_slices<T>(h, a, p + 1, nl, kern);
    if (e != LS_OK) return e;
    if (two || nl > 2) {
      a.src_kind = kSrcUnitE;
      a.dstE = nullptr;
      a.dstF = h->IN.as<C<T>>();
      e = two ? solve_slices<T>(h, a, 1, p, kern) : solve_slices<T>(h, a, 1, nl - 1, kern);
      if (e == LS_OK && two) e = solve_slices<T>(h, a, p + 1, 2 * p, kern);
      if (e == LS_OK && two) {
        // the middle slice: N_m into its slot of IN, Q_m into IQ
        SliceSolveArgs<T> am = a;
        am.sk = 0;
        am.dstF = h->IN.as<C<T>>() + (size_t)(nl - 1) * LL;
        am.dstE = h->IQ.as<C<T>>();
        e = solve_slices<T>(h, am, nl - 1, nl, kern);
      }
      if (e != LS_OK) return e;
    }
  }
  // re-lay every map set in the operand order of the interface products
  for (DBuf* Mp : {&h->IM, &h->IP, &h->IN, &h->IQ}) {
    if (!Mp->p) continue;
    const int count = Mp == &h->IQ ? 1 : nl;
    DBuf z;
    LSW_ALLOC(z, (size_t)count * iface_map_stride<T>(L) * cs);
    LSW_HIP_TRY(launch_swizzle_maps<T>(Mp->as<C<T>>(), z.as<C<T>>(), L, count, h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    Mp->swap(z);  // the row-major maps are released with z
  }
  return LS_OK;
}

// ---- flexible GMRES, float64 outer loop (Sec. 2.5, reading G11) -----------
struct RhsState {
  int j = 0;          // Arnoldi steps in the current cycle
  int iters = 0;      // over all cycles
  int done = 0;       // 1 converged, 2 gave up
  double beta0 = 0;   // ||g||
  double relres = 0;
  std::vector<std::complex<double>> Hm;  // (restart+1) x restart, column-major
  std::vector<double> cs;
  std::vector<std::complex<double>> sn, s;
  // norms of the basis vectors of the cycle as stored (u_0 = r / ||r|| has
  // norm 1; u_{k+1} = w - sum_i c_i u_i is kept unnormalised)
  std::vector<double> bn;
};

void givens(std::complex<double> f, std::complex<double> g, double& c, std::complex<double>& s,
            std::complex<double>& r) {
  if (g == 0.0) {
    c = 1.0;
    s = 0.0;
    r = f;
    return;
  }
  if (f == 0.0) {
    c = 0.0;
    s = std::conj(g) / std::abs(g);
    r = std::abs(g);
    return;
  }
  const double af = std::abs(f), ag = std::abs(g);
  const double rho = std::hypot(af, ag);
  c = af / rho;
  s = (f / af) * std::conj(g) / rho;
  r = (f / af) * rho;
}

template <typename T>
ls_status gmres(ls_handle* h, int nrhs, double tol, std::vector<ls_rhs_info>& info) {
  // G holds g, X receives the solution.
  const size_t N = h->N;
  const int rs = h->opt.restart;
  hipStream_t st = h->st;
  double2* Vb = h->V.as<double2>();
  C<T>* Zb = h->Z.as<C<T>>();
  double2* Wb = h->W.as<double2>();
  double2* Xb = h->X.as<double2>();
  double2* Gb = h->G.as<double2>();
  double2* Rb = h->R.as<double2>();
  double2* coefs = h->coefs.as<double2>();
  auto Vp = [&](int r, int k) { return Vb + ((size_t)r * (rs + 1) + k) * N; };
  auto Zp = [&](int r, int k) { return Zb + ((size_t)r * rs + k) * N; };

  std::vector<RhsState> S(nrhs);
  for (auto& s : S) {
    s.Hm.assign((size_t)(rs + 1) * rs, 0.0);
    s.cs.assign(rs, 0.0);
    s.sn.assign(rs, 0.0);
    s.s.assign(rs + 1, 0.0);
    s.bn.assign(rs + 1, 1.0);
  }
  LSW_HIP_TRY(hipMemsetAsync(Xb, 0, (size_t)nrhs * N * sizeof(double2), st));

  std::vector<DotPair> hp;
  std::vector<DotGroup> hg;
  std::vector<AxpyOut> ho;
  std::vector<AxpyTerm<double>> ht64;
  std::vector<AxpyTerm<T>> htT;
  std::vector<double2> hc;
  std::vector<void*> pa, pb;
  const double2 one = make_double2(1.0, 0.0);

  // norms of a set of vectors -> host
  auto norms = [&](const std::vector<const double2*>& vecs, std::vector<double>& out) -> ls_status {
    hp.clear();
    for (auto v : vecs) hp.push_back({v, v});
    if (upload(h, h->pairs, hp) != LS_OK) return LS_E_DEVICE;
    LSW_HIP_TRY(launch_dots(h->pairs.as<DotPair>(), (int)hp.size(), N, h->partials.as<double2>(), coefs, st));
    hc.resize(hp.size());
    LSW_HIP_TRY(hipMemcpyAsync(hc.data(), coefs, hc.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    LSW_HIP_TRY(hipStreamSynchronize(st));
    out.resize(vecs.size());
    for (size_t i = 0; i < vecs.size(); ++i) out[i] = std::sqrt(std::max(hc[i].x, 0.0));
    return LS_OK;
  };
  // y_i = src_i / nrm_i (host scalars) for a set of (y, src)
  auto scaled_copies = [&](const std::vector<std::pair<double2*, const double2*>>& ys,
                           const std::vector<double>& scal) -> ls_status {
    ho.clear();
    ht64.clear();
    hc.assign(ys.size() + 1, one);
    for (size_t i = 0; i < ys.size(); ++i) {
      hc[i + 1] = make_double2(1.0 / scal[i], 0.0);
      ht64.push_back({ys[i].second, (int)i + 1, 0});
      ho.push_back({ys[i].first, (int)i, (int)i + 1, 1, -1, 0});
    }
    if (upload(h, h->coefs, hc) != LS_OK || upload(h, h->outs, ho) != LS_OK || upload(h, h->terms64, ht64) != LS_OK)
      return LS_E_DEVICE;
    LSW_HIP_TRY(launch_axpys<double>(h->outs.as<AxpyOut>(), (int)ho.size(), h->terms64.as<AxpyTerm<double>>(),
                                     coefs, N, st));
    return LS_OK;
  };

  // initial residual r = g (x0 = 0)
  {
    std::vector<const double2*> v;
    for (int r = 0; r < nrhs; ++r) v.push_back(Gb + (size_t)r * N);
    std::vector<double> nr;
    ls_status e = norms(v, nr);
    if (e != LS_OK) return e;
    std::vector<std::pair<double2*, const double2*>> ys;
    std::vector<double> sc;
    for (int r = 0; r < nrhs; ++r) {
      S[r].beta0 = nr[r];
      if (!std::isfinite(nr[r])) {
        set_error("right-hand side has a non-finite norm");
        return LS_E_NUMERIC;
      }
      if (nr[r] == 0.0) {
        S[r].done = 1;
        continue;
      }
      S[r].s[0] = nr[r];
      ys.push_back({Vp(r, 0), Gb + (size_t)r * N});
      sc.push_back(nr[r]);
    }
    if (!ys.empty() && (e = scaled_copies(ys, sc)) != LS_OK) return e;
  }

  const int max_iters = h->opt.max_iters;
  while (true) {
    std::vector<int> act;
    for (int r = 0; r < nrhs; ++r)
      if (!S[r].done) act.push_back(r);
    if (act.empty()) break;
    const int na = (int)act.size();
    C<T>* vin = h->vin.as<C<T>>();
    C<T>* zout = h->zout.as<C<T>>();
    C<T>* aout = h->aout.as<C<T>>();
    // Every descriptor of this step up to the readback goes through one
    // asynchronous copy of the main stage; the host does not wait for the
    // device until the readback.
    Stage& sm = h->stage_main;
    sm.reset();
    pa.clear();
    pb.clear();
    for (int p = 0; p < na; ++p) {
      pa.push_back(vin + (size_t)p * N);
      pb.push_back(Vp(act[p], S[act[p]].j));
    }
    C<T>** cin_d = reinterpret_cast<C<T>**>(sm.put(pa));
    const double2* const* cin_s = reinterpret_cast<const double2* const*>(sm.put(pb));
    pa.clear();
    pb.clear();
    for (int p = 0; p < na; ++p) {
      pa.push_back(Zp(act[p], S[act[p]].j));
      pb.push_back(zout + (size_t)p * N);
    }
    C<T>** cz_d = reinterpret_cast<C<T>**>(sm.put(pa));
    const C<T>* const* cz_s = reinterpret_cast<const C<T>* const*>(sm.put(pb));
    pa.clear();
    pb.clear();
    for (int p = 0; p < na; ++p) {
      pa.push_back(Wb + (size_t)act[p] * N);
      pb.push_back(aout + (size_t)p * N);
    }
    double2** cw_d = reinterpret_cast<double2**>(sm.put(pa));
    const C<T>* const* cw_s = reinterpret_cast<const C<T>* const*>(sm.put(pb));
    // classical Gram-Schmidt, one pass, with the exact norm of its result.
    // The basis vectors of a cycle are orthogonal but not normalised: u_0 =
    // r / ||r||, then u_{j+1} = w - sum_k (u_k^H w / b_k^2) u_k with
    // b_k = ||u_k||, written straight into its slot with b_{j+1}^2 summed by the
    // same pass (no normalisation pass). With q_k = u_k / b_k and
    // z_j = P u_j, A z_j = sum_k (u_k^H w / b_k) q_k + b_{j+1} q_{j+1}: that is the
    // Hessenberg column, and x = Z y as with a normalised basis. The norm is
    // summed exactly: ||w||^2 - |c|^2 would cancel, w lying close to span(V).
    hp.clear();
    std::vector<int> off(na + 1, 0);
    std::vector<double> kscale;
    for (int p = 0; p < na; ++p) {
      const int r = act[p];
      for (int k = 0; k <= S[r].j; ++k) {
        hp.push_back({Vp(r, k), Wb + (size_t)r * N});
        kscale.push_back(1.0 / (S[r].bn[k] * S[r].bn[k]));
      }
      off[p + 1] = (int)hp.size();
    }
    // coefficients: the products u_k^H w (base1), the update's u_k^H w / b_k^2
    // (base2), then b_{j+1}^2 per right-hand side (base3)
    const int np = (int)hp.size();
    const int base1 = 1, base2 = 1 + np, base3 = 1 + 2 * np;
    ho.clear();
    ht64.clear();
    for (int p = 0; p < na; ++p) {
      const int r = act[p];
      AxpyOut o{Vp(r, S[r].j + 1), (int)ht64.size(), 0, 1, -1, 0};
      ht64.push_back({Wb + (size_t)r * N, 0, 0});  // the unit term w (coefs[0] = 1)
      for (int k = 0; k <= S[r].j; ++k) ht64.push_back({Vp(r, k), base2 + off[p] + k, 1});
      o.tend = (int)ht64.size();
      ho.push_back(o);
    }
    // the dot products of a right-hand side share its w: groups of up to
    // kDotGroup basis vectors read it once
    hg.clear();
    for (int p = 0; p < na; ++p)
      for (int i = off[p]; i < off[p + 1]; i += kDotGroup) {
        DotGroup g{};
        g.y = Wb + (size_t)act[p] * N;
        g.count = std::min(kDotGroup, off[p + 1] - i);
        g.pbase = i;
        for (int k = 0; k < g.count; ++k) g.x[k] = hp[i + k].x;
        hg.push_back(g);
      }
    const AxpyOut* outs_d = sm.put(ho);
    const AxpyTerm<double>* terms_d = sm.put(ht64);
    const DotGroup* groups_d = sm.put(hg);
    const double2* one_d = sm.put(&one, 1);
    const double* kscale_d = sm.put(kscale);
    if (!cin_d || !cin_s || !cz_d || !cz_s || !cw_d || !cw_s || !outs_d || !terms_d || !groups_d || !one_d ||
        !kscale_d) {
      set_error("internal: descriptor stage too small");
      return LS_E_STATE;
    }
    LSW_HIP_TRY(sm.flush(st));
    // coefs[0] = 1 (the unit coefficient of the normalisation below)
    LSW_HIP_TRY(hipMemcpyAsync(coefs, one_d, sizeof(double2), hipMemcpyDeviceToDevice, st));
    // z = P v_j (precision T), kept in Z. In 2D with the interface schedule
    // the Q stencil reads v_j in float64 itself and the extraction writes z
    // into its slot of Z, which the operator then reads
    const bool q64 = h->dim == 2 && !h->hmode && h->opt.sweep_schedule != LS_SWEEP_SEQUENTIAL;
    if (!q64) LSW_HIP_TRY((launch_copy_cast<T, double>(cin_d, cin_s, na, N, st)));
    ls_status e = h->hmode ? apply_sweep_ext<T>(h, vin, na, zout)
                           : apply_P<T>(h, vin, na, zout, q64 ? cin_s : nullptr, q64 ? cz_d : nullptr);
    if (e != LS_OK) return e;
    if (!q64) LSW_HIP_TRY((launch_copy_cast<T, T>(cz_d, cz_s, na, N, st)));
    // w = A z (precision T) -> float64 work vector W[r]; in 2D the
    // convolution's epilogue writes W[r] itself
    if (h->hmode) {
      LSW_HIP_TRY(launch_apply_H<T>(h->stencils(), zout, na, aout, st));
      LSW_HIP_TRY((launch_copy_cast<double, T>(cw_d, cw_s, na, N, st)));
    } else if (h->dim == 2) {
      if ((e = apply_A<T>(h, zout, na, aout, cw_d, q64 ? cz_d : nullptr)) != LS_OK) return e;
    } else {
      if ((e = apply_A<T>(h, zout, na, aout)) != LS_OK) return e;
      LSW_HIP_TRY((launch_copy_cast<double, T>(cw_d, cw_s, na, N, st)));
    }
    double2* part = h->partials.as<double2>();
    LSW_HIP_TRY(launch_mdots(groups_d, (int)hg.size(), np, N, part, coefs + base1, st));
    LSW_HIP_TRY(launch_scale_coefs(coefs + base1, kscale_d, coefs + base2, np, st));
    LSW_HIP_TRY(launch_axpys_norms(outs_d, na, terms_d, coefs, N, part, coefs + base3, st));
    hc.resize(base3 + na);
    LSW_HIP_TRY(hipMemcpyAsync(hc.data(), coefs, hc.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    LSW_HIP_TRY(hipStreamSynchronize(st));
    std::vector<int> ending;
    for (int p = 0; p < na; ++p) {
      const int r = act[p];
      RhsState& s = S[r];
      const int j = s.j;
      std::complex<double>* col = &s.Hm[(size_t)j * (rs + 1)];
      for (int k = 0; k <= j; ++k) {
        const double2 a = hc[base1 + off[p] + k];
        col[k] = std::complex<double>(a.x, a.y) / s.bn[k];
      }
      const double w2 = hc[base3 + p].x;
      const double hn = std::sqrt(std::max(w2, 0.0));
      if (!std::isfinite(hn)) {
        set_error("non-finite norm in the Arnoldi process");
        return LS_E_NUMERIC;
      }
      col[j + 1] = hn;
      s.bn[j + 1] = hn;
      for (int k = 0; k < j; ++k) {
        const std::complex<double> a = col[k], c = col[k + 1];
        col[k] = s.cs[k] * a + s.sn[k] * c;
        col[k + 1] = -std::conj(s.sn[k]) * a + s.cs[k] * c;
      }
      double c;
      std::complex<double> sg, rr;
      givens(col[j], col[j + 1], c, sg, rr);
      s.cs[j] = c;
      s.sn[j] = sg;
      col[j] = rr;
      col[j + 1] = 0.0;
      s.s[j + 1] = -std::conj(sg) * s.s[j];
      s.s[j] = c * s.s[j];
      s.iters += 1;
      s.j += 1;
      const bool conv = std::abs(s.s[j + 1]) <= tol * s.beta0;
      // v_{j+1} is already in V; a right-hand side that ends its cycle here
      // (or breaks down: h = 0) does not read it
      if (conv || s.j == rs || s.iters >= max_iters || hn == 0.0) ending.push_back(r);
    }
    if (ending.empty()) continue;
    // cycle end: x += Z y, true residual in float64
    ho.clear();
    htT.clear();
    hc.assign(1, one);
    for (int r : ending) {
      RhsState& s = S[r];
      const int j = s.j;
      std::vector<std::complex<double>> y(j);
      for (int i = j - 1; i >= 0; --i) {
        std::complex<double> acc = s.s[i];
        for (int k = i + 1; k < j; ++k) acc -= s.Hm[(size_t)k * (rs + 1) + i] * y[k];
        y[i] = acc / s.Hm[(size_t)i * (rs + 1) + i];
      }
      AxpyOut o{Xb + (size_t)r * N, (int)htT.size(), 0, 0, -1, 0};
      for (int i = 0; i < j; ++i) {
        hc.push_back(make_double2(y[i].real(), y[i].imag()));
        htT.push_back({Zp(r, i), (int)hc.size() - 1, 0});
      }
      o.tend = (int)htT.size();
      ho.push_back(o);
    }
    if (upload(h, h->coefs, hc) != LS_OK || upload(h, h->outs, ho) != LS_OK) return LS_E_DEVICE;
    DBuf& tb = std::is_same<T, double>::value ? h->terms64 : h->terms32;
    if (upload(h, tb, htT) != LS_OK) return LS_E_DEVICE;
    LSW_HIP_TRY(launch_axpys<T>(h->outs.as<AxpyOut>(), (int)ho.size(), tb.as<AxpyTerm<T>>(), coefs, N, st));
    // A x of the ending set in float64 (2D: read from X in place; 3D: packed
    // into T1 first), r = g - A x
    const int ne = (int)ending.size();
    double2* T1 = h->T1.as<double2>();
    double2* T2 = h->T2.as<double2>();
    pa.clear();
    pb.clear();
    for (int p = 0; p < ne; ++p) {
      pa.push_back(T1 + (size_t)p * N);
      pb.push_back(Xb + (size_t)ending[p] * N);
    }
    if (upload(h, h->ptrs_a, pa) != LS_OK || upload(h, h->ptrs_b, pb) != LS_OK) return LS_E_DEVICE;
    if (h->dim == 2 && !h->hmode) {
      // the operator reads each x from its slot of X
      if ((e = apply_A<double>(h, T1, ne, T2, nullptr, h->ptrs_b.as<const double2*>())) != LS_OK) return e;
    } else {
      LSW_HIP_TRY(
          (launch_copy_cast<double, double>(h->ptrs_a.as<double2*>(), h->ptrs_b.as<const double2*>(), ne, N, st)));
      if (h->hmode)
        LSW_HIP_TRY(launch_apply_H<double>(h->stencils(), T1, ne, T2, st));
      else if ((e = apply_A<double>(h, T1, ne, T2)) != LS_OK)
        return e;
    }
    ho.clear();
    ht64.clear();
    for (int p = 0; p < ne; ++p) {
      const int r = ending[p];
      ht64.push_back({Gb + (size_t)r * N, 0, 0});
      ht64.push_back({T2 + (size_t)p * N, 0, 1});
      ho.push_back({Rb + (size_t)r * N, 2 * p, 2 * p + 2, 1, -1, 0});
    }
    hc.assign(1, one);
    if (upload(h, h->coefs, hc) != LS_OK || upload(h, h->outs, ho) != LS_OK || upload(h, h->terms64, ht64) != LS_OK)
      return LS_E_DEVICE;
    LSW_HIP_TRY(launch_axpys<double>(h->outs.as<AxpyOut>(), ne, h->terms64.as<AxpyTerm<double>>(), coefs, N, st));
    std::vector<const double2*> rv;
    for (int r : ending) rv.push_back(Rb + (size_t)r * N);
    std::vector<double> rn;
    if ((e = norms(rv, rn)) != LS_OK) return e;
    std::vector<std::pair<double2*, const double2*>> ys;
    std::vector<double> sc;
    for (int p = 0; p < ne; ++p) {
      const int r = ending[p];
      RhsState& s = S[r];
      if (!std::isfinite(rn[p])) {
        set_error("non-finite true residual");
        return LS_E_NUMERIC;
      }
      s.relres = rn[p] / s.beta0;
      if (s.relres <= tol) {
        s.done = 1;
      } else if (s.iters >= max_iters) {
        s.done = 2;
      } else if (rn[p] == 0.0) {
        s.done = 1;
      } else {
        // restart from the true residual
        s.j = 0;
        std::fill(s.s.begin(), s.s.end(), 0.0);
        s.s[0] = rn[p];
        s.bn.assign(s.bn.size(), 1.0);
        ys.push_back({Vp(r, 0), Rb + (size_t)r * N});
        sc.push_back(rn[p]);
      }
    }
    if (!ys.empty() && (e = scaled_copies(ys, sc)) != LS_OK) return e;
    LSW_HIP_TRY(hipStreamSynchronize(st));
  }
  info.resize(nrhs);
  bool all = true;
  for (int r = 0; r < nrhs; ++r) {
    info[r].iterations = S[r].iters;
    info[r].rel_residual = S[r].beta0 == 0.0 ? 0.0 : S[r].relres;
    info[r].converged = S[r].done == 1;
    all = all && S[r].done == 1;
  }
  if (!all) {
    set_error("GMRES reached max_iters before the tolerance for some right-hand side");
    return LS_E_NOCONV;
  }
  return LS_OK;
}

// ---- block flexible GMRES (ls_options.block_size > 1) -------------------------
// The batch of Sec. 2.5 with one shared block Krylov space per block of
// right-hand sides (consecutive columns): per step Z_j = P V_j and W = A Z_j
// for every column (the batched applies of the per-column loop), then two
// passes of classical block Gram-Schmidt against V_0..V_j and the block QR
// W = V_{j+1} R by Cholesky QR done twice. The Gram products are GEMMs of
// (N x (j+1)B)^H (N x B) on the matrix cores (library zgemm); the small
// Cholesky factorizations, the Householder QR of the block Hessenberg matrix
// and the least-squares solves run on the host in float64. A column leaves
// its block at a restart once its true residual meets the tolerance; a zero
// right-hand side never enters it.

#define LSW_BLAS_TRY(expr)                                                      \
  do {                                                                          \
    rocblas_status _b = (expr);                                                 \
    if (_b != rocblas_status_success) {                                         \
      set_error(std::string(#expr) + ": " + rocblas_status_to_string(_b));      \
      return LS_E_DEVICE;                                                       \
    }                                                                           \
  } while (0)

using cplx = std::complex<double>;

// G = R^H R for a Hermitian b x b matrix (column-major), R upper triangular.
// A pivot at or below rel * G_kk (column k lies in the span of the earlier
// columns to that relative accuracy, or is zero) leaves row k of R zero and
// makes the result false.
bool cholesky_upper(const cplx* G, int b, cplx* R, double rel) {
  bool ok = true;
  std::fill(R, R + (size_t)b * b, cplx(0.0));
  for (int k = 0; k < b; ++k) {
    const double gkk = G[(size_t)k * b + k].real();
    double d = gkk;
    for (int i = 0; i < k; ++i) d -= std::norm(R[(size_t)k * b + i]);
    if (!(gkk > 0.0) || !(d > rel * gkk)) {
      ok = false;
      continue;
    }
    const double rkk = std::sqrt(d);
    R[(size_t)k * b + k] = rkk;
    for (int c = k + 1; c < b; ++c) {
      cplx acc = G[(size_t)c * b + k];
      for (int i = 0; i < k; ++i) acc -= std::conj(R[(size_t)k * b + i]) * R[(size_t)c * b + i];
      R[(size_t)c * b + k] = acc / rkk;
    }
  }
  return ok;
}

// Ri = R^{-1} for a nonsingular upper triangular b x b R (column-major).
void upper_inverse(const cplx* R, int b, cplx* Ri) {
  std::fill(Ri, Ri + (size_t)b * b, cplx(0.0));
  for (int c = 0; c < b; ++c) {
    Ri[(size_t)c * b + c] = 1.0 / R[(size_t)c * b + c];
    for (int i = c - 1; i >= 0; --i) {
      cplx acc = 0.0;
      for (int k = i + 1; k <= c; ++k) acc += R[(size_t)k * b + i] * Ri[(size_t)c * b + k];
      Ri[(size_t)c * b + i] = -acc / R[(size_t)i * b + i];
    }
  }
}

// Host state of one block of right-hand sides.
struct BlockState {
  int first = 0;           // first global column of the block
  std::vector<int> cols;   // global columns in the block this cycle
  int j = 0;               // block steps in the cycle
  int iters = 0;           // block steps over all cycles
  bool in_cycle = false;
  bool end = false;        // the cycle ends after this step
  int p0 = 0;              // first position of the block's columns in the step's batch
  // Householder QR of the block Hessenberg matrix ((rs+1)b x rs b,
  // column-major, reflectors below the diagonal) and Q^H E ((rs+1)b x b)
  std::vector<cplx> Hb, E, tau;
  // host copies of the small matrices; the uploaded ones stay untouched
  // until the next synchronisation
  std::vector<cplx> C1, C2, G, R, R1, R2, R1i, R2i, Y;
  bool qr_ok = true;
  int b() const { return (int)cols.size(); }
};

template <typename T>
ls_status block_gmres(ls_handle* h, int nrhs, double tol, std::vector<ls_rhs_info>& info) {
  const size_t N = h->N;
  const int rs = h->opt.restart;
  const int Bsz = std::min(h->opt.block_size, nrhs);
  const int nblk = (nrhs + Bsz - 1) / Bsz;
  const int max_iters = h->opt.max_iters;
  hipStream_t st = h->st;
  if (!h->blas) {
    LSW_BLAS_TRY(rocblas_create_handle(&h->blas));
    LSW_BLAS_TRY(rocblas_set_atomics_mode(h->blas, rocblas_atomics_not_allowed));
    LSW_BLAS_TRY(rocblas_set_pointer_mode(h->blas, rocblas_pointer_mode_host));
  }
  LSW_BLAS_TRY(rocblas_set_stream(h->blas, st));
  rocblas_handle bl = h->blas;
  const size_t rsz = (size_t)(2 * rs + 3) * Bsz * Bsz;  // complex entries per block
  LSW_ALLOC(h->bcoef, (size_t)nblk * rsz * sizeof(double2));
  // Gram products C = A^H B with A (N x m), B (N x nc): split over N into
  // nch chunks of Lc rows (one strided-batched GEMM; the last N - nch Lc rows
  // in one more), then the chunk results summed in a fixed order
  const int nch = (int)std::max<size_t>(1, std::min<size_t>(256, N / 8192));
  const int Lc = (int)(N / nch), tail = (int)(N - (size_t)nch * Lc);
  LSW_ALLOC(h->gpart, (size_t)(nch + 1) * rs * Bsz * Bsz * sizeof(double2));
  double2* Vb = h->V.as<double2>();
  double2* Zb = h->Z.as<double2>();
  double2* Wb = h->W.as<double2>();
  double2* Xb = h->X.as<double2>();
  double2* Gb = h->G.as<double2>();
  double2* Rb = h->R.as<double2>();
  double2* T1 = h->T1.as<double2>();
  double2* T2 = h->T2.as<double2>();
  double2* bc = h->bcoef.as<double2>();
  auto Vp = [&](const BlockState& B, int k) { return Vb + (size_t)B.first * (rs + 1) * N + (size_t)k * B.b() * N; };
  auto Zp = [&](const BlockState& B, int k) { return Zb + (size_t)B.first * rs * N + (size_t)k * B.b() * N; };
  auto region = [&](int blk) { return bc + (size_t)blk * rsz; };
  auto C1d = [&](int blk) { return region(blk); };
  auto C2d = [&](int blk) { return region(blk) + (size_t)rs * Bsz * Bsz; };
  auto Gd = [&](int blk) { return region(blk) + (size_t)2 * rs * Bsz * Bsz; };
  auto R1id = [&](int blk) { return Gd(blk) + (size_t)Bsz * Bsz; };
  auto R2id = [&](int blk) { return Gd(blk) + (size_t)2 * Bsz * Bsz; };
  const cplx one(1.0, 0.0), zero(0.0, 0.0), mone(-1.0, 0.0);
  auto zc = [](const double2* p) { return reinterpret_cast<const rocblas_double_complex*>(p); };
  auto zm = [](double2* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
  auto zs = [](const cplx& c) { return reinterpret_cast<const rocblas_double_complex*>(&c); };
  const rocblas_operation OC = rocblas_operation_conjugate_transpose, ON = rocblas_operation_none;
  const int iN = (int)N;
  double2* gp = h->gpart.as<double2>();
  auto gram = [&](int m, int nc, const double2* A, const double2* Bm, double2* Cout) -> ls_status {
    const rocblas_stride sc = (rocblas_stride)m * nc;
    LSW_BLAS_TRY(rocblas_zgemm_strided_batched(bl, OC, ON, m, nc, Lc, zs(one), zc(A), iN, (rocblas_stride)Lc,
                                               zc(Bm), iN, (rocblas_stride)Lc, zs(zero), zm(gp), m, sc, nch));
    if (tail > 0)
      LSW_BLAS_TRY(rocblas_zgemm(bl, OC, ON, m, nc, tail, zs(one), zc(A + (size_t)nch * Lc), iN,
                                 zc(Bm + (size_t)nch * Lc), iN, zs(zero), zm(gp + (size_t)nch * sc), m));
    LSW_HIP_TRY(launch_sum_parts(gp, nch + (tail > 0 ? 1 : 0), (size_t)sc, Cout, st));
    return LS_OK;
  };

  // column norms of ncols contiguous columns (fixed-order reductions)
  std::vector<double> parts;
  auto colnorms = [&](const double2* x, int ncols, std::vector<double>& out) -> ls_status {
    double* pd = h->partials.as<double>();
    LSW_HIP_TRY(launch_colnorm2(x, ncols, N, pd, st));
    parts.resize((size_t)ncols * kDotBlocks);
    LSW_HIP_TRY(hipMemcpyAsync(parts.data(), pd, parts.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LSW_HIP_TRY(hipStreamSynchronize(st));
    out.assign(ncols, 0.0);
    for (int c = 0; c < ncols; ++c) {
      double acc = 0.0;
      for (int k = 0; k < kDotBlocks; ++k) acc += parts[(size_t)c * kDotBlocks + k];
      out[c] = std::sqrt(std::max(acc, 0.0));
    }
    return LS_OK;
  };
  // dst_i = src_i for pointer pairs (float64 copies through the pointer tables)
  std::vector<void*> pa, pb;
  auto gather = [&](const std::vector<double2*>& dst, const std::vector<const double2*>& src) -> ls_status {
    if (dst.empty()) return LS_OK;
    pa.assign(dst.begin(), dst.end());
    pb.clear();
    for (auto p : src) pb.push_back(const_cast<double2*>(p));
    if (upload(h, h->ptrs_a, pa) != LS_OK || upload(h, h->ptrs_b, pb) != LS_OK) return LS_E_DEVICE;
    LSW_HIP_TRY((launch_copy_cast<double, double>(h->ptrs_a.as<double2*>(), h->ptrs_b.as<const double2*>(),
                                                  (int)dst.size(), N, st)));
    return LS_OK;
  };

  // Cholesky QR, twice, of the b columns at in[blk] (contiguous) into
  // out[blk], through tmp[blk]; R into B.R. B.qr_ok false: numerically rank
  // deficient (R from the first pass, out not written).
  std::vector<BlockState> S(nblk);
  auto block_qr = [&](const std::vector<int>& bls, const std::vector<double2*>& in, const std::vector<double2*>& tmp,
                      const std::vector<double2*>& out) -> ls_status {
    Timed tm(h, kKGram, 0);
    ls_status e = LS_OK;
    for (size_t q = 0; q < bls.size(); ++q) {
      BlockState& B = S[bls[q]];
      const int b = B.b();
      if ((e = gram(b, b, in[q], in[q], Gd(bls[q]))) != LS_OK) return e;
      B.G.resize((size_t)b * b);
      LSW_HIP_TRY(hipMemcpyAsync(B.G.data(), Gd(bls[q]), B.G.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    }
    LSW_HIP_TRY(hipStreamSynchronize(st));
    for (size_t q = 0; q < bls.size(); ++q) {
      BlockState& B = S[bls[q]];
      const int b = B.b();
      for (const cplx& g : B.G)
        if (!std::isfinite(g.real()) || !std::isfinite(g.imag())) {
          set_error("non-finite value in the block Arnoldi process");
          return LS_E_NUMERIC;
        }
      B.R1.resize((size_t)b * b);
      B.qr_ok = cholesky_upper(B.G.data(), b, B.R1.data(), 1e-14);
      if (!B.qr_ok) {
        B.R = B.R1;
        continue;
      }
      B.R1i.resize((size_t)b * b);
      upper_inverse(B.R1.data(), b, B.R1i.data());
      LSW_HIP_TRY(hipMemcpyAsync(R1id(bls[q]), B.R1i.data(), B.R1i.size() * sizeof(double2), hipMemcpyHostToDevice, st));
      LSW_BLAS_TRY(rocblas_zgemm(bl, ON, ON, iN, b, b, zs(one), zc(in[q]), iN, zc(R1id(bls[q])), b, zs(zero),
                                 zm(tmp[q]), iN));
      if ((e = gram(b, b, tmp[q], tmp[q], Gd(bls[q]))) != LS_OK) return e;
      LSW_HIP_TRY(hipMemcpyAsync(B.G.data(), Gd(bls[q]), B.G.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    }
    LSW_HIP_TRY(hipStreamSynchronize(st));
    for (size_t q = 0; q < bls.size(); ++q) {
      BlockState& B = S[bls[q]];
      if (!B.qr_ok) continue;
      const int b = B.b();
      B.R2.resize((size_t)b * b);
      if (!cholesky_upper(B.G.data(), b, B.R2.data(), 1e-14)) {
        B.qr_ok = false;
        B.R = B.R1;
        continue;
      }
      B.R2i.resize((size_t)b * b);
      upper_inverse(B.R2.data(), b, B.R2i.data());
      LSW_HIP_TRY(hipMemcpyAsync(R2id(bls[q]), B.R2i.data(), B.R2i.size() * sizeof(double2), hipMemcpyHostToDevice, st));
      LSW_BLAS_TRY(rocblas_zgemm(bl, ON, ON, iN, b, b, zs(one), zc(tmp[q]), iN, zc(R2id(bls[q])), b, zs(zero),
                                 zm(out[q]), iN));
      // R = R2 R1
      B.R.assign((size_t)b * b, 0.0);
      for (int c = 0; c < b; ++c)
        for (int i = 0; i <= c; ++i) {
          cplx acc = 0.0;
          for (int k = i; k <= c; ++k) acc += B.R2[(size_t)k * b + i] * B.R1[(size_t)c * b + k];
          B.R[(size_t)c * b + i] = acc;
        }
    }
    return LS_OK;
  };
  // a new cycle of block B: E = [S; 0] with the initial block's R = S
  auto start_cycle = [&](BlockState& B) {
    const int b = B.b();
    const size_t ldh = (size_t)(rs + 1) * b;
    B.j = 0;
    B.in_cycle = true;
    B.Hb.assign(ldh * rs * b, 0.0);
    B.tau.assign((size_t)rs * b, 0.0);
    B.E.assign(ldh * b, 0.0);
    for (int c = 0; c < b; ++c)
      for (int i = 0; i < b; ++i) B.E[(size_t)c * ldh + i] = B.R[(size_t)c * b + i];
  };

  std::vector<int> col_its(nrhs, 0), cdone(nrhs, 0);
  std::vector<double> gn, relres(nrhs, 0.0);
  LSW_HIP_TRY(hipMemsetAsync(Xb, 0, (size_t)nrhs * N * sizeof(double2), st));
  ls_status e = colnorms(Gb, nrhs, gn);
  if (e != LS_OK) return e;
  for (int c = 0; c < nrhs; ++c)
    if (!std::isfinite(gn[c])) {
      set_error("right-hand side has a non-finite norm");
      return LS_E_NUMERIC;
    }
  // initial blocks: the nonzero columns of G
  {
    std::vector<int> bls;
    std::vector<double2*> dst, in, tmp, out;
    std::vector<const double2*> src;
    int pos = 0;
    for (int k = 0; k < nblk; ++k) {
      BlockState& B = S[k];
      B.first = k * Bsz;
      for (int c = B.first; c < std::min(nrhs, B.first + Bsz); ++c) {
        if (gn[c] == 0.0) cdone[c] = 1;
        else B.cols.push_back(c);
      }
      if (B.cols.empty()) continue;
      bls.push_back(k);
      in.push_back(T1 + (size_t)pos * N);
      tmp.push_back(T2 + (size_t)pos * N);
      out.push_back(Vp(B, 0));
      for (int c : B.cols) {
        dst.push_back(T1 + (size_t)pos++ * N);
        src.push_back(Gb + (size_t)c * N);
      }
    }
    if ((e = gather(dst, src)) != LS_OK) return e;
    if (!bls.empty() && (e = block_qr(bls, in, tmp, out)) != LS_OK) return e;
    for (int k : bls)
      if (!S[k].qr_ok) {
        // linearly dependent right-hand sides: no block Krylov space of full
        // width; nothing has been done yet, so solve them column by column
        return gmres<T>(h, nrhs, tol, info);
      }
    for (int k : bls) start_cycle(S[k]);
  }

  const bool q64 = h->dim == 2 && !h->hmode && h->opt.sweep_schedule != LS_SWEEP_SEQUENTIAL;
  C<T>* vin = h->vin.as<C<T>>();
  C<T>* zout = h->zout.as<C<T>>();
  C<T>* aout = h->aout.as<C<T>>();
  while (true) {
    std::vector<int> act;
    int na = 0;
    for (int k = 0; k < nblk; ++k)
      if (S[k].in_cycle) {
        act.push_back(k);
        S[k].p0 = na;
        na += S[k].b();
      }
    if (act.empty()) break;
    // Z_j = P V_j, W = A Z_j for every column of the active blocks
    std::vector<void*> vptr, wptr;
    for (int k : act)
      for (int c = 0; c < S[k].b(); ++c) {
        vptr.push_back(Vp(S[k], S[k].j) + (size_t)c * N);
        wptr.push_back(Wb + (size_t)(S[k].p0 + c) * N);
      }
    if (upload(h, h->ptrs_a, vptr) != LS_OK || upload(h, h->ptrs_b, wptr) != LS_OK) return LS_E_DEVICE;
    if (q64) {
      e = apply_P<T>(h, vin, na, zout, h->ptrs_a.as<const double2*>(), nullptr);
    } else {
      for (int k : act)
        LSW_HIP_TRY((launch_cast_flat<T, double>(vin + (size_t)S[k].p0 * N, Vp(S[k], S[k].j), (size_t)S[k].b() * N, st)));
      e = h->hmode ? apply_sweep_ext<T>(h, vin, na, zout) : apply_P<T>(h, vin, na, zout);
    }
    if (e != LS_OK) return e;
    for (int k : act)
      LSW_HIP_TRY((launch_cast_flat<double, T>(Zp(S[k], S[k].j), zout + (size_t)S[k].p0 * N, (size_t)S[k].b() * N, st)));
    if (h->hmode) {
      LSW_HIP_TRY(launch_apply_H<T>(h->stencils(), zout, na, aout, st));
      LSW_HIP_TRY((launch_cast_flat<double, T>(Wb, aout, (size_t)na * N, st)));
    } else if (h->dim == 2) {
      if ((e = apply_A<T>(h, zout, na, aout, h->ptrs_b.as<double2* const>())) != LS_OK) return e;
    } else {
      if ((e = apply_A<T>(h, zout, na, aout)) != LS_OK) return e;
      LSW_HIP_TRY((launch_cast_flat<double, T>(Wb, aout, (size_t)na * N, st)));
    }
    // two passes of classical block Gram-Schmidt against V_0 .. V_j
    {
      for (int k : act) {
        BlockState& B = S[k];
        const int b = B.b(), K = (B.j + 1) * b;
        double2* Wk = Wb + (size_t)B.p0 * N;
        const double2* V0 = Vp(B, 0);
        for (double2* Cd : {C1d(k), C2d(k)}) {
          {
            Timed tg(h, kKGram, b);
            if ((e = gram(K, b, V0, Wk, Cd)) != LS_OK) return e;
          }
          Timed tu(h, kKGramUpd, b);
          LSW_BLAS_TRY(rocblas_zgemm(bl, ON, ON, iN, b, K, zs(mone), zc(V0), iN, zc(Cd), K, zs(one), zm(Wk), iN));
        }
        B.C1.resize((size_t)K * b);
        B.C2.resize((size_t)K * b);
        LSW_HIP_TRY(hipMemcpyAsync(B.C1.data(), C1d(k), B.C1.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
        LSW_HIP_TRY(hipMemcpyAsync(B.C2.data(), C2d(k), B.C2.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
      }
    }
    // W = V_{j+1} R (block_qr's first synchronisation also completes the
    // coefficient read-backs above)
    {
      std::vector<double2*> in, tmp, out;
      for (int k : act) {
        in.push_back(Wb + (size_t)S[k].p0 * N);
        tmp.push_back(T1 + (size_t)S[k].p0 * N);
        out.push_back(Vp(S[k], S[k].j + 1));
      }
      if ((e = block_qr(act, in, tmp, out)) != LS_OK) return e;
    }
    // host: the new block column of the block Hessenberg matrix, its
    // Householder QR and the residual estimates
    std::vector<int> ending;
    for (int k : act) {
      BlockState& B = S[k];
      const int b = B.b(), j = B.j, K = (j + 1) * b, c0 = j * b;
      const size_t ldh = (size_t)(rs + 1) * b;
      cplx* Hb = B.Hb.data();
      for (int c = 0; c < b; ++c) {
        cplx* col = Hb + (size_t)(c0 + c) * ldh;
        for (int i = 0; i < K; ++i) col[i] = B.C1[(size_t)c * K + i] + B.C2[(size_t)c * K + i];
        for (int i = 0; i < b; ++i) col[K + i] = i <= c ? B.R[(size_t)c * b + i] : cplx(0.0);
      }
      // earlier reflectors: reflector r acts on rows r .. r+b
      for (int r = 0; r < c0; ++r) {
        const cplx* v = Hb + (size_t)r * ldh + r;  // v[0] = 1 implied
        const cplx tc = std::conj(B.tau[r]);
        for (int c = c0; c < c0 + b; ++c) {
          cplx* y = Hb + (size_t)c * ldh + r;
          cplx w = y[0];
          for (int i = 1; i <= b; ++i) w += std::conj(v[i]) * y[i];
          w *= tc;
          y[0] -= w;
          for (int i = 1; i <= b; ++i) y[i] -= v[i] * w;
        }
      }
      // new reflectors for the columns c0 .. c0+b-1 (Householder vectors as
      // in LAPACK's zlarfg: H^H x = beta e_1, beta real)
      for (int col = c0; col < c0 + b; ++col) {
        cplx* x = Hb + (size_t)col * ldh + col;
        double xn = 0.0;
        for (int i = 1; i <= b; ++i) xn += std::norm(x[i]);
        xn = std::sqrt(xn);
        cplx tau = 0.0;
        if (xn != 0.0 || x[0].imag() != 0.0) {
          const double ar = x[0].real(), ai = x[0].imag();
          const double beta = -std::copysign(std::sqrt(ar * ar + ai * ai + xn * xn), ar);
          tau = cplx((beta - ar) / beta, -ai / beta);
          const cplx sc = 1.0 / (x[0] - beta);
          for (int i = 1; i <= b; ++i) x[i] *= sc;
          x[0] = beta;
        }
        B.tau[col] = tau;
        const cplx tc = std::conj(tau);
        auto reflect = [&](cplx* y) {
          cplx w = y[0];
          for (int i = 1; i <= b; ++i) w += std::conj(x[i]) * y[i];
          w *= tc;
          y[0] -= w;
          for (int i = 1; i <= b; ++i) y[i] -= x[i] * w;
        };
        if (tau != 0.0) {
          for (int c = col + 1; c < c0 + b; ++c) reflect(Hb + (size_t)c * ldh + col);
          for (int c = 0; c < b; ++c) reflect(B.E.data() + (size_t)c * ldh + col);
        }
      }
      B.j += 1;
      B.iters += 1;
      double est = 0.0;
      for (int c = 0; c < b; ++c) {
        col_its[B.cols[c]] += 1;
        double r2 = 0.0;
        for (int i = 0; i < b; ++i) r2 += std::norm(B.E[(size_t)c * ldh + K + i]);
        est = std::max(est, std::sqrt(r2) / gn[B.cols[c]]);
      }
      if (!std::isfinite(est)) {
        set_error("non-finite residual estimate in the block Arnoldi process");
        return LS_E_NUMERIC;
      }
      B.end = est <= tol || B.j == rs || B.iters >= max_iters || !B.qr_ok;
      if (B.end) ending.push_back(k);
    }
    if (ending.empty()) continue;
    // cycle end: Y = R^{-1} (Q^H E)[0:k], X += [Z_0 .. Z_{j-1}] Y
    std::vector<int> ecol;  // ending columns, in order
    {
      Timed tm(h, kKGramUpd, 0);
      for (int k : ending) {
        BlockState& B = S[k];
        const int b = B.b(), kk = B.j * b;
        const size_t ldh = (size_t)(rs + 1) * b;
        B.Y.assign((size_t)kk * b, 0.0);
        for (int c = 0; c < b; ++c)
          for (int i = kk - 1; i >= 0; --i) {
            cplx acc = B.E[(size_t)c * ldh + i];
            for (int m = i + 1; m < kk; ++m) acc -= B.Hb[(size_t)m * ldh + i] * B.Y[(size_t)c * kk + m];
            const cplx d = B.Hb[(size_t)i * ldh + i];
            B.Y[(size_t)c * kk + i] = d == 0.0 ? cplx(0.0) : acc / d;
          }
        LSW_HIP_TRY(hipMemcpyAsync(C1d(k), B.Y.data(), B.Y.size() * sizeof(double2), hipMemcpyHostToDevice, st));
        double2* out = T1 + (size_t)ecol.size() * N;
        LSW_BLAS_TRY(rocblas_zgemm(bl, ON, ON, iN, b, kk, zs(one), zc(Zp(B, 0)), iN, zc(C1d(k)), kk, zs(zero),
                                   zm(out), iN));
        for (int c : B.cols) ecol.push_back(c);
      }
    }
    const int ne = (int)ecol.size();
    {
      std::vector<AxpyOut> ho;
      std::vector<AxpyTerm<double>> ht;
      for (int q = 0; q < ne; ++q) {
        ht.push_back({T1 + (size_t)q * N, 0, 0});
        ho.push_back({Xb + (size_t)ecol[q] * N, q, q + 1, 0, -1, 0});
      }
      std::vector<double2> hc(1, make_double2(1.0, 0.0));
      if (upload(h, h->coefs, hc) != LS_OK || upload(h, h->outs, ho) != LS_OK || upload(h, h->terms64, ht) != LS_OK)
        return LS_E_DEVICE;
      LSW_HIP_TRY(launch_axpys<double>(h->outs.as<AxpyOut>(), ne, h->terms64.as<AxpyTerm<double>>(),
                                       h->coefs.as<double2>(), N, st));
    }
    // true residuals R[q] = g - A x of the ending columns (float64)
    {
      std::vector<void*> xp;
      for (int c : ecol) xp.push_back(Xb + (size_t)c * N);
      if (upload(h, h->ptrs_b, xp) != LS_OK) return LS_E_DEVICE;
      if (h->dim == 2 && !h->hmode) {
        if ((e = apply_A<double>(h, T1, ne, T2, nullptr, h->ptrs_b.as<const double2*>())) != LS_OK) return e;
      } else {
        std::vector<double2*> dst;
        std::vector<const double2*> src;
        for (int q = 0; q < ne; ++q) {
          dst.push_back(T1 + (size_t)q * N);
          src.push_back(Xb + (size_t)ecol[q] * N);
        }
        if ((e = gather(dst, src)) != LS_OK) return e;
        if (h->hmode) LSW_HIP_TRY(launch_apply_H<double>(h->stencils(), T1, ne, T2, st));
        else if ((e = apply_A<double>(h, T1, ne, T2)) != LS_OK) return e;
      }
      std::vector<AxpyOut> ho;
      std::vector<AxpyTerm<double>> ht;
      for (int q = 0; q < ne; ++q) {
        ht.push_back({Gb + (size_t)ecol[q] * N, 0, 0});
        ht.push_back({T2 + (size_t)q * N, 0, 1});
        ho.push_back({Rb + (size_t)q * N, 2 * q, 2 * q + 2, 1, -1, 0});
      }
      if (upload(h, h->outs, ho) != LS_OK || upload(h, h->terms64, ht) != LS_OK) return LS_E_DEVICE;
      LSW_HIP_TRY(launch_axpys<double>(h->outs.as<AxpyOut>(), ne, h->terms64.as<AxpyTerm<double>>(),
                                       h->coefs.as<double2>(), N, st));
    }
    std::vector<double> rn;
    if ((e = colnorms(Rb, ne, rn)) != LS_OK) return e;
    // which columns stay; the blocks that go on restart from their residuals
    std::vector<int> bls;
    std::vector<double2*> dst, in, tmp, out;
    std::vector<const double2*> src;
    int q = 0, pos = 0;
    for (int k : ending) {
      BlockState& B = S[k];
      std::vector<int> keep;
      std::vector<int> keep_q;
      for (int c : B.cols) {
        if (!std::isfinite(rn[q])) {
          set_error("non-finite true residual");
          return LS_E_NUMERIC;
        }
        relres[c] = rn[q] / gn[c];
        if (relres[c] <= tol) cdone[c] = 1;
        else if (B.iters >= max_iters) cdone[c] = 2;
        else {
          keep.push_back(c);
          keep_q.push_back(q);
        }
        ++q;
      }
      B.in_cycle = false;
      B.cols = keep;
      if (keep.empty()) continue;
      bls.push_back(k);
      in.push_back(T1 + (size_t)pos * N);
      tmp.push_back(T2 + (size_t)pos * N);
      out.push_back(Vp(B, 0));
      for (int qq : keep_q) {
        dst.push_back(T1 + (size_t)pos++ * N);
        src.push_back(Rb + (size_t)qq * N);
      }
    }
    if ((e = gather(dst, src)) != LS_OK) return e;
    if (!bls.empty() && (e = block_qr(bls, in, tmp, out)) != LS_OK) return e;
    for (int k : bls) {
      if (!S[k].qr_ok) {
        set_error("the residuals of a block became linearly dependent at a restart");
        return LS_E_NUMERIC;
      }
      start_cycle(S[k]);
    }
  }
  info.resize(nrhs);
  bool all = true;
  for (int c = 0; c < nrhs; ++c) {
    info[c].iterations = col_its[c];
    info[c].rel_residual = gn[c] == 0.0 ? 0.0 : relres[c];
    info[c].converged = cdone[c] == 1;
    all = all && cdone[c] == 1;
  }
  if (!all) {
    set_error("block GMRES reached max_iters before the tolerance for some right-hand side");
    return LS_E_NOCONV;
  }
  return LS_OK;
}

ls_status run_gmres(ls_handle* h, int nrhs, double tol, std::vector<ls_rhs_info>& info) {
  if (h->opt.block_size > 1 && nrhs > 1)
    return h->prec == LS_FP64 ? block_gmres<double>(h, nrhs, tol, info) : block_gmres<float>(h, nrhs, tol, info);
  return h->prec == LS_FP64 ? gmres<double>(h, nrhs, tol, info) : gmres<float>(h, nrhs, tol, info);
}

ls_status device_setup(ls_handle* h, const double* m_dev) {
  HostSetup& Hs = h->H;
  const int n = h->n, L = h->L, P = h->P;
  hipStream_t st = h->st;
  // tables to the device
  LSW_ALLOC(h->m, (size_t)n * n * sizeof(double));
  LSW_HIP_TRY(hipMemcpyAsync(h->m.p, m_dev, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<float> m32((size_t)n * n);
  {
    std::vector<double> mh((size_t)n * n);
    LSW_HIP_TRY(hipMemcpy(mh.data(), m_dev, mh.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < mh.size(); ++i) m32[i] = (float)mh[i];
  }
  LSW_ALLOC(h->m32, m32.size() * sizeof(float));
  LSW_HIP_TRY(hipMemcpyAsync(h->m32.p, m32.data(), m32.size() * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<double2> tw(P);
  std::vector<float2> tw32(P);
  for (int k = 0; k < P; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)P;
    tw[k] = make_double2(std::cos(a), std::sin(a));
    tw32[k] = make_float2((float)tw[k].x, (float)tw[k].y);
  }
  LSW_ALLOC(h->tw, P * sizeof(double2));
  LSW_ALLOC(h->tw32, P * sizeof(float2));
  LSW_HIP_TRY(hipMemcpyAsync(h->tw.p, tw.data(), P * sizeof(double2), hipMemcpyHostToDevice, st));
  LSW_HIP_TRY(hipMemcpyAsync(h->tw32.p, tw32.data(), P * sizeof(float2), hipMemcpyHostToDevice, st));
  auto to_d2 = [](const std::vector<cd>& v) {
    std::vector<double2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2(v[i].real(), v[i].imag());
    return o;
  };
  // Green's table quadrant -> khat
  {
    DBuf kq, scratch;
    const std::vector<double2> kq_h = to_d2(Hs.kq);
    LSW_ALLOC(kq, kq_h.size() * sizeof(double2));
    LSW_ALLOC(scratch, (size_t)P * P * sizeof(double2));
    const size_t half = (size_t)(P / 2 + 1) * (P / 2 + 1);
    LSW_ALLOC(h->khat, half * sizeof(double2));
    LSW_ALLOC(h->khat32, half * sizeof(float2));
    LSW_HIP_TRY(hipMemcpyAsync(kq.p, kq_h.data(), kq_h.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    LSW_HIP_TRY(launch_green_spectrum(kq.as<double2>(), n, h->tw.as<double2>(), scratch.as<double2>(),
                                      h->khat.as<double2>(), h->khat32.as<float2>(), st));
    LSW_HIP_TRY(hipStreamSynchronize(st));
  }
  std::vector<double2> ab(9), bb(9);
  for (int i = 0; i < 9; ++i) {
    ab[i] = make_double2(Hs.alpha[i].real(), Hs.alpha[i].imag());
    bb[i] = make_double2(Hs.beta[i].real(), Hs.beta[i].imag());
  }
  LSW_ALLOC(h->alpha, 9 * sizeof(double2));
  LSW_ALLOC(h->beta, 9 * sizeof(double2));
  if (upload(h, h->alpha, ab) != LS_OK || upload(h, h->beta, bb) != LS_OK) return LS_E_DEVICE;
  const std::vector<double2> gg = to_d2(Hs.gamma_glob), ga = to_d2(Hs.gamma_aux);
  LSW_ALLOC(h->gglob, gg.size() * sizeof(double2));
  LSW_ALLOC(h->gaux, std::max<size_t>(ga.size(), 1) * sizeof(double2));
  LSW_ALLOC(h->kmap, Hs.kmap.size() * sizeof(int));
  if (upload(h, h->gglob, gg) != LS_OK || upload(h, h->gaux, ga) != LS_OK || upload(h, h->kmap, Hs.kmap) != LS_OK)
    return LS_E_DEVICE;
  // slice plan and factor storage
  const int nl = h->nslices;
  std::vector<int> lo(nl), hi(nl), first(nl), t(nl), naux(nl), org(nl), dir(nl), prev(nl), next(nl), nlam(nl);
  std::vector<size_t> fso(nl), fgo(nl);
  size_t fs_tot = 0, fg_tot = 0;
  h->tbl_of_grid.assign(nl, 0);
  for (int k = 0; k < nl; ++k) {
    const SlicePlan& p = Hs.slices[k];
    lo[k] = p.lo;
    hi[k] = p.hi;
    first[k] = p.first;
    t[k] = p.t;
    naux[k] = p.naux;
    org[k] = p.org;
    dir[k] = p.dir;
    prev[k] = p.prev;
    next[k] = p.next;
    nlam[k] = p.next_lam;
    h->tbl_of_grid[p.grid] = k;
    fso[k] = fs_tot;
    fgo[k] = fg_tot;
    fs_tot += (size_t)L * factor_stride(p.t, p.hi - p.lo + 1);
    fg_tot += (size_t)L * factor_stride(p.t, 0);
  }
  h->t_host = t;
  h->fstride_host.assign(nl, 0);
  h->tw_host.assign(nl, 0);
  for (int k = 0; k < nl; ++k) {
    h->fstride_host[k] = factor_stride(t[k], hi[k] - lo[k] + 1);
    h->tw_host[k] = hi[k] - lo[k] + 1;
  }
  LSW_ALLOC(h->s_lo, nl * sizeof(int));
  LSW_ALLOC(h->s_hi, nl * sizeof(int));
  LSW_ALLOC(h->s_first, nl * sizeof(int));
  LSW_ALLOC(h->s_t, nl * sizeof(int));
  for (DBuf* d : {&h->s_naux, &h->s_org, &h->s_dir, &h->s_prev, &h->s_next, &h->s_nlam}) LSW_ALLOC(*d, nl * sizeof(int));
  LSW_ALLOC(h->fs_off, nl * sizeof(size_t));
  LSW_ALLOC(h->fg_off, nl * sizeof(size_t));
  if (upload(h, h->s_lo, lo) != LS_OK || upload(h, h->s_hi, hi) != LS_OK || upload(h, h->s_first, first) != LS_OK ||
      upload(h, h->s_t, t) != LS_OK || upload(h, h->fs_off, fso) != LS_OK || upload(h, h->fg_off, fgo) != LS_OK ||
      upload(h, h->s_naux, naux) != LS_OK || upload(h, h->s_org, org) != LS_OK || upload(h, h->s_dir, dir) != LS_OK ||
      upload(h, h->s_prev, prev) != LS_OK || upload(h, h->s_next, next) != LS_OK || upload(h, h->s_nlam, nlam) != LS_OK)
    return LS_E_DEVICE;
  const size_t cs = h->prec == LS_FP64 ? sizeof(double2) : sizeof(float2);
  // padding: the last 16-byte copy of a chunk may read one value past the end
  LSW_ALLOC(h->FS, (fs_tot + 128) * cs);
  LSW_ALLOC(h->FG, (fg_tot + 128) * cs);
  LSW_ALLOC(h->Hm, (size_t)nl * L * 3 * cs);
  LSW_ALLOC(h->Hp, (size_t)nl * L * 3 * cs);
  LSW_ALLOC(h->status, sizeof(int));
  LSW_HIP_TRY(hipMemsetAsync(h->status.p, 0, sizeof(int), st));
  const StencilTables S = h->stencils();
  if (h->prec == LS_FP64) {
    LSW_HIP_TRY(launch_factor_slices<double>(S, h->slices(), h->FS.as<double2>(), h->FG.as<double2>(),
                                             h->Hm.as<double2>(), h->Hp.as<double2>(), h->status.as<int>(), st));
  } else {
    LSW_HIP_TRY(launch_factor_slices<float>(S, h->slices(), h->FS.as<float2>(), h->FG.as<float2>(),
                                            h->Hm.as<float2>(), h->Hp.as<float2>(), h->status.as<int>(), st));
  }
  int status = 0;
  LSW_HIP_TRY(hipMemcpyAsync(&status, h->status.p, sizeof(int), hipMemcpyDeviceToHost, st));
  LSW_HIP_TRY(hipStreamSynchronize(st));
  if (status != 0) {
    set_error("zero pivot in the factorization of slice " + std::to_string(Hs.slices[status - 1].grid));
    return LS_E_SINGULAR;
  }
  {
    ls_status e = h->prec == LS_FP64 ? build_mfma_factors<double>(h) : build_mfma_factors<float>(h);
    if (e != LS_OK) return e;
  }
  if (h->opt.sweep_schedule == LS_SWEEP_INTERFACE) {
    ls_status e = h->prec == LS_FP64 ? build_interface<double>(h) : build_interface<float>(h);
    if (e != LS_OK) return e;
  }
  return LS_OK;
}

ls_status check_precision(const ls_handle* h, int precision, bool factors) {
  if (precision != LS_FP64 && precision != LS_MIXED) {
    set_error("precision must be LS_FP64 or LS_MIXED");
    return LS_E_INVALID;
  }
  if (factors && precision != h->prec) {
    set_error("this entry point needs the handle's own precision");
    return LS_E_INVALID;
  }
  return LS_OK;
}

// ---- autotuning ------------------------------------------------------------

// Layer thicknesses w >= 2 whose slice subproblems all have at most 32 lines:
// the first slice b PML lines + w, the middle ones b auxiliary lines + w, the
// last b auxiliary lines + the remaining lines + b PML lines (one slice: all L).
std::vector<int> layer_candidates(int n, int b, int fronts = 1) {
  std::vector<int> out;
  const int lines = n + 2;
  for (int w = 2; w <= lines; ++w) {
    int tmax = 0;
    for (const SlicePlan& p : plan_slices(n, b, w, fronts)) tmax = std::max(tmax, p.t);
    if (tmax <= 32) out.push_back(w);
  }
  return out;
}

// One solve of k plane waves to a 1e-6 residual, timed on the host around the
// call (which ends with a stream synchronisation), after an untimed solve to a
// loose tolerance that sizes the workspaces and captures the graphs.
ls_status probe_solve(ls_handle* h, int k, double& ms, int& iters, bool& converged) {
  DBuf rhs, u;
  LSW_ALLOC(rhs, (size_t)k * h->N * sizeof(double2));
  LSW_ALLOC(u, (size_t)k * h->N * sizeof(double2));
  LSW_HIP_TRY(launch_plane_waves(rhs.as<double2>(), h->n, h->omega, k, h->st));
  std::vector<ls_rhs_info> info(k);
  ls_status e = ls_solve(h, rhs.p, k, LS_RHS_INCIDENT, 1e-1, u.p, info.data());
  if (e != LS_OK && e != LS_E_NOCONV) return e;
  const auto t0 = std::chrono::steady_clock::now();
  e = ls_solve(h, rhs.p, k, LS_RHS_INCIDENT, 1e-6, u.p, info.data());
  const auto t1 = std::chrono::steady_clock::now();
  if (e != LS_OK && e != LS_E_NOCONV) return e;
  ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  converged = e == LS_OK;
  iters = 0;
  for (const ls_rhs_info& i : info) iters = std::max(iters, i.iterations);
  return LS_OK;
}

// Batch sizes the kernel choice is measured at, up to kmax (and kmax itself).
std::vector<int> tune_sizes(int kmax) {
  kmax = std::min(kmax, kChoiceMax);
  std::vector<int> s;
  for (int nb : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256})
    if (nb <= kmax) s.push_back(nb);
  if (s.back() != kmax) s.push_back(kmax);
  return s;
}

// Times one preconditioner apply (the best of three, after an untimed one) per
// kernel choice at each measured batch size on a zero batch (no kernel's work
// depends on the values), keeps the fastest, and gives every batch size the
// choice of the nearest measured size at or above it.
template <typename T>
ls_status tune_kernels(ls_handle* h, int kmax) {
  const std::vector<int> sizes = tune_sizes(kmax);
  const int top = sizes.back();
  ls_status e = ensure_workspace(h, top);
  if (e != LS_OK) return e;
  DBuf r, z;
  LSW_ALLOC(r, (size_t)top * h->N * sizeof(C<T>));
  LSW_ALLOC(z, (size_t)top * h->N * sizeof(C<T>));
  LSW_HIP_TRY(hipMemsetAsync(r.p, 0, r.bytes, h->st));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  LSW_HIP_TRY(hipEventCreate(&ev0));
  LSW_HIP_TRY(hipEventCreate(&ev1));
  auto time_apply = [&](int nb, KernelChoice c, double& ms) -> ls_status {
    h->choice.assign(kChoiceMax + 1, c);
    ls_status s = apply_P<T>(h, r.as<C<T>>(), nb, z.as<C<T>>());
    if (s != LS_OK) return s;
    ms = std::numeric_limits<double>::infinity();
    for (int rep = 0; rep < 3; ++rep) {
      LSW_HIP_TRY(hipEventRecord(ev0, h->st));
      if ((s = apply_P<T>(h, r.as<C<T>>(), nb, z.as<C<T>>())) != LS_OK) return s;
      LSW_HIP_TRY(hipEventRecord(ev1, h->st));
      LSW_HIP_TRY(hipEventSynchronize(ev1));
      float t = 0;
      LSW_HIP_TRY(hipEventElapsedTime(&t, ev0, ev1));
      ms = std::min(ms, (double)t);
    }
    return LS_OK;
  };
  std::vector<ls_tune_kernels> rows;
  for (int nb : sizes) {
    KernelChoice best{16, 1};
    double best_ms = std::numeric_limits<double>::infinity();
    const int iface0 = nb <= 4 ? 0 : 1;
    for (int sk : {1, 4, 8, 16}) {
      if ((sk == 4 && nb < 2) || (sk == 8 && nb < 5)) continue;  // whole idle waves
      double ms;
      if ((e = time_apply(nb, {sk, iface0}, ms)) != LS_OK) break;
      if (ms < best_ms) best_ms = ms, best = {sk, iface0};
    }
    // the other interface kernels with that slice kernel
    for (int ik : {0, 1}) {
      if (e != LS_OK || ik == iface0 || (ik == 0 && nb > 4)) continue;
      double ms;
      if ((e = time_apply(nb, {best.slice, ik}, ms)) == LS_OK && ms < best_ms) best_ms = ms, best.iface = ik;
    }
    if (e != LS_OK) break;
    rows.push_back({nb, best.slice, best.iface, best_ms});
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  set_default_choices(h);
  if (e != LS_OK) return e;
  for (int nb = 1; nb <= kChoiceMax; ++nb) {
    size_t i = 0;
    while (i + 1 < rows.size() && rows[i].nrhs < nb) ++i;
    KernelChoice c{rows[i].slice_kernel, rows[i].iface_kernel};
    if (nb > 4 && c.iface == 0) c.iface = 1;
    h->choice[nb] = c;
  }
  h->choice[0] = h->choice[1];
  h->tune_k = rows;
  h->drop_graphs();
  return LS_OK;
}

// y = a x + c K (s .* x) with s = m (with_m) or 1, on the handle's grid
template <typename T>
ls_status convolve_any(ls_handle* h, const C<T>* x, bool with_m, int nb, T a, T c, C<T>* y) {
  const T* m = with_m ? Prec<T>::m(h) : nullptr;
  if (h->dim == 3)
    LSW_HIP_TRY(launch_convolve3<T>(x, m, h->n, nb, Prec<T>::khat3(h), Prec<T>::tw(h), a, c, h->s3->w1.as<C<T>>(),
                                    h->s3->w2.as<C<T>>(), y, h->st));
  else
    LSW_HIP_TRY(launch_convolve<T>(x, m, h->n, nb, Prec<T>::khat(h), Prec<T>::tw(h), a, c, Prec<T>::fftw(h), y,
                                   h->st));
  return LS_OK;
}

// 3D setup on the device: medium, twiddles, Green's spectrum octant,
// stencil tables, and the factors of every slab (all slabs at once).
template <typename T>
ls_status factor3(ls_handle* h) {
  Sweep3& s = *h->s3;
  const int L = h->L, nl = (int)s.slabs.size();
  hipStream_t st = h->st;
  const Stencil3 S = stencil3(h);
  // two chains per slab (top and bottom), each with its own work arrays
  const int ne = 2 * nl;
  std::vector<DBuf> wS(ne), wW(ne), wSp(ne), wXr(ne), wcf(ne), wpiv(ne), wperm(ne);
  std::vector<Slab3Work> works(ne);
  std::vector<Slab3> eslabs(ne);
  std::vector<C<T>*> eF(ne);
  s.F.resize(nl);
  s.cbc.resize(nl);
  s.cm.resize(nl);
  s.cp.resize(nl);
  std::vector<C<T>*> Fp(nl), cbp(nl), cmp(nl, nullptr), cpp(nl, nullptr);
  for (int k = 0; k < nl; ++k) {
    const size_t nb = s.slabs[k].nb, nb2 = nb * nb;
    for (int e = 2 * k; e < 2 * k + 2; ++e) {
      LSW_ALLOC(wS[e], nb2 * sizeof(double2));
      LSW_ALLOC(wW[e], nb2 * sizeof(double2));
      LSW_ALLOC(wSp[e], nb2 * sizeof(double2));
      LSW_ALLOC(wXr[e], 32 * nb * sizeof(double2));
      LSW_ALLOC(wcf[e], 27 * nb * sizeof(double2));
      LSW_ALLOC(wpiv[e], nb * sizeof(int));
      LSW_ALLOC(wperm[e], nb * sizeof(int));
      works[e] = {wS[e].as<double2>(), wW[e].as<double2>(), wSp[e].as<double2>(), wXr[e].as<double2>(),
                  wcf[e].as<double2>(), wpiv[e].as<int>(), wperm[e].as<int>(), e == 2 * k ? +1 : -1};
      eslabs[e] = s.slabs[k];
    }
    LSW_ALLOC(s.F[k], (size_t)L * nb2 * sizeof(C<T>));
    LSW_ALLOC(s.cbc[k], (size_t)L * 2 * nb * 9 * sizeof(C<T>));
    Fp[k] = s.F[k].as<C<T>>();
    eF[2 * k] = eF[2 * k + 1] = Fp[k];
    cbp[k] = s.cbc[k].as<C<T>>();
    if (k > 0) {
      LSW_ALLOC(s.cm[k], (size_t)L * L * 9 * sizeof(C<T>));
      cmp[k] = s.cm[k].as<C<T>>();
    }
    if (k < nl - 1) {
      LSW_ALLOC(s.cp[k], (size_t)L * L * 9 * sizeof(C<T>));
      cpp[k] = s.cp[k].as<C<T>>();
    }
  }
  DBuf slabs_d, eslabs_d, works_d, F_d, cb_d, cm_d, cp_d, status;
  LSW_ALLOC(slabs_d, nl * sizeof(Slab3));
  LSW_ALLOC(eslabs_d, ne * sizeof(Slab3));
  LSW_ALLOC(works_d, ne * sizeof(Slab3Work));
  LSW_ALLOC(F_d, ne * sizeof(void*));
  LSW_ALLOC(cb_d, nl * sizeof(void*));
  LSW_ALLOC(cm_d, nl * sizeof(void*));
  LSW_ALLOC(cp_d, nl * sizeof(void*));
  LSW_ALLOC(status, sizeof(int));
  if (upload(h, slabs_d, s.slabs) != LS_OK || upload(h, eslabs_d, eslabs) != LS_OK ||
      upload(h, works_d, works) != LS_OK || upload(h, F_d, eF) != LS_OK ||
      upload(h, cb_d, cbp) != LS_OK || upload(h, cm_d, cmp) != LS_OK || upload(h, cp_d, cpp) != LS_OK)
    return LS_E_DEVICE;
  LSW_HIP_TRY(hipMemsetAsync(status.p, 0, sizeof(int), st));
  LSW_HIP_TRY(launch3_factor<T>(S, eslabs_d.as<Slab3>(), works_d.as<Slab3Work>(), ne, s.maxnb,
                                F_d.as<C<T>* const>(), status.as<int>(), st));
  LSW_HIP_TRY(launch3_apply_coefs<T>(S, slabs_d.as<Slab3>(), nl, s.maxnb, cb_d.as<C<T>* const>(),
                                     cm_d.as<C<T>* const>(), cp_d.as<C<T>* const>(), st));
  int bad = 0;
  LSW_HIP_TRY(hipMemcpyAsync(&bad, status.p, sizeof(int), hipMemcpyDeviceToHost, st));
  LSW_HIP_TRY(hipStreamSynchronize(st));
  if (bad) {
    set_error("zero pivot in the factorization of slab " + std::to_string(bad - 1));
    return LS_E_SINGULAR;
  }
  return LS_OK;
}

ls_status device_setup3(ls_handle* h, const double* m_dev, const std::vector<double>& mh) {
  Sweep3& s = *h->s3;
  const HostSetup3& H3 = s.H;
  const int n = h->n, P = h->P;
  const size_t n3 = (size_t)n * n * n;
  hipStream_t st = h->st;
  LSW_ALLOC(h->m, n3 * sizeof(double));
  LSW_HIP_TRY(hipMemcpyAsync(h->m.p, m_dev, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<float> m32(n3);
  for (size_t i = 0; i < n3; ++i) m32[i] = (float)mh[i];
  LSW_ALLOC(h->m32, n3 * sizeof(float));
  LSW_HIP_TRY(hipMemcpyAsync(h->m32.p, m32.data(), n3 * sizeof(float), hipMemcpyHostToDevice, st));
  std::vector<double2> tw(P);
  std::vector<float2> tw32(P);
  for (int k = 0; k < P; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)P;
    tw[k] = make_double2(std::cos(a), std::sin(a));
    tw32[k] = make_float2((float)tw[k].x, (float)tw[k].y);
  }
  LSW_ALLOC(h->tw, P * sizeof(double2));
  LSW_ALLOC(h->tw32, P * sizeof(float2));
  LSW_HIP_TRY(hipMemcpyAsync(h->tw.p, tw.data(), P * sizeof(double2), hipMemcpyHostToDevice, st));
  LSW_HIP_TRY(hipMemcpyAsync(h->tw32.p, tw32.data(), P * sizeof(float2), hipMemcpyHostToDevice, st));
  auto to_d2 = [](const cd* v, size_t count) {
    std::vector<double2> o(count);
    for (size_t i = 0; i < count; ++i) o[i] = make_double2(v[i].real(), v[i].imag());
    return o;
  };
  {
    DBuf kq, scratch;
    const std::vector<double2> kq_h = to_d2(H3.kq.data(), H3.kq.size());
    LSW_ALLOC(kq, kq_h.size() * sizeof(double2));
    LSW_ALLOC(scratch, (size_t)P * P * P * sizeof(double2));
    const size_t Hh = P / 2 + 1;
    LSW_ALLOC(s.khat, Hh * Hh * Hh * sizeof(double2));
    LSW_ALLOC(s.khat32, Hh * Hh * Hh * sizeof(float2));
    LSW_HIP_TRY(hipMemcpyAsync(kq.p, kq_h.data(), kq_h.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    LSW_HIP_TRY(launch_green_spectrum3(kq.as<double2>(), n, h->tw.as<double2>(), scratch.as<double2>(),
                                       s.khat.as<double2>(), s.khat32.as<float2>(), st));
    LSW_HIP_TRY(hipStreamSynchronize(st));
  }
  const std::vector<double2> al = to_d2(H3.alpha, 27), be = to_d2(H3.beta, 27),
                             gg = to_d2(H3.gamma_glob.data(), H3.gamma_glob.size()),
                             ga = to_d2(H3.gamma_aux.data(), H3.gamma_aux.size());
  LSW_ALLOC(s.alpha, al.size() * sizeof(double2));
  LSW_ALLOC(s.beta, be.size() * sizeof(double2));
  LSW_ALLOC(s.gglob, gg.size() * sizeof(double2));
  LSW_ALLOC(s.gaux, ga.size() * sizeof(double2));
  LSW_ALLOC(s.kmap, H3.kmap.size() * sizeof(int));
  if (upload(h, s.alpha, al) != LS_OK || upload(h, s.beta, be) != LS_OK || upload(h, s.gglob, gg) != LS_OK ||
      upload(h, s.gaux, ga) != LS_OK || upload(h, s.kmap, H3.kmap) != LS_OK)
    return LS_E_DEVICE;
  return h->prec == LS_FP64 ? factor3<double>(h) : factor3<float>(h);
}

// ls_setup for grid dim 3 (options already checked)
ls_status setup3_handle(const ls_grid* grid, double omega, const double* m_dev, int pml_width, int layer_thickness,
                        const ls_options& o, ls_handle** out) {
  const int n = grid->n;
  if (n < 1 || n > 1023) {
    set_error("3D: n must be in [1, 1023]");
    return LS_E_INVALID;
  }
  if (layer_thickness < 1) {
    set_error("3D: layer_thickness must be >= 1 (no autotuning in 3D)");
    return LS_E_INVALID;
  }
  std::unique_ptr<ls_handle> h(new ls_handle());
  h->dim = 3;
  h->s3.reset(new Sweep3());
  h->opt = o;
  h->st = static_cast<hipStream_t>(o.hip_stream);
  LSW_HIP_TRY(hipGetDevice(&h->device));
  const size_t n3 = (size_t)n * n * n;
  std::vector<double> mh(n3);
  LSW_HIP_TRY(hipMemcpy(mh.data(), m_dev, n3 * sizeof(double), hipMemcpyDeviceToHost));
  Sweep3& s = *h->s3;
  const std::string err = build_host_setup3(mh.data(), n, omega, pml_width, layer_thickness, o.pml_C,
                                            o.freq_samples, kSlab3MaxLines, kSlab3MaxBlock, s.H);
  if (!err.empty()) {
    set_error(err);
    return LS_E_INVALID;
  }
  h->n = n;
  h->b = pml_width;
  h->w = layer_thickness;
  h->L = s.H.L;
  h->P = fft_len(n);
  h->ns = s.H.ns;
  h->nslices = s.H.nslices;
  h->omega = omega;
  h->prec = o.precision;
  h->H.C = o.pml_C;
  h->H.h = s.H.h;
  h->H.freq_lo = s.H.freq_lo;
  h->H.freq_delta = s.H.freq_delta;
  h->H.slices = s.H.slices;
  set_default_choices(h.get());
  h->N = n3;
  h->E = (size_t)h->L * h->L * h->L;
  for (const SlicePlan& p : s.H.slices) {
    const Slab3 sl{p.first, p.lo, p.hi, p.t, p.naux, p.t * h->L};
    s.slabs.push_back(sl);
    s.maxnb = std::max(s.maxnb, sl.nb);
  }
  if (s.maxnb > kSlab3MaxBlock) {
    set_error("3D: a slab block has " + std::to_string(s.maxnb) + " unknowns (slab lines x L); at most " +
              std::to_string(kSlab3MaxBlock) + " are supported (reduce w or b)");
    return LS_E_INVALID;
  }
  const ls_status e = device_setup3(h.get(), m_dev, mh);
  if (e != LS_OK) return e;
  *out = h.release();
  return LS_OK;
}

// ---- scratch of the allocation-free operator apply ---------------------------
// The FFT work array of ls_apply_A_noalloc (the n x P row transforms of every
// right-hand side) lives in this code object's own device memory, one copy
// per GPU, held until the process ends. On the host the name `scratch` is
// only a stand-in for the symbol: host code uses the device address that
// hipGetSymbolAddress returns, resolved once per device with that device
// current, and never passes the name itself to a kernel.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) static unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array; the lookup runs once per
// device (at the first ls_setup on it, or at the first allocation-free call).
ls_status scratch_for_device(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index out of range for the static scratch table");
    return LS_E_DEVICE;
  }
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    LSW_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) LSW_HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) LSW_HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress of the static scratch array failed: ") + hipGetErrorString(e));
      return LS_E_DEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return LS_OK;
}

}  // namespace

extern "C" {

void ls_default_options(ls_options* o) {
  if (!o) return;
  o->precision = LS_FP64;
  o->restart = 30;
  o->max_iters = 1000;
  o->pml_C = 10.0;
  o->freq_samples = 0;
  o->autotune = 0;
  o->hip_stream = nullptr;
  o->sweep_schedule = LS_SWEEP_INTERFACE;
  o->fronts = 1;
  o->block_size = 1;
}

const char* ls_last_error(void) { return lsw::get_error(); }

ls_status ls_setup(const ls_grid* grid, double omega, const double* m_dev, int pml_width, int layer_thickness,
                   const ls_options* opts, ls_handle** out) {
  try {
    set_error("");
    if (!out) {
      set_error("out must not be NULL");
      return LS_E_INVALID;
    }
    *out = nullptr;
    if (!grid || !m_dev) {
      set_error("grid and m_dev must not be NULL");
      return LS_E_INVALID;
    }
    if (grid->dim != 2 && grid->dim != 3) {
      set_error("dim must be 2 or 3");
      return LS_E_INVALID;
    }
    ls_options o;
    ls_default_options(&o);
    if (opts) o = *opts;
    if (o.precision != LS_FP64 && o.precision != LS_MIXED) {
      set_error("precision must be LS_FP64 or LS_MIXED");
      return LS_E_INVALID;
    }
    if (o.sweep_schedule != LS_SWEEP_INTERFACE && o.sweep_schedule != LS_SWEEP_SEQUENTIAL) {
      set_error("sweep_schedule must be LS_SWEEP_INTERFACE or LS_SWEEP_SEQUENTIAL");
      return LS_E_INVALID;
    }
    if (o.fronts != 1 && o.fronts != 2) {
      set_error("fronts must be 1 or 2");
      return LS_E_INVALID;
    }
    if (o.fronts == 2 && (grid->dim != 2 || o.sweep_schedule != LS_SWEEP_INTERFACE)) {
      set_error("fronts = 2 needs a 2D grid and the interface sweep schedule");
      return LS_E_INVALID;
    }
    if (o.block_size < 1 || o.block_size > 64 || (o.block_size > 1 && o.block_size * o.restart > 2048)) {
      set_error("block_size must be in [1, 64], with block_size * restart <= 2048 when above 1");
      return LS_E_INVALID;
    }
    if (o.restart < 1 || o.restart > 200 || o.max_iters < 1) {
      set_error("restart must be in [1, 200] and max_iters >= 1");
      return LS_E_INVALID;
    }
    if (o.autotune < 0 || o.autotune > 4096) {
      set_error("autotune must be in [0, 4096] (right-hand sides to tune for)");
      return LS_E_INVALID;
    }
    if (grid->dim == 3) {
      if (o.autotune != 0) {
        set_error("3D: autotune is not available");
        return LS_E_INVALID;
      }
      return setup3_handle(grid, omega, m_dev, pml_width, layer_thickness, o, out);
    }
    if (layer_thickness <= 0) {
      if (o.autotune == 0) {
        set_error("layer_thickness must be >= 1, or <= 0 with opts->autotune > 0");
        return LS_E_INVALID;
      }
      // choose w: set up every candidate and time a probe solve on it
      std::vector<int> cands = layer_candidates(grid->n, pml_width, o.fronts);
      if (grid->n < 1 || pml_width < 1 || cands.empty()) {
        set_error("no layer thickness gives slices of at most 32 lines for this n and pml_width");
        return LS_E_INVALID;
      }
      // the four thinnest: thicker layers only lengthen every slice solve
      // (and push the slices into the 32-line class) for a shorter chain
      if (cands.size() > 4) cands.resize(4);
      ls_options oc = o;
      oc.autotune = 0;
      oc.max_iters = std::min(o.max_iters, 300);  // bounds the cost of a poor candidate
      std::vector<ls_tune_layer> rows;
      int best = -1;
      double best_ms = std::numeric_limits<double>::infinity();
      for (int w : cands) {
        ls_handle* hc = nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        ls_status e = ls_setup(grid, omega, m_dev, pml_width, w, &oc, &hc);
        const auto t1 = std::chrono::steady_clock::now();
        if (e != LS_OK) return e;
        double ms = 0;
        int iters = 0;
        bool conv = false;
        e = probe_solve(hc, o.autotune, ms, iters, conv);
        const int nl = hc->nslices;
        ls_destroy(hc);
        if (e != LS_OK) return e;
        rows.push_back({w, nl, iters, std::chrono::duration<double, std::milli>(t1 - t0).count(), ms});
        const double score = conv ? ms : std::numeric_limits<double>::infinity();
        if (best < 0 || score < best_ms) best = w, best_ms = score;
      }
      ls_handle* hb = nullptr;
      const ls_status e = ls_setup(grid, omega, m_dev, pml_width, best, &o, &hb);
      if (e != LS_OK) return e;
      hb->tune_w = rows;
      *out = hb;
      return LS_OK;
    }
    std::unique_ptr<ls_handle> h(new ls_handle());
    h->opt = o;
    h->st = static_cast<hipStream_t>(o.hip_stream);
    LSW_HIP_TRY(hipGetDevice(&h->device));
    const int n = grid->n;
    // the FFT passes hold S >= 1 complex128 sequences of length P plus the
    // twiddles in LDS: (S + 1) P 16 bytes <= 160 KB, so P <= 4096
    if (n < 1 || fft_len(n) > 4096) {
      set_error("n must be in [1, 2047] in 2D (FFT length at most 4096)");
      return LS_E_INVALID;
    }
    std::vector<double> mh((size_t)n * n);
    LSW_HIP_TRY(hipMemcpy(mh.data(), m_dev, mh.size() * sizeof(double), hipMemcpyDeviceToHost));
    const std::string err = build_host_setup(mh.data(), n, omega, pml_width, layer_thickness, o.pml_C,
                                             o.freq_samples, h->H, o.fronts);
    if (!err.empty()) {
      set_error(err);
      return LS_E_INVALID;
    }
    h->n = n;
    h->b = pml_width;
    h->w = layer_thickness;
    h->L = h->H.L;
    h->P = fft_len(n);
    h->ns = h->H.ns;
    h->nslices = h->H.nslices;
    h->omega = omega;
    h->prec = o.precision;
    set_default_choices(h.get());
    h->N = (size_t)n * n;
    h->E = (size_t)h->L * h->L;
    ls_status e = device_setup(h.get(), m_dev);
    if (e != LS_OK) return e;
    {
      // the allocation-free apply's scratch address on this device
      void* ws = nullptr;
      if ((e = scratch_for_device(h->device, &ws)) != LS_OK) return e;
    }
    if (o.autotune > 0) {
      e = h->prec == LS_FP64 ? tune_kernels<double>(h.get(), o.autotune) : tune_kernels<float>(h.get(), o.autotune);
      if (e != LS_OK) return e;
    }
    *out = h.release();
    return LS_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return LS_E_NOMEM;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

void ls_destroy(ls_handle* h) { delete h; }

ls_status ls_solve(ls_handle* h, const void* rhs_dev, int nrhs, int rhs_kind, double tol, void* u_dev,
                   ls_rhs_info* info_host) {
  try {
    if (check_handle(h) != LS_OK) return LS_E_INVALID;
    if (nrhs < 1 || !rhs_dev || !u_dev || !(tol > 0.0) || !std::isfinite(tol) ||
        (rhs_kind != LS_RHS_SOURCE && rhs_kind != LS_RHS_INCIDENT)) {
      set_error("ls_solve: bad argument (nrhs >= 1, non-null arrays, tol > 0, rhs_kind)");
      return LS_E_INVALID;
    }
    ls_status e = ensure_workspace(h, nrhs);
    if (e != LS_OK) return e;
    const size_t N = h->N;
    double2* G = h->G.as<double2>();
    if (rhs_kind == LS_RHS_INCIDENT) {
      // g = -omega^2 K (m u_I)
      e = convolve_any<double>(h, static_cast<const double2*>(rhs_dev), true, nrhs, 0.0, -h->omega * h->omega, G);
      if (e != LS_OK) return e;
    } else {
      LSW_HIP_TRY(hipMemcpyAsync(G, rhs_dev, (size_t)nrhs * N * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
    }
    std::vector<ls_rhs_info> info;
    h->last_nrhs = 0;
    const ls_status gs = run_gmres(h, nrhs, tol, info);
    if (gs != LS_OK && gs != LS_E_NOCONV) return gs;
    // u, and the total field psi = u + u_I (incident) or u (source) kept for
    // ls_adjoint, in one pass over the solution
    LSW_ALLOC(h->psi, (size_t)nrhs * N * sizeof(double2));
    LSW_HIP_TRY(launch_solution_out(static_cast<double2*>(u_dev), h->psi.as<double2>(), h->X.as<double2>(),
                                    rhs_kind == LS_RHS_INCIDENT ? static_cast<const double2*>(rhs_dev) : nullptr,
                                    (size_t)nrhs * N, h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    h->last_nrhs = nrhs;
    if (info_host)
      for (int r = 0; r < nrhs; ++r) info_host[r] = info[r];
    return gs;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return LS_E_NOMEM;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

ls_status ls_adjoint(ls_handle* h, const void* resid_dev, int nrhs, double tol, double* grad_dev,
                     ls_rhs_info* info_host) {
  try {
    if (check_handle(h) != LS_OK) return LS_E_INVALID;
    if (h->last_nrhs == 0 || nrhs != h->last_nrhs) {
      set_error("ls_adjoint needs a preceding ls_solve with the same nrhs");
      return LS_E_STATE;
    }
    if (!resid_dev || !grad_dev || !(tol > 0.0)) {
      set_error("ls_adjoint: bad argument");
      return LS_E_INVALID;
    }
    const size_t N = h->N;
    // b_j = K conj(r_j)
    double2* T1 = h->T1.as<double2>();
    LSW_HIP_TRY(launch_conj(T1, static_cast<const double2*>(resid_dev), (size_t)nrhs * N, h->st));
    ls_status e = convolve_any<double>(h, T1, false, nrhs, 0.0, 1.0, h->G.as<double2>());
    if (e != LS_OK) return e;
    std::vector<ls_rhs_info> info;
    const ls_status gs = run_gmres(h, nrhs, tol, info);
    if (gs != LS_OK && gs != LS_E_NOCONV) return gs;
    LSW_HIP_TRY(launch_adjoint_product(h->psi.as<double2>(), h->X.as<double2>(), nrhs, N, h->omega * h->omega,
                                       grad_dev, h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    if (info_host)
      for (int r = 0; r < nrhs; ++r) info_host[r] = info[r];
    return gs;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

ls_status ls_apply_A(ls_handle* h, const void* x, int nrhs, void* y, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !x || !y) {
    set_error("ls_apply_A: bad argument");
    return LS_E_INVALID;
  }
  ls_status e = ensure_workspace(h, nrhs);
  if (e != LS_OK) return e;
  e = precision == LS_FP64
          ? apply_A<double>(h, static_cast<const double2*>(x), nrhs, static_cast<double2*>(y))
          : apply_A<float>(h, static_cast<const float2*>(x), nrhs, static_cast<float2*>(y));
  if (e != LS_OK) return e;
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_apply_A_noalloc(ls_handle* h, const void* x, int nrhs, void* y, int precision) {
  try {
    if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
    if (h->dim != 2) {
      set_error("ls_apply_A_noalloc: 2D handles only");
      return LS_E_INVALID;
    }
    if (nrhs < 1 || !x || !y) {
      set_error("ls_apply_A_noalloc: bad argument");
      return LS_E_INVALID;
    }
    const size_t cs = precision == LS_FP64 ? sizeof(double2) : sizeof(float2);
    const size_t per_rhs = fft_work_elems<double>(h->n, 1) * cs;
    if ((size_t)nrhs * per_rhs > kNoAllocScratchBytes) {
      set_error("ls_apply_A_noalloc: " + std::to_string(nrhs) + " right-hand sides need " +
                std::to_string((size_t)nrhs * per_rhs) + " bytes of FFT work; the static scratch holds " +
                std::to_string(kNoAllocScratchBytes) + " bytes, so at most " +
                std::to_string(kNoAllocScratchBytes / per_rhs) + " at n = " + std::to_string(h->n) +
                " in this precision (use ls_apply_A, which allocates)");
      return LS_E_INVALID;
    }
    void* ws = nullptr;
    ls_status e = scratch_for_device(h->device, &ws);
    if (e != LS_OK) return e;
    // every value of the work array that the column and inverse passes read is
    // written first by the forward row pass, so nothing needs clearing
    if (precision == LS_FP64) {
      LSW_HIP_TRY(launch_convolve<double>(static_cast<const double2*>(x), Prec<double>::m(h), h->n, nrhs,
                                          Prec<double>::khat(h), Prec<double>::tw(h), 1.0, h->omega * h->omega,
                                          static_cast<double2*>(ws), static_cast<double2*>(y), h->st));
    } else {
      LSW_HIP_TRY(launch_convolve<float>(static_cast<const float2*>(x), Prec<float>::m(h), h->n, nrhs,
                                         Prec<float>::khat(h), Prec<float>::tw(h), 1.0f,
                                         (float)(h->omega * h->omega), static_cast<float2*>(ws),
                                         static_cast<float2*>(y), h->st));
    }
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    return LS_OK;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

ls_status ls_apply_K(ls_handle* h, const void* x, int nrhs, void* y, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !x || !y) {
    set_error("ls_apply_K: bad argument");
    return LS_E_INVALID;
  }
  ls_status e = ensure_workspace(h, nrhs);
  if (e != LS_OK) return e;
  e = precision == LS_FP64
          ? convolve_any<double>(h, static_cast<const double2*>(x), false, nrhs, 0.0, 1.0, static_cast<double2*>(y))
          : convolve_any<float>(h, static_cast<const float2*>(x), false, nrhs, 0.0f, 1.0f, static_cast<float2*>(y));
  if (e != LS_OK) return e;
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_apply_Q(ls_handle* h, const void* r, int nrhs, void* f, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !r || !f) {
    set_error("ls_apply_Q: bad argument");
    return LS_E_INVALID;
  }
  if (h->dim == 3) {
    const Stencil3 S3 = stencil3(h);
    if (precision == LS_FP64)
      LSW_HIP_TRY(launch3_apply_Q<double>(S3, static_cast<const double2*>(r), nrhs, static_cast<double2*>(f), h->st));
    else
      LSW_HIP_TRY(launch3_apply_Q<float>(S3, static_cast<const float2*>(r), nrhs, static_cast<float2*>(f), h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    return LS_OK;
  }
  const StencilTables S = h->stencils();
  if (precision == LS_FP64)
    LSW_HIP_TRY(launch_apply_Q<double>(S, static_cast<const double2*>(r), nrhs, static_cast<double2*>(f), false,
                                       h->st));
  else
    LSW_HIP_TRY(launch_apply_Q<float>(S, static_cast<const float2*>(r), nrhs, static_cast<float2*>(f), false,
                                      h->st));
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_apply_B(ls_handle* h, const void* f, int nrhs, void* b, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
  if (h->dim != 2 || nrhs < 1 || !f || !b) {
    set_error("ls_apply_B: bad argument (2D handle, nrhs >= 1, non-null arrays)");
    return LS_E_INVALID;
  }
  // the Q stencil's kernel with beta in place of alpha
  StencilTables S = h->stencils();
  S.alpha = S.beta;
  if (precision == LS_FP64)
    LSW_HIP_TRY(launch_apply_Q<double>(S, static_cast<const double2*>(f), nrhs, static_cast<double2*>(b), false, h->st));
  else
    LSW_HIP_TRY(launch_apply_Q<float>(S, static_cast<const float2*>(f), nrhs, static_cast<float2*>(b), false, h->st));
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_solve_H(ls_handle* h, const void* rhs_dev, int nrhs, double tol, void* u_dev, ls_rhs_info* info_host) {
  try {
    if (check_handle(h) != LS_OK) return LS_E_INVALID;
    if (h->dim != 2 || nrhs < 1 || !rhs_dev || !u_dev || !(tol > 0.0) || !std::isfinite(tol)) {
      set_error("ls_solve_H: bad argument (2D handle, nrhs >= 1, non-null arrays, tol > 0)");
      return LS_E_INVALID;
    }
    // the Krylov loop on extended-grid vectors: its workspaces are sized for
    // E values per right-hand side for this call; afterwards the handle is
    // back on the interior grid (the larger buffers are kept)
    struct Restore {
      ls_handle* h;
      size_t N;
      ~Restore() {
        h->N = N;
        h->hmode = false;
        h->cap = 0;
      }
    } restore{h, h->N};
    h->last_nrhs = 0;
    h->N = h->E;
    h->cap = 0;
    ls_status e = ensure_workspace(h, nrhs);
    if (e != LS_OK) return e;
    const size_t E = h->E;
    LSW_HIP_TRY(hipMemcpyAsync(h->G.p, rhs_dev, (size_t)nrhs * E * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
    h->hmode = true;
    std::vector<ls_rhs_info> info;
    const ls_status gs = run_gmres(h, nrhs, tol, info);
    if (gs != LS_OK && gs != LS_E_NOCONV) return gs;
    LSW_HIP_TRY(hipMemcpyAsync(u_dev, h->X.p, (size_t)nrhs * E * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    if (info_host)
      for (int r = 0; r < nrhs; ++r) info_host[r] = info[r];
    return gs;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return LS_E_NOMEM;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

ls_status ls_apply_H(ls_handle* h, const void* u, int nrhs, void* y, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, false) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !u || !y) {
    set_error("ls_apply_H: bad argument");
    return LS_E_INVALID;
  }
  if (h->dim == 3) {
    const Stencil3 S3 = stencil3(h);
    if (precision == LS_FP64)
      LSW_HIP_TRY(launch3_apply_H<double>(S3, static_cast<const double2*>(u), nrhs, static_cast<double2*>(y), h->st));
    else
      LSW_HIP_TRY(launch3_apply_H<float>(S3, static_cast<const float2*>(u), nrhs, static_cast<float2*>(y), h->st));
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    return LS_OK;
  }
  const StencilTables S = h->stencils();
  if (precision == LS_FP64)
    LSW_HIP_TRY(launch_apply_H<double>(S, static_cast<const double2*>(u), nrhs, static_cast<double2*>(y), h->st));
  else
    LSW_HIP_TRY(launch_apply_H<float>(S, static_cast<const float2*>(u), nrhs, static_cast<float2*>(y), h->st));
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_apply_precond(ls_handle* h, const void* r, int nrhs, void* z, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, true) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !r || !z) {
    set_error("ls_apply_precond: bad argument");
    return LS_E_INVALID;
  }
  ls_status e = ensure_workspace(h, nrhs);
  if (e != LS_OK) return e;
  e = precision == LS_FP64 ? apply_P<double>(h, static_cast<const double2*>(r), nrhs, static_cast<double2*>(z))
                           : apply_P<float>(h, static_cast<const float2*>(r), nrhs, static_cast<float2*>(z));
  if (e != LS_OK) return e;
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_slice_solve(ls_handle* h, int slice, const void* v, int nrhs, void* w, int precision) {
  if (check_handle(h) != LS_OK || check_precision(h, precision, true) != LS_OK) return LS_E_INVALID;
  if (nrhs < 1 || !v || !w || slice < 0 || slice >= h->nslices) {
    set_error("ls_slice_solve: bad argument");
    return LS_E_INVALID;
  }
  ls_status e = ensure_workspace(h, nrhs);
  if (e != LS_OK) return e;
  if (h->dim == 3) {
    auto run3 = [&](auto tag) -> ls_status {
      using T = decltype(tag);
      const Slab3& p = h->s3->slabs[slice];
      const size_t rs = (size_t)(p.hi - p.lo + 1) * h->L * h->L;
      Slab3Apply<T> a = slab3_args<T>(h, slice, nrhs);
      a.src = static_cast<const C<T>*>(v);
      a.src_rs = rs;
      a.dst = static_cast<C<T>*>(w);
      a.dst_rs = rs;
      LSW_HIP_TRY(launch3_slab_solve<T>(a, h->st));
      return LS_OK;
    };
    e = precision == LS_FP64 ? run3(double{}) : run3(float{});
    if (e != LS_OK) return e;
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    return LS_OK;
  }
  const KernelChoice kc = choice_for(h, nrhs);
  if (kc.slice == 16 && (e = ensure_mscr(h, nrhs)) != LS_OK) return e;
  auto run = [&](auto tag) -> ls_status {
    using T = decltype(tag);
    SliceSolveArgs<T> a = slice_args<T>(h);
    a.nrhs = nrhs;
    a.yscr = h->sscr.as<C<T>>();
    a.mfma_scr = h->mscr.as<T>();
    a.src_kind = kSrcSlice;
    a.src = static_cast<const C<T>*>(v);
    a.dst_kind = kDstSlice;
    a.dst = static_cast<C<T>*>(w);
    const int k = h->tbl_of_grid[slice];  // slices are numbered in grid order here
    return solve_slices<T>(h, a, k, k + 1, kc.slice);
  };
  e = precision == LS_FP64 ? run(double{}) : run(float{});
  if (e != LS_OK) return e;
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}

ls_status ls_get_info(const ls_handle* h, ls_setup_info* o) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (!o) {
    set_error("info must not be NULL");
    return LS_E_INVALID;
  }
  o->dim = h->dim;
  o->n = h->n;
  o->pml_width = h->b;
  o->layer_thickness = h->w;
  o->L = h->L;
  o->nslices = h->nslices;
  o->freq_samples = h->ns;
  o->precision = h->prec;
  o->omega = h->omega;
  o->h = h->H.h;
  o->pml_C = h->H.C;
  o->freq_lo = h->H.freq_lo;
  o->freq_delta = h->H.freq_delta;
  o->fronts = h->dim == 2 ? h->H.fronts : 1;
  return LS_OK;
}

ls_status ls_layer_candidates(int n, int pml_width, int* out_host, int cap, int* count) {
  if (n < 1 || pml_width < 1 || cap < 0 || (cap > 0 && !out_host) || !count) {
    set_error("ls_layer_candidates: bad argument (n >= 1, pml_width >= 1, cap >= 0, count not NULL)");
    return LS_E_INVALID;
  }
  const std::vector<int> c = layer_candidates(n, pml_width);
  for (int i = 0; i < (int)c.size() && i < cap; ++i) out_host[i] = c[i];
  *count = (int)c.size();
  return LS_OK;
}

ls_status ls_get_tuning(const ls_handle* h, ls_tune_layer* w_host, int wcap, int* nw, ls_tune_kernels* k_host,
                        int kcap, int* nk) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (wcap < 0 || kcap < 0 || (wcap > 0 && !w_host) || (kcap > 0 && !k_host)) {
    set_error("ls_get_tuning: bad argument");
    return LS_E_INVALID;
  }
  for (int i = 0; i < (int)h->tune_w.size() && i < wcap; ++i) w_host[i] = h->tune_w[i];
  for (int i = 0; i < (int)h->tune_k.size() && i < kcap; ++i) k_host[i] = h->tune_k[i];
  if (nw) *nw = (int)h->tune_w.size();
  if (nk) *nk = (int)h->tune_k.size();
  return LS_OK;
}

ls_status ls_set_kernels(ls_handle* h, int nrhs, int slice_kernel, int iface_kernel) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (h->dim == 3) {
    set_error("ls_set_kernels: the 2D slice and interface kernels only");
    return LS_E_INVALID;
  }
  if (nrhs < 0 || nrhs > kChoiceMax) {
    set_error("ls_set_kernels: 0 <= nrhs <= 256");
    return LS_E_INVALID;
  }
  if (slice_kernel == 0) {  // back to the defaults
    const bool fp64 = h->prec == LS_FP64;
    if (nrhs == 0)
      set_default_choices(h);
    else
      h->choice[nrhs] = default_choice(nrhs, fp64);
    return LS_OK;
  }
  const bool sk_ok = slice_kernel == 1 || slice_kernel == 4 || slice_kernel == 8 || slice_kernel == 16;
  if (!sk_ok || iface_kernel < 0 || iface_kernel > 1 || (iface_kernel == 0 && nrhs > 4)) {
    set_error("ls_set_kernels: slice_kernel in {0, 1, 4, 8, 16}, iface_kernel 0 (nrhs <= 4) or 1");
    return LS_E_INVALID;
  }
  if (nrhs == 0) {
    for (int nb = 0; nb <= kChoiceMax; ++nb)
      h->choice[nb] = {slice_kernel, nb > 4 && iface_kernel == 0 ? 1 : iface_kernel};
  } else {
    h->choice[nrhs] = {slice_kernel, iface_kernel};
  }
  return LS_OK;
}

ls_status ls_get_slice(const ls_handle* h, int slice, int* first_line, int* last_line, int* aux_lines) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (slice < 0 || slice >= h->nslices) {
    set_error("slice out of range");
    return LS_E_INVALID;
  }
  const SlicePlan& p = h->dim == 2 ? h->H.slices[h->tbl_of_grid[slice]] : h->H.slices[slice];
  if (first_line) *first_line = p.lo;
  if (last_line) *last_line = p.hi;
  if (aux_lines) *aux_lines = p.naux + p.nauxr;
  return LS_OK;
}

ls_status ls_get_stencils(const ls_handle* h, double* alpha, double* beta, double* gamma, double* aux) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  auto put = [](double* dst, const cd* src, size_t count) {
    for (size_t i = 0; i < count; ++i) {
      dst[2 * i] = src[i].real();
      dst[2 * i + 1] = src[i].imag();
    }
  };
  if (h->dim == 3) {
    const HostSetup3& H3 = h->s3->H;
    if (alpha) put(alpha, H3.alpha, 27);
    if (beta) put(beta, H3.beta, 27);
    if (gamma) put(gamma, H3.gamma_glob.data(), H3.gamma_glob.size());
    if (aux) put(aux, H3.gamma_aux.data(), H3.gamma_aux.size());
    return LS_OK;
  }
  if (alpha) put(alpha, h->H.alpha, 9);
  if (beta) put(beta, h->H.beta, 9);
  if (gamma) put(gamma, h->H.gamma_glob.data(), h->H.gamma_glob.size());
  if (aux) put(aux, h->H.gamma_aux.data(), h->H.gamma_aux.size());
  return LS_OK;
}

ls_status ls_get_sample_map(const ls_handle* h, int* kmap) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (!kmap) {
    set_error("kmap must not be NULL");
    return LS_E_INVALID;
  }
  const std::vector<int>& km = h->dim == 3 ? h->s3->H.kmap : h->H.kmap;
  std::copy(km.begin(), km.end(), kmap);
  return LS_OK;
}

ls_status ls_profile(ls_handle* h, int enable) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (enable) {
    LSW_HIP_TRY(hipStreamSynchronize(h->st));
    for (auto& r : h->recs) {
      h->pool.push_back(r.a);
      h->pool.push_back(r.b);
    }
    h->recs.clear();
  }
  h->profiling = enable != 0;
  return LS_OK;
}

ls_status ls_profile_read(ls_handle* h, ls_kernel_time* out, int max, int* count) {
  if (check_handle(h) != LS_OK) return LS_E_INVALID;
  if (!out || !count) {
    set_error("out and count must not be NULL");
    return LS_E_INVALID;
  }
  int launches[kKNumKinds] = {};
  double ms[kKNumKinds] = {};
  long long cols[kKNumKinds] = {};
  for (auto& r : h->recs) {
    LSW_HIP_TRY(hipEventSynchronize(r.b));
    float t = 0.f;
    LSW_HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    launches[r.kind] += 1;
    ms[r.kind] += t;
    cols[r.kind] += r.cols;
  }
  int c = 0;
  for (int k = 0; k < kKNumKinds && c < max; ++k) {
    if (!launches[k]) continue;
    std::snprintf(out[c].name, sizeof out[c].name, "%s", kKindNames[k]);
    out[c].launches = launches[k];
    out[c].total_ms = ms[k];
    out[c].columns = cols[k];
    ++c;
  }
  *count = c;
  return LS_OK;
}

ls_status ls_host_green3(int n, double omega, double* green_host) {
  try {
    set_error("");
    if (n < 1 || n > 1023 || !(omega > 0.0) || !std::isfinite(omega) || !green_host) {
      set_error("ls_host_green3: 1 <= n <= 1023, omega > 0, green_host not NULL");
      return LS_E_INVALID;
    }
    const std::vector<cd> kq = green3_octant(n, omega);
    for (size_t i = 0; i < kq.size(); ++i) {
      green_host[2 * i] = kq[i].real();
      green_host[2 * i + 1] = kq[i].imag();
    }
    return LS_OK;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_NOMEM;
  }
}

ls_status ls_op3_create(int n, double omega, const double* m_dev, void* hip_stream, ls_op3** out) {
  try {
    set_error("");
    if (!out) {
      set_error("out must not be NULL");
      return LS_E_INVALID;
    }
    *out = nullptr;
    if (n < 1 || n > 1023 || !(omega > 0.0) || !std::isfinite(omega) || !m_dev) {
      set_error("ls_op3_create: 1 <= n <= 1023, omega > 0, m_dev not NULL");
      return LS_E_INVALID;
    }
    std::unique_ptr<ls_op3> h(new ls_op3());
    LSW_HIP_TRY(hipGetDevice(&h->device));
    h->st = static_cast<hipStream_t>(hip_stream);
    h->n = n;
    h->P = fft_len(n);
    h->omega = omega;
    const int P = h->P;
    const size_t n3 = (size_t)n * n * n;
    hipStream_t st = h->st;
    std::vector<double> mh(n3);
    LSW_HIP_TRY(hipMemcpy(mh.data(), m_dev, n3 * sizeof(double), hipMemcpyDeviceToHost));
    for (double v : mh)
      if (!std::isfinite(v) || v >= 1.0) {
        set_error("m must be finite and < 1 everywhere");
        return LS_E_INVALID;
      }
    std::vector<float> m32(n3);
    for (size_t i = 0; i < n3; ++i) m32[i] = (float)mh[i];
    LSW_ALLOC(h->m, n3 * sizeof(double));
    LSW_ALLOC(h->m32, n3 * sizeof(float));
    LSW_HIP_TRY(hipMemcpyAsync(h->m.p, m_dev, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    LSW_HIP_TRY(hipMemcpyAsync(h->m32.p, m32.data(), n3 * sizeof(float), hipMemcpyHostToDevice, st));
    std::vector<double2> tw(P);
    std::vector<float2> tw32(P);
    for (int k = 0; k < P; ++k) {
      const double a = -2.0 * M_PI * (double)k / (double)P;
      tw[k] = make_double2(std::cos(a), std::sin(a));
      tw32[k] = make_float2((float)tw[k].x, (float)tw[k].y);
    }
    LSW_ALLOC(h->tw, P * sizeof(double2));
    LSW_ALLOC(h->tw32, P * sizeof(float2));
    LSW_HIP_TRY(hipMemcpyAsync(h->tw.p, tw.data(), P * sizeof(double2), hipMemcpyHostToDevice, st));
    LSW_HIP_TRY(hipMemcpyAsync(h->tw32.p, tw32.data(), P * sizeof(float2), hipMemcpyHostToDevice, st));
    {
      const std::vector<cd> kq = green3_octant(n, omega);
      std::vector<double2> kq_h(kq.size());
      for (size_t i = 0; i < kq.size(); ++i) kq_h[i] = make_double2(kq[i].real(), kq[i].imag());
      DBuf kqd, scratch;
      LSW_ALLOC(kqd, kq_h.size() * sizeof(double2));
      LSW_ALLOC(scratch, (size_t)P * P * P * sizeof(double2));
      const size_t H = P / 2 + 1;
      LSW_ALLOC(h->khat, H * H * H * sizeof(double2));
      LSW_ALLOC(h->khat32, H * H * H * sizeof(float2));
      LSW_HIP_TRY(hipMemcpyAsync(kqd.p, kq_h.data(), kq_h.size() * sizeof(double2), hipMemcpyHostToDevice, st));
      LSW_HIP_TRY(launch_green_spectrum3(kqd.as<double2>(), n, h->tw.as<double2>(), scratch.as<double2>(),
                                         h->khat.as<double2>(), h->khat32.as<float2>(), st));
      LSW_HIP_TRY(hipStreamSynchronize(st));
    }
    *out = h.release();
    return LS_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return LS_E_NOMEM;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_INVALID;
  }
}

namespace {
// y = a x + c K (s .* x) for the 3D operator; s = m (with_m) or 1
ls_status op3_apply(ls_op3* h, const void* x, int nrhs, void* y, int precision, bool with_m, double a, double c) {
  if (!h) {
    set_error("null handle");
    return LS_E_INVALID;
  }
  if (nrhs < 1 || !x || !y || (precision != LS_FP64 && precision != LS_MIXED)) {
    set_error("ls_op3_apply: nrhs >= 1, non-null arrays, precision LS_FP64 or LS_MIXED");
    return LS_E_INVALID;
  }
  if (nrhs > h->cap) {
    // sized for complex128 so that either precision fits; a failed growth
    // may have released the old arrays, so the handle then holds none
    h->cap = 0;
    LSW_ALLOC(h->w1, (size_t)nrhs * fft3_w1_elems(h->n) * sizeof(double2));
    LSW_ALLOC(h->w2, (size_t)nrhs * fft3_w2_elems(h->n) * sizeof(double2));
    h->cap = nrhs;
  }
  if (precision == LS_FP64) {
    LSW_HIP_TRY(launch_convolve3<double>(static_cast<const double2*>(x), with_m ? h->m.as<double>() : nullptr, h->n,
                                         nrhs, h->khat.as<double2>(), h->tw.as<double2>(), a, c, h->w1.as<double2>(),
                                         h->w2.as<double2>(), static_cast<double2*>(y), h->st));
  } else {
    LSW_HIP_TRY(launch_convolve3<float>(static_cast<const float2*>(x), with_m ? h->m32.as<float>() : nullptr, h->n,
                                        nrhs, h->khat32.as<float2>(), h->tw32.as<float2>(), (float)a, (float)c,
                                        h->w1.as<float2>(), h->w2.as<float2>(), static_cast<float2*>(y), h->st));
  }
  LSW_HIP_TRY(hipStreamSynchronize(h->st));
  return LS_OK;
}
}  // namespace

ls_status ls_op3_apply_A(ls_op3* h, const void* x_dev, int nrhs, void* y_dev, int precision) {
  return op3_apply(h, x_dev, nrhs, y_dev, precision, true, 1.0, h ? h->omega * h->omega : 0.0);
}

ls_status ls_op3_apply_K(ls_op3* h, const void* x_dev, int nrhs, void* y_dev, int precision) {
  return op3_apply(h, x_dev, nrhs, y_dev, precision, false, 0.0, 1.0);
}

void ls_op3_destroy(ls_op3* h) { delete h; }

ls_status ls_stencil_cache(int clear, long long* hits, long long* misses) {
  lsw::stencil_cache(clear != 0, hits, misses);
  return LS_OK;
}

ls_status ls_host_tables(int n, double omega, const double* m_host, int pml_width, int layer_thickness,
                         double pml_C, int freq_samples, double* alpha, double* beta, double* gamma, double* aux,
                         int* kmap, double* green) {
  try {
    set_error("");
    if (!m_host) {
      set_error("m_host must not be NULL");
      return LS_E_INVALID;
    }
    HostSetup Hs;
    const std::string err = build_host_setup(m_host, n, omega, pml_width, layer_thickness, pml_C, freq_samples, Hs);
    if (!err.empty()) {
      set_error(err);
      return LS_E_INVALID;
    }
    auto put = [](double* dst, const cd* src, size_t count) {
      for (size_t i = 0; i < count; ++i) {
        dst[2 * i] = src[i].real();
        dst[2 * i + 1] = src[i].imag();
      }
    };
    if (alpha) put(alpha, Hs.alpha, 9);
    if (beta) put(beta, Hs.beta, 9);
    if (gamma) put(gamma, Hs.gamma_glob.data(), Hs.gamma_glob.size());
    if (aux) put(aux, Hs.gamma_aux.data(), Hs.gamma_aux.size());
    if (kmap) std::copy(Hs.kmap.begin(), Hs.kmap.end(), kmap);
    if (green) put(green, Hs.kq.data(), Hs.kq.size());
    return LS_OK;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_NOMEM;
  }
}

ls_status ls_host_tables3(int n, double omega, const double* m_host, int pml_width, int layer_thickness,
                          double pml_C, int freq_samples, double* alpha, double* beta, double* gamma, double* aux,
                          int* kmap) {
  try {
    set_error("");
    if (!m_host) {
      set_error("m_host must not be NULL");
      return LS_E_INVALID;
    }
    HostSetup3 Hs;
    const std::string err = build_host_setup3(m_host, n, omega, pml_width, layer_thickness, pml_C, freq_samples,
                                              kSlab3MaxLines, kSlab3MaxBlock, Hs);
    if (!err.empty()) {
      set_error(err);
      return LS_E_INVALID;
    }
    auto put = [](double* dst, const cd* src, size_t count) {
      for (size_t i = 0; i < count; ++i) {
        dst[2 * i] = src[i].real();
        dst[2 * i + 1] = src[i].imag();
      }
    };
    if (alpha) put(alpha, Hs.alpha, 27);
    if (beta) put(beta, Hs.beta, 27);
    if (gamma) put(gamma, Hs.gamma_glob.data(), Hs.gamma_glob.size());
    if (aux) put(aux, Hs.gamma_aux.data(), Hs.gamma_aux.size());
    if (kmap) std::copy(Hs.kmap.begin(), Hs.kmap.end(), kmap);
    return LS_OK;
  } catch (const std::exception& ex) {
    set_error(ex.what());
    return LS_E_NOMEM;
  }
}

}  // extern "C"
