/*
 * lsweep: sparsify-and-sweep preconditioned GMRES for the discretized
 * Lippmann-Schwinger equation on AMD MI355X (gfx950).
 *
 * Method: F. Liu and L. Ying, "Sparsify and sweep: an efficient
 * preconditioner for the Lippmann-Schwinger equation".
 *
 * Problem (Sec. 1, eq. LS; Sec. 2.1, eqs. LS_d and LS_d_c): on the unit square
 * with n interior points per axis (h = 1/(n+1)), find u on the interior grid I
 * with
 *     u_i + omega^2 sum_{j in I} k_{i-j} m_j u_j = g_i,
 *     g_i = -omega^2 sum_{j in I} k_{i-j} m_j [u_I]_j,
 * where k_delta = G(|delta| h) h^2 for delta != 0 (G the free-space Green's
 * function) and k_0 is the integral of G over the disk of area h^2.
 * The solver is right-preconditioned restarted GMRES; the preconditioner is
 * the sparsified system H (Sec. 2.2) inverted approximately by the
 * moving-PML sweep (Sec. 2.3, Algorithms 1 and 2).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers on the handle's device unless a
 *    parameter name ends in _host.
 *  - Arrays are C-ordered; a grid array is [i1][i2] with i2 fastest; i1 is the
 *    sweep axis. Interior arrays are [n][n], extended-grid arrays are [L][L]
 *    with L = n + 2 + 2b and extended index e = i + b (i in [-b, n+1+b]).
 *  - A batch is [nrhs][grid]. Complex values are interleaved (re, im):
 *    complex128 (double2) when a precision argument is LS_FP64, complex64
 *    (float2) when it is LS_MIXED.
 *  - The caller owns every array it passes; the library copies what it keeps.
 *  - Every call returns an ls_status; ls_last_error() gives a message for the
 *    last failure on the calling thread. No C++ exception crosses this ABI.
 *  - Work is enqueued on opts.hip_stream (NULL: the default stream); every
 *    entry point returns with its work complete (host-synchronised).
 *  - Calls on one handle must not overlap.
 *  - ls_setup takes dim = 2 (Sec. 2) or dim = 3 (Sec. 3.1); other values
 *    return LS_E_INVALID. In 3D every grid array gains a third axis
 *    ([n][n][n] interior, [L][L][L] extended) and the whole solver, the
 *    sweeping preconditioner included, works on it (see ls_setup). The 3D
 *    operator alone also has a handle of its own (ls_op3, below).
 */
#ifndef LSWEEP_H
#define LSWEEP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_handle ls_handle;

typedef enum {
  LS_OK = 0,
  LS_E_INVALID = 1,   /* bad argument (dim, n, omega, b, w, m not finite or m >= 1, ...) */
  LS_E_NOMEM = 2,     /* a device or host allocation failed */
  LS_E_DEVICE = 3,    /* a HIP runtime call failed */
  LS_E_SINGULAR = 4,  /* zero pivot in a slice factorization */
  LS_E_NOCONV = 5,    /* max_iters reached; the best iterate and info are still written */
  LS_E_NUMERIC = 6,   /* NaN or Inf met in a norm */
  LS_E_STATE = 7      /* call out of order (ls_adjoint without a matching ls_solve) */
} ls_status;

typedef enum { LS_FP64 = 0, LS_MIXED = 1 } ls_precision;
typedef enum { LS_RHS_SOURCE = 0, LS_RHS_INCIDENT = 1 } ls_rhs_kind;

typedef struct {
  int dim;  /* 2 (unit square) or 3 (unit cube) */
  int n;    /* interior points per axis, h = 1/(n+1) */
} ls_grid;

typedef struct {
  int precision;     /* ls_precision. LS_FP64: every apply in complex128.
                        LS_MIXED: FFT, stencil, slice factors and sweep in
                        complex64 inside a complex128 flexible GMRES loop. */
  int restart;       /* GMRES restart length (default 30) */
  int max_iters;     /* total Arnoldi steps per right-hand side (default 1000) */
  double pml_C;      /* PML strength C of Sec. 2.2.2 (default 10) */
  int freq_samples;  /* local-frequency samples for the auxiliary PML (0: n, Sec. 2.3) */
  int autotune;      /* 0: no tuning. k > 0: tune for batches of k right-hand sides
                        (ls_setup: the layer thickness when layer_thickness <= 0, and the
                        kernel choice per batch size; see "Autotuning" below) */
  void* hip_stream;  /* hipStream_t to enqueue on (NULL: default stream) */
  int sweep_schedule;  /* LS_SWEEP_INTERFACE (default): all slice solves at once plus the
                          interface recurrences; LS_SWEEP_SEQUENTIAL: Algorithm 2 slice by slice.
                          Both compute the same preconditioner up to rounding. */
  int fronts;          /* 1 (default): one sweeping front along x1 (Algorithms 1-2).
                          2: two fronts (the first remark after Algorithm 2, Sec. 2.4):
                          p = floor((n+1)/(2w)) slices of w lines swept from each end toward a
                          middle slice of the remaining 1..2w lines, which carries auxiliary
                          PML on both sides and is eliminated last; each front's slices take
                          their auxiliary PML on the side of the front's earlier slices.
                          A different preconditioner (iteration counts differ). 2D with the
                          interface schedule only; LS_E_INVALID otherwise. */
  int block_size;      /* 1 (default): GMRES per right-hand side (every column its own
                          Krylov space). B in [2, 64]: block flexible GMRES, consecutive groups
                          of B columns (the last may be smaller) each sharing one block Krylov
                          space (Cholesky QR twice for the block QR, the Gram products as
                          matrix-core GEMMs); restart then counts block
                          steps per cycle and max_iters block steps (ls_rhs_info.iterations: the
                          block steps taken while the column was in its block). A column leaves
                          its block at a restart once its true residual meets tol; a zero
                          right-hand side never enters it. Linearly dependent right-hand sides
                          in a block fall back to the per-column loop. Needs
                          block_size * restart <= 2048. Same u to the tolerance, different
                          iterates and counts. */
} ls_options;

typedef enum { LS_SWEEP_INTERFACE = 0, LS_SWEEP_SEQUENTIAL = 1 } ls_sweep_schedule;

typedef struct {
  int iterations;       /* Arnoldi steps over all restart cycles */
  double rel_residual;  /* true ||g - A u||_2 / ||g||_2, in float64 */
  int converged;        /* 1 if rel_residual <= tol */
} ls_rhs_info;

/* Fill *opts with the defaults listed above. */
void ls_default_options(ls_options* opts);

/*
 * Algorithm 1 (setup). Builds the Green's-function table and its FFT, the
 * type-1 stencils alpha and beta (eqs. alpha, beta), the PML stencils gamma
 * (eq. gamma) for the global PML and for the auxiliary PML at the sampled
 * local frequencies, slices the extended grid along i1 into floor((n+2)/w)
 * slices, and factors every moving-PML slice subproblem (eq. Hwv_approx).
 *   grid             dim and n; in 2D 1 <= n <= 2047 (the zero-padded FFT
 *                    length P = 2^k >= 2(n+1) is at most 4096: one complex128
 *                    sequence of length P and its twiddles fill the LDS of a
 *                    compute unit), LS_E_INVALID otherwise
 *   omega            angular frequency, > 0
 *   m_dev            float64 [n][n] perturbation m = 1 - 1/c^2 on the interior grid;
 *                    every value finite and < 1
 *   pml_width        b >= 1, PML width in cells (global and auxiliary)
 *   layer_thickness  w >= 1, interior lines per slice (the last slice takes the remainder);
 *                    <= 0 with opts->autotune > 0: chosen by timing (Autotuning below)
 *   opts             NULL for defaults
 *   out              receives the handle (NULL on failure)
 */
ls_status ls_setup(const ls_grid* grid, double omega, const double* m_dev, int pml_width,
                   int layer_thickness, const ls_options* opts, ls_handle** out);
/*
 * dim = 3 (Sec. 3.1): m_dev is [n][n][n] and every grid array of the entry
 * points below gains the third axis ([n][n][n] interior, [L][L][L] extended,
 * slice arrays [lines][L][L]); the slices are slabs of planes i1. Each slab
 * subproblem is block tridiagonal along i2 with blocks of (slab lines) x L
 * unknowns; setup forms S_j^{-1} of every block by blocked Gauss-Jordan with
 * partial pivoting in float64 (kept in the handle's precision:
 * L (t L)^2 complex per slab of t lines) and the sweep is applied slab by
 * slab (Algorithm 2; sweep_schedule is ignored). The 3D operator is the FFT
 * convolution of ls_op3_create. Not available in 3D: autotune (must be 0),
 * layer_thickness <= 0, ls_set_kernels. n <= 1023, slabs of at most 32 lines
 * and blocks (slab lines x L) of at most 4800 unknowns (LS_E_INVALID otherwise).
 * A slab whose block has a zero pivot gives LS_E_SINGULAR.
 */

/*
 * Solve (I + omega^2 K M) u = g for a batch of right-hand sides with
 * right-preconditioned restarted GMRES (flexible form), stopping each
 * right-hand side when its true relative residual is <= tol (Sec. 2.5).
 *   rhs_dev    complex128 [nrhs][n][n] ([nrhs][n][n][n] in 3D): g itself
 *              (LS_RHS_SOURCE) or the incident wave u_I on the interior grid
 *              (LS_RHS_INCIDENT, g = -omega^2 K (m u_I))
 *   u_dev      complex128, same shape, output: the scattered field; may be
 *              rhs_dev itself (each input value is read before u is written)
 *   info_host  host array of nrhs entries (may be NULL)
 * A zero right-hand side gives u = 0 after 0 iterations. Returns LS_E_NOCONV
 * if any right-hand side hit max_iters (u and info are still written).
 * Keeps the total fields needed by ls_adjoint.
 */
ls_status ls_solve(ls_handle* h, const void* rhs_dev, int nrhs, int rhs_kind, double tol,
                   void* u_dev, ls_rhs_info* info_host);

/*
 * Gradient of J = sum_j 1/2 |R u_j - d_j|^2 with respect to the grid vector m,
 * for the fields of the last ls_solve (same nrhs). Derived from eq. LS_d_c
 * (the paper states no adjoint): with psi = u + u_I the discrete equation reads
 * A(m) psi = u_I, A = I + omega^2 K M, so d psi = -A^{-1} omega^2 K diag(dm) psi;
 * K is complex symmetric (k depends on |delta| only), hence the adjoint solve
 * A^H lambda = r becomes A (K conj lambda) = K conj(r), a solve with the same
 * A and the same preconditioner:
 *   dJ/dm = -omega^2 Re sum_j psi_j * nu_j,   A nu_j = K conj(r_j),
 * psi_j = u_j + u_I,j (incident kind) or u_j (source kind), r_j = R^T (R u_j - d_j).
 *   resid_dev  complex128 [nrhs][n][n] ([nrhs][n][n][n] in 3D), the residuals r_j
 *   grad_dev   float64 [n][n] ([n][n][n] in 3D) output
 *   info_host  host array of nrhs entries for the adjoint solves (may be NULL)
 * Returns LS_E_STATE unless the handle's last ls_solve had the same nrhs, and
 * LS_E_NOCONV (gradient still written) if an adjoint solve hit max_iters.
 */
ls_status ls_adjoint(ls_handle* h, const void* resid_dev, int nrhs, double tol, double* grad_dev,
                     ls_rhs_info* info_host);

/* Release every resource of the handle; NULL is a no-op. */
void ls_destroy(ls_handle* h);

/* Message of the last failure on the calling thread ("" if none). */
const char* ls_last_error(void);

/* ---- Per-operator entry points (parity tests and benchmarks) ----
 * Shapes are given for dim = 2; in 3D each grid axis list gains one more n or L. */

/* y = (I + omega^2 K M) x on the interior grid (eq. LS_d_c). x, y: [nrhs][n][n]. */
ls_status ls_apply_A(ls_handle* h, const void* x_dev, int nrhs, void* y_dev, int precision);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = (I + omega^2 K M) x as ls_apply_A on a 2D handle, with the FFT work
 * array (nrhs x P x n8 complex values, P = fft length, n8 = n rounded up to
 * a multiple of 8) taken from a static
 * array of 64 MiB in the library's device memory, one per GPU, held until
 * the process ends. The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); the caller passes x and y as for ls_apply_A.
 *   Limit: nrhs x P x n8 x (16 B for LS_FP64, 8 B for LS_MIXED) <= 64 MiB, so
 *   at n = 1023 (P = 2048) at most 2 right-hand sides in complex128 and 4 in
 *   complex64; larger batches return LS_E_INVALID with the limit in the
 *   message. 3D handles return LS_E_INVALID.
 *   Every call on one GPU shares that GPU's array: calls that overlap on one
 *   GPU (other threads, other handles, other streams) race and must not be
 *   made. The array's contents need no clearing between calls.
 */
ls_status ls_apply_A_noalloc(ls_handle* h, const void* x_dev, int nrhs, void* y_dev, int precision);

/* y = K x (the convolution with k alone). x, y: [nrhs][n][n]. */
ls_status ls_apply_K(ls_handle* h, const void* x_dev, int nrhs, void* y_dev, int precision);

/* f = Q r: f_i = alpha^* r_{mu_i} on I^h = [0, n+1]^2, 0 on the PML (eq. Huf).
 * r: [nrhs][n][n] interior, f: [nrhs][L][L] extended. */
ls_status ls_apply_Q(ls_handle* h, const void* r_dev, int nrhs, void* f_dev, int precision);

/* y = H u on the extended grid (eqs. sp_stc, Huf), u = 0 on the Dirichlet ring.
 * u, y: [nrhs][L][L]. */
ls_status ls_apply_H(ls_handle* h, const void* u_dev, int nrhs, void* y_dev, int precision);

/* ---- The sparsifying stencils as a direct Helmholtz scheme (Sec. 4) ----
 * On a handle set up with m = 0, H is the scheme's matrix: at every point i
 * of I^h the row alpha^* u_{mu_i}, the PML rows gamma_i^* u_{mu_i}; the
 * equation alpha^* u_{mu_i} = beta^* f_{mu_i} discretises
 * (-Laplacian - omega^2) u = f, and with f = delta_c / h^2 (a point source at
 * grid point c) its solution approximates the free-space Green's function
 * about c. (With m != 0 the same calls solve H u = b for that medium.) */

/* b = beta^* f_{mu_i} on I^h = [0, n+1]^2, 0 on the PML (2D handles).
 * f: [nrhs][n][n] interior, b: [nrhs][L][L] extended. */
ls_status ls_apply_B(ls_handle* h, const void* f_dev, int nrhs, void* b_dev, int precision);

/* Solve H u = b on the extended grid for a batch (2D handles): right-
 * preconditioned flexible GMRES in float64, the sweep of Algorithm 2 (its
 * steps 3-8, in the handle's precision, fronts and schedule) as the
 * preconditioner, each right-hand side stopped at ||b - H u|| <= tol ||b||.
 *   rhs_dev, u_dev  complex128 [nrhs][L][L] (u = 0 on the Dirichlet ring)
 *   info_host       nrhs entries (may be NULL)
 * LS_E_NOCONV as for ls_solve (u and info still written). The call sizes the
 * handle's Krylov workspaces for extended-grid vectors; a following ls_solve
 * keeps the larger buffers. ls_adjoint after it returns LS_E_STATE. */
ls_status ls_solve_H(ls_handle* h, const void* rhs_dev, int nrhs, double tol, void* u_dev, ls_rhs_info* info_host);

/* z = P r, Algorithm 2: f = Q r, forward and backward sweep, restrict to I.
 * r, z: [nrhs][n][n]. precision must equal the handle's. */
ls_status ls_apply_precond(ls_handle* h, const void* r_dev, int nrhs, void* z_dev, int precision);

/* w = T~_k v for slice k (0-based, grid order): the D_k part of the subproblem
 * solution with right-hand side 0 on the auxiliary PML and v on D_k (eq.
 * Hwv_approx). v, w: [nrhs][lines of D_k][L], lines in grid order. precision
 * must equal the handle's. */
ls_status ls_slice_solve(ls_handle* h, int slice, const void* v_dev, int nrhs, void* w_dev,
                         int precision);

typedef struct {
  int dim, n, pml_width, layer_thickness, L, nslices, freq_samples, precision;
  double omega, h, pml_C, freq_lo, freq_delta;
  int fronts;  /* ls_options.fronts of the setup */
} ls_setup_info;

/* Sizes of the setup. */
ls_status ls_get_info(const ls_handle* h, ls_setup_info* info_host);

/* First and last grid line i1 of slice k (slices numbered in grid order along
 * x1, also with two fronts), and its number of auxiliary lines (both sides). */
ls_status ls_get_slice(const ls_handle* h, int slice, int* first_line, int* last_line, int* aux_lines);

/* Copies of the setup tables, float64 interleaved complex, on the host:
 *   alpha_host, beta_host  9 complex each (neighbourhood offsets (d1, d2) in
 *                          {-1,0,1}^2, d1 slowest)
 *   gamma_host             (2b+1)^2 x 9 complex, global PML stencils by per-axis
 *                          class (c1, c2), c = 0 interior, 1..b for i = -b..-1,
 *                          b+1..2b for i = n+2..n+1+b; entry (0,0) unused
 *   aux_host               b x (2b+1) x freq_samples x 9 complex, auxiliary PML
 *                          stencils by (depth q, class c2, sample k)
 * Any pointer may be NULL. In 3D the layouts of ls_host_tables3 (27 entries
 * per stencil, gamma by (c1, c2, c3), aux by (q, c2, c3, sample)). */
ls_status ls_get_stencils(const ls_handle* h, double* alpha_host, double* beta_host,
                          double* gamma_host, double* aux_host);

/* Sample index k* for every extended-grid point, int32 [L][L] ([L][L][L] in 3D) on the host. */
ls_status ls_get_sample_map(const ls_handle* h, int* kmap_host);

/* ---- Autotuning (batching form: layer thickness and kernel choice) ----
 *
 * The layer thickness w is a free parameter of the method: the remarks closing
 * Sec. 2.3 allow any slice width, and argue for w = b from the operation counts
 * of a serial setup and apply; on this device the best w follows from the
 * kernels' shapes (slices of at most 16 or 32 lines) and is measured. With
 * opts->autotune = k > 0 and layer_thickness <= 0, ls_setup sets up each of
 * the four thinnest candidates w (ls_layer_candidates for one front; with
 * two fronts the same rule applied to the two-front slices, the middle slice
 * included), times one solve of k plane waves
 * u_I = exp(i omega (cos t_j x1 + sin t_j x2)), t_j = 2 pi j / k, to a 1e-6
 * relative residual on the device, and keeps the fastest w. For the kept
 * setup it then times one preconditioner apply per kernel choice at batch
 * sizes 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, ... up to k, and every batch size
 * takes the choice measured fastest at the nearest measured size at or above
 * it (the largest measured size for larger batches). Tuning adds a few setups
 * and solves to ls_setup; results are identical up to rounding whatever the
 * choice (each choice is a different schedule of the same arithmetic).
 */

/* Host-only: the layer thicknesses w >= 2 for which every slice subproblem of
 * an n-point grid with PML width b has at most 32 lines (the slice kernels'
 * limit), ascending. out_host: array of cap entries (may be NULL with cap 0);
 * *count receives the number of candidates (which may exceed cap). */
ls_status ls_layer_candidates(int n, int pml_width, int* out_host, int cap, int* count);

typedef struct {
  int layer_thickness;  /* candidate w */
  int nslices;          /* slices of that setup (one front: floor((n+2)/w)) */
  int iterations;       /* most Arnoldi steps over the probe batch */
  double setup_ms;      /* its setup (Algorithm 1) */
  double solve_ms;      /* the probe solve */
} ls_tune_layer;

typedef struct {
  int nrhs;          /* batch size measured */
  int slice_kernel;  /* 1, 4, 8: slice solves on the vector ALUs, that many right-hand
                        sides per workgroup; 16: on the matrix cores, 16-column tiles */
  int iface_kernel;  /* 0: interface products as vector dot products (nrhs <= 4);
                        1: on the matrix cores */
  double apply_ms;   /* one preconditioner apply with this choice */
} ls_tune_kernels;

/* What the autotuner measured: the candidates of w (nothing when w was given)
 * and the kernel choice kept at each measured batch size. Host arrays of wcap
 * and kcap entries (either may be NULL with cap 0); *nw and *nk receive the
 * counts. */
ls_status ls_get_tuning(const ls_handle* h, ls_tune_layer* w_host, int wcap, int* nw, ls_tune_kernels* k_host,
                        int kcap, int* nk);

/* Force the kernel choice for batches of nrhs right-hand sides (1 <= nrhs <=
 * 256; batches above 256 follow 256), or for every batch size with nrhs = 0.
 * slice_kernel in {1, 4, 8, 16}, or 0 to restore the default (iface_kernel is
 * then ignored); iface_kernel 0 or 1, and 0 only for batches of at most 4
 * (with nrhs = 0, larger batches take 1 instead). The defaults, the
 * fastest measured on MI355X at n = 1023, b = 12, w = 4: LS_MIXED slice 1 up
 * to 2 right-hand sides, 4 up to 4, 16 above, interface 1; LS_FP64 slice 1,
 * interface 0 for one right-hand side, slice 4 for two, 16 above, interface 1
 * from two. */
ls_status ls_set_kernels(ls_handle* h, int nrhs, int slice_kernel, int iface_kernel);

/* ---- Kernel timing (HIP events recorded on the handle's stream) ---- */

typedef struct {
  char name[32];      /* "fft_convolve" (complex64 operator applies),
                         "fft_convolve_c128" (complex128 ones), "stencil_Q",
                         "slice_solves", "slice_solves_last", "interface",
                         "extract", "factor", "block_gram", "block_update",
                         "sweep" (sequential schedule) */
  int launches;       /* launches recorded since profiling was enabled */
  double total_ms;    /* summed event-to-event durations */
  long long columns;  /* right-hand-side columns processed, summed over launches */
} ls_kernel_time;

/* enable = 1: clear and start recording events around every kernel launch of
 * the handle; enable = 0: stop recording (the records stay readable). */
ls_status ls_profile(ls_handle* h, int enable);

/* Per-kind totals of the recorded launches; waits for them to finish.
 * out: host array of max entries; *count receives the number of kinds. */
ls_status ls_profile_read(ls_handle* h, ls_kernel_time* out_host, int max, int* count);

/*
 * Host-only (no device needed): the float64 setup tables of Algorithm 1,
 * steps 1-2, for a medium given on the host. Same tables and layouts as
 * ls_get_stencils / ls_get_sample_map, plus
 *   green_host  (n+2) x (n+2) complex, k_delta for delta in [0, n+1]^2
 *               (k is even in each axis), float64 interleaved
 * Any output pointer may be NULL. aux_host needs b x (2b+1) x ns x 9
 * complex entries with ns = freq_samples (or n if freq_samples is 0, or 1
 * when m is constant); entries no auxiliary point uses are zero.
 */
ls_status ls_host_tables(int n, double omega, const double* m_host, int pml_width, int layer_thickness,
                         double pml_C, int freq_samples, double* alpha_host, double* beta_host,
                         double* gamma_host, double* aux_host, int* kmap_host, double* green_host);

/*
 * The stencil cache. The setup tables that depend neither on m nor on the
 * layer thickness are kept for the last four (dim, n, omega, pml_width,
 * pml_C), compared exactly, and reused by ls_setup, ls_host_tables and
 * ls_host_tables3:
 * the Green's table (Sec. 2.1), alpha, beta (eqs. alpha, beta) and the
 * global PML stencils (eq. gamma). The stencils are fixed by the discretization
 * and the frequency alone, so repeated setups skip them. Examples are the
 * autotuner's candidates, or an inversion that changes m.
 *   clear   nonzero: empty the cache and reset the counters (after reading)
 *   hits, misses   may be NULL; lookups since the last clear
 * Thread-safe.
 */
ls_status ls_stencil_cache(int clear, long long* hits, long long* misses);

/*
 * Host-only: the float64 setup tables of the 3D method (Sec. 3.1: the
 * neighbourhood mu = {-1,0,1}^3, lexicographic with axis 0 slowest, and PML
 * stencils that annihilate the 26 neighbour directions), m_host [n][n][n]:
 *   alpha_host, beta_host  27 complex
 *   gamma_host  (2b+1)^3 x 27 complex, by per-axis class (c1, c2, c3)
 *   aux_host    b x (2b+1) x (2b+1) x ns x 27 complex, by (depth q, c2, c3,
 *               sample); entries no auxiliary point uses are zero
 *   kmap_host   L^3 int, the sample index of every extended point
 * Classes, samples and slabs as in 2D; a slab may have at most 32 lines and
 * blocks (lines x L) of at most 4800 unknowns.
 * Any output pointer may be NULL.
 */
ls_status ls_host_tables3(int n, double omega, const double* m_host, int pml_width, int layer_thickness,
                          double pml_C, int freq_samples, double* alpha_host, double* beta_host,
                          double* gamma_host, double* aux_host, int* kmap_host);

/*
 * The 3D operator (Sec. 1, eq. LS with d = 3; Sec. 2.1, eq. LS_d_c): on the
 * unit cube with n interior points per axis, h = 1/(n+1),
 *     k_delta = G(|delta| h) h^3,  G(r) = exp(i omega r) / (4 pi r),
 * and k_0 the integral of G over the ball of volume h^3 in closed form:
 *     a = h (3/(4 pi))^(1/3),  k_0 = (exp(i omega a)(1 - i omega a) - 1) / omega^2.
 * A 3D handle holds the Green's spectrum and the medium and applies A and K
 * by a zero-padded FFT convolution of length P = fft_len(n) >= 2n per axis.
 * It is the operator alone, for callers that need A or K without a setup;
 * the preconditioned 3D solve is ls_setup with grid->dim = 3.
 *
 * ls_op3_create: m_dev is float64 [n][n][n] (i3 fastest, finite, < 1
 *   everywhere), copied. hip_stream: hipStream_t for every later call (NULL:
 *   default stream). 1 <= n <= 1023. Device memory: the spectrum octant
 *   (P/2+1)^3 in both precisions, plus, during creation only, P^3 complex128.
 * ls_op3_apply_A: y = x + omega^2 K (m .* x); ls_op3_apply_K: y = K x.
 *   x_dev, y_dev: [nrhs][n][n][n] complex (complex128 for LS_FP64, complex64
 *   for LS_MIXED), caller-owned, must not overlap. The first call with a
 *   larger nrhs grows the handle's work arrays to
 *   nrhs (n P^2 + n^2 P) complex128 entries.
 * Errors: LS_E_INVALID for bad arguments (the handle is left unchanged),
 *   LS_E_NOMEM when an allocation fails, LS_E_DEVICE when a HIP call fails.
 */
typedef struct ls_op3 ls_op3;
ls_status ls_op3_create(int n, double omega, const double* m_dev, void* hip_stream, ls_op3** out);
ls_status ls_op3_apply_A(ls_op3* h, const void* x_dev, int nrhs, void* y_dev, int precision);
ls_status ls_op3_apply_K(ls_op3* h, const void* x_dev, int nrhs, void* y_dev, int precision);
void ls_op3_destroy(ls_op3* h);

/*
 * Host-only: the 3D Green's table of ls_op3_create, k_delta for delta in
 * [0, n+1]^3 (k is even in each axis), written to green_host as
 * (n+2)^3 complex float64 interleaved, delta3 fastest.
 */
ls_status ls_host_green3(int n, double omega, double* green_host);

#ifdef __cplusplus
}
#endif

#endif /* LSWEEP_H */
