// Host-side float64 setup of the sparsify-and-sweep preconditioner
// (Algorithm 1, steps 1-3): Green's-function table, type-1 stencils alpha and
// beta (eqs. alpha, beta), PML stencils gamma (eq. gamma) for the global PML
// and for the auxiliary PML at sampled local frequencies (Sec. 2.3), and the
// slice plan along x1.
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace lsw {

using cd = std::complex<double>;

// One slice subproblem. Its t lines are numbered locally a = 0..t-1 in the
// order of its front: grid line org + dir * a. Local lines [0, naux) are
// auxiliary PML before D_k, [naux, naux + (hi - lo + 1)) are D_k, the rest
// (nauxr lines) auxiliary PML after it. The one-front sweep and the left front
// of the two-front sweep run along x1 (dir = +1, auxiliary lines left of
// D_k); the right front runs against it (dir = -1: its auxiliary lines, right
// of D_k in the grid, come first locally); the two-front middle slice has
// auxiliary lines on both sides.
struct SlicePlan {
  int lo;     // first grid line i1 of D_k
  int hi;     // last grid line of D_k
  int first;  // lowest grid line of the subproblem
  int t;      // lines in the subproblem
  int naux;   // auxiliary lines before D_k (local order)
  int nauxr = 0;     // auxiliary lines after D_k (local order)
  int org = 0;       // grid line of local line 0
  int dir = 1;       // +1 or -1
  int prev = -1;     // slice (table index) eliminated just before, coupled to D_k's first local line; -1: none
  int next = -1;     // slice coupled to D_k's last local line, eliminated after; -1: none
  int next_lam = 0;  // 1: that coupling takes the next slice's last line (lambda), 0 its first line (mu)
  int grid = 0;      // position of the slice in grid order
};

struct HostSetup {
  int n = 0, b = 0, w = 0, L = 0, P = 0, nslices = 0, ns = 0, fronts = 1;
  double omega = 0, h = 0, C = 0;
  double freq_lo = 0, freq_delta = 0;
  std::vector<cd> kq;          // k_delta for delta in [0, n+1]^2, [(n+2)][(n+2)]
  cd alpha[9], beta[9];        // neighbourhood order (d1, d2), d1 slowest
  double alpha_sv[9];          // singular values of K_{mu,mu^c}, descending
  std::vector<cd> gamma_glob;  // [(2b+1)^2][9] by per-axis class (c1, c2)
  std::vector<cd> gamma_aux;   // [b][2b+1][ns][9] by (depth q, class c2, sample k)
  std::vector<int> kmap;       // [L][L] sample index of every extended point
  std::vector<SlicePlan> slices;
};

// Own float64 Bessel functions (series, Miller recurrence with the Neumann
// series for Y0, Hankel's asymptotic expansion for large arguments).
void bessel_j0y0(double x, double* j0, double* y0);
void bessel_j1y1_small(double x, double* j1, double* y1);

// The same setup in 3D (Sec. 3.1): 27-point neighbourhood mu = {-1,0,1}^3 in
// lexicographic order (axis 0 slowest), PML stencils annihilating the 26
// neighbour directions, the sample map over the extended cube.
struct HostSetup3 {
  int n = 0, b = 0, w = 0, L = 0, nslices = 0, ns = 0;
  double omega = 0, h = 0, C = 0;
  double freq_lo = 0, freq_delta = 0;
  std::vector<cd> kq;          // k_delta for delta in [0, n+1]^3, [(n+2)]^3
  cd alpha[27], beta[27];
  double alpha_sv[27];         // singular values of K_{mu,mu^c}, descending
  std::vector<cd> gamma_glob;  // [(2b+1)^3][27] by per-axis class (c1, c2, c3)
  std::vector<cd> gamma_aux;   // [b][2b+1][2b+1][ns][27] by (depth q, c2, c3, sample k)
  std::vector<int> kmap;       // [L]^3 sample index of every extended point
  std::vector<SlicePlan> slices;
};

// Per-axis stretch class of grid index i (0 interior, 1..b low, b+1..2b high).
int axis_class(int i, int n, int b);

// 3D Green's table k_delta for delta in [0, n+1]^3, [(n+2)][(n+2)][(n+2)]:
// G(r) = exp(i omega r) / (4 pi r) times h^3 off the origin (Sec. 1, eq.
// LS_d), k_0 the integral of G over the ball of volume h^3 (reading G1):
// (exp(i omega a)(1 - i omega a) - 1) / omega^2, a = h (3 / (4 pi))^(1/3).
std::vector<cd> green3_octant(int n, double omega);

// Build everything (2D) from m on the host. Returns "" on success, else a message.
// The tables that do not depend on m or w (the Green table, alpha, beta and
// the global PML stencils: functions of n, omega, b and C) are kept in a
// process-wide cache of the last kStencilCacheEntries keys (shared with the
// 3D setup, keyed by dimension too) and reused.
std::string build_host_setup(const double* m_host, int n, double omega, int b, int w, double C,
                             int freq_samples, HostSetup& out, int fronts = 1);
// The slices in table order (see SlicePlan). One front (Algorithms 1-2,
// reading G8): l = floor((n+2)/w) slices along x1, the last taking the
// remainder. Two fronts (the first remark after Algorithm 2, Sec. 2.4;
// reading G18): p = floor((n+1)/(2w)) slices of w lines from each end, then
// the middle slice of the remaining 1..2w lines, eliminated last; table order
// is the left front outward-in, the right front outward-in, the middle.
std::vector<SlicePlan> plan_slices(int n, int b, int w, int fronts);
constexpr int kStencilCacheEntries = 4;
// Counters of that cache since the last clear; clear = true empties it.
void stencil_cache(bool clear, long long* hits, long long* misses);

// 3D: m is [n][n][n]; slices are slabs of lines i1 with at most
// max_slab_lines lines and blocks (lines x L) of at most max_block unknowns.
std::string build_host_setup3(const double* m_host, int n, double omega, int b, int w, double C,
                              int freq_samples, int max_slab_lines, int max_block, HostSetup3& out);

}  // namespace lsw
