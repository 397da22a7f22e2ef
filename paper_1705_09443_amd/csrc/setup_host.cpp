// Host-side float64 setup (Algorithm 1, steps 1-3). Compiled with
// -ffp-contract=off: the local-frequency sample index of every point is an
// integer decided in floating point, and the expression order here is the
// documented one (nearest sample, Sec. 2.3), evaluated without fused
// multiply-adds.
#include "setup_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

namespace lsw {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;

unsigned worker_count() {
  unsigned t = std::thread::hardware_concurrency();
  if (t == 0) t = 4;
  return std::min(t, 16u);
}

template <typename F>
void parallel_for(int count, F&& body) {
  unsigned nt = std::min<unsigned>(worker_count(), std::max(1, count));
  if (nt <= 1) {
    for (int i = 0; i < count; ++i) body(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int i = (int)t; i < count; i += (int)nt) body(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

// ---------------------------------------------------------------------------
// Bessel functions of order 0 and 1 (float64).
//  x <= 25: Miller's backward recurrence for J_k normalised by
//           J_0 + 2 sum J_2k = 1; Y_0 from the Neumann series
//           Y_0 = (2/pi)(ln(x/2) + gamma) J_0 - (4/pi) sum (-1)^k J_2k / k.
//  x > 25:  Hankel's asymptotic expansion, J_0 + i Y_0 =
//           sqrt(2/(pi x)) (P + i Q) exp(i (x - pi/4)), summed to round-off.
// ---------------------------------------------------------------------------
void bessel_j0y0(double x, double* j0, double* y0) {
  if (x > 25.0) {
    const double z8 = 8.0 * x;
    double P = 1.0, Q = 0.0, a = 1.0;
    for (int k = 1; k < 200; ++k) {
      const double f = (2.0 * k - 1.0) * (2.0 * k - 1.0) / (k * z8);
      if (f >= 1.0) break;  // the asymptotic series starts to grow
      a *= f;
      // P = a0 - a2 + a4 - ...,  Q = -a1 + a3 - a5 + ...
      switch (k & 3) {
        case 0: P += a; break;
        case 1: Q -= a; break;
        case 2: P -= a; break;
        case 3: Q += a; break;
      }
      if (a < 1e-18) break;
    }
    const double s = std::sin(x), c = std::cos(x);
    const double cchi = (c + s) * (1.0 / std::sqrt(2.0));  // cos(x - pi/4)
    const double schi = (s - c) * (1.0 / std::sqrt(2.0));  // sin(x - pi/4)
    const double amp = std::sqrt(2.0 / (kPi * x));
    *j0 = amp * (P * cchi - Q * schi);
    *y0 = amp * (P * schi + Q * cchi);
    return;
  }
  int N = 2 * (int)((x + 10.0 * std::cbrt(x) + 24.0) / 2.0);
  double jp1 = 0.0, jk = 1e-280;  // J_{N+1}, J_N (unnormalised)
  double norm = 0.0, neu = 0.0;   // J0 + 2 sum J_2k, sum (-1)^k J_2k / k
  double jzero = 0.0;
  for (int k = N; k >= 1; --k) {
    const double jm1 = (2.0 * k / x) * jk - jp1;  // J_{k-1}
    jp1 = jk;
    jk = jm1;
    const int km1 = k - 1;
    if (km1 > 0 && (km1 & 1) == 0) {
      const int h = km1 / 2;
      norm += 2.0 * jk;
      neu += ((h & 1) ? -1.0 : 1.0) * jk / h;
    }
    if (std::fabs(jk) > 1e250) {  // rescale to stay in range
      jk *= 1e-250;
      jp1 *= 1e-250;
      norm *= 1e-250;
      neu *= 1e-250;
    }
  }
  jzero = jk;
  norm += jzero;
  const double J0 = jzero / norm;
  *j0 = J0;
  *y0 = (2.0 / kPi) * (std::log(0.5 * x) + kEulerGamma) * J0 - (4.0 / kPi) * (neu / norm);
}

// J_1 and Y_1 by their power series (small arguments: the central weight
// needs them at omega h / sqrt(pi) < 2).
//  J_1 = sum (-1)^k (x/2)^(2k+1) / (k! (k+1)!)
//  Y_1 = -2/(pi x) + (2/pi) ln(x/2) J_1
//        - (x/(2 pi)) sum (psi(k+1) + psi(k+2)) (-x^2/4)^k / (k! (k+1)!)
void bessel_j1y1_small(double x, double* j1, double* y1) {
  const double q = 0.25 * x * x;
  double term = 1.0;  // (-q)^k / (k! (k+1)!)
  double sj = 0.0, sy = 0.0;
  double psi1 = -kEulerGamma;      // psi(k+1)
  double psi2 = 1.0 - kEulerGamma; // psi(k+2)
  for (int k = 0; k < 60; ++k) {
    sj += term;
    sy += (psi1 + psi2) * term;
    psi1 += 1.0 / (k + 1);
    psi2 += 1.0 / (k + 2);
    term *= -q / ((k + 1.0) * (k + 2.0));
    if (std::fabs(term) < 1e-20 * std::fabs(sj)) break;
  }
  const double J1 = 0.5 * x * sj;
  *j1 = J1;
  *y1 = -2.0 / (kPi * x) + (2.0 / kPi) * std::log(0.5 * x) * J1 - (x / (2.0 * kPi)) * sy;
}

int axis_class(int i, int n, int b) {
  if (i < 0) return i + b + 1;
  if (i > n + 1) return i - (n + 2) + b + 1;
  return 0;
}

namespace {

// Representative grid index of per-axis class c.
int class_index(int c, int n, int b) {
  if (c == 0) return 0;
  if (c <= b) return c - 1 - b;
  return n + 2 + (c - b - 1);
}

// Global PML stretch times omega at grid index i: omega*sigma = -/+ C (q/b)^2
// (Sec. 2.2.2), continued to the Dirichlet points (reading G3).
double omega_sigma_global(int i, int n, int b, double C) {
  if (i <= -1) {
    const double q = (-1.0 - i) / b;
    return -C * q * q;
  }
  if (i >= n + 2) {
    const double q = (i - n - 2.0) / b;
    return C * q * q;
  }
  return 0.0;
}

// Auxiliary x1 stretch times omega at depth q left of the slice (q <= 0 inside).
double omega_sigma_aux(int q, int b, double C) {
  if (q <= 0) return 0.0;
  const double r = (double)q / b;
  return -C * r * r;
}

// ---- small dense complex linear algebra (column-major helpers) -------------

// Smallest right singular vector of the rows x cols matrix A (row-major),
// rows >= 1, cols <= 32, by one-sided (Hestenes) Jacobi: rotate column pairs
// until all are orthogonal; V accumulates the rotations. Singular values are
// returned descending in sv (cols entries) when sv != nullptr.
void jacobi_min_right_vector(std::vector<cd> A, int rows, int cols, cd* out, double* sv) {
  std::vector<cd> V((size_t)cols * cols, cd(0.0));
  for (int i = 0; i < cols; ++i) V[(size_t)i * cols + i] = 1.0;
  auto col = [&](int r, int c) -> cd& { return A[(size_t)r * cols + c]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        double al = 0.0, be = 0.0;
        cd ga(0.0);
        for (int r = 0; r < rows; ++r) {
          al += std::norm(col(r, p));
          be += std::norm(col(r, q));
          ga += std::conj(col(r, p)) * col(r, q);
        }
        const double ag = std::abs(ga);
        if (ag == 0.0 || ag <= 1e-17 * std::sqrt(al * be)) continue;
        rotated = true;
        const cd e = ga / ag;
        const double zeta = (be - al) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < rows; ++r) {
          const cd ap = col(r, p), aq = std::conj(e) * col(r, q);
          col(r, p) = c * ap - s * aq;
          col(r, q) = s * ap + c * aq;
        }
        for (int r = 0; r < cols; ++r) {
          const cd vp = V[(size_t)r * cols + p], vq = std::conj(e) * V[(size_t)r * cols + q];
          V[(size_t)r * cols + p] = c * vp - s * vq;
          V[(size_t)r * cols + q] = s * vp + c * vq;
        }
      }
    if (!rotated) break;
  }
  std::vector<double> nrm(cols);
  for (int c = 0; c < cols; ++c) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += std::norm(col(r, c));
    nrm[c] = std::sqrt(s);
  }
  int best = 0;
  for (int c = 1; c < cols; ++c)
    if (nrm[c] < nrm[best]) best = c;
  for (int r = 0; r < cols; ++r) out[r] = V[(size_t)r * cols + best];
  if (sv) {
    std::vector<double> s(nrm);
    std::sort(s.begin(), s.end(), [](double a, double b) { return a > b; });
    for (int c = 0; c < cols; ++c) sv[c] = s[c];
  }
}

// Householder QR update: R (cols x cols upper triangular, row-major) <- R
// factor of [R; B] with B (nb x cols, row-major). Unit-norm reflectors.
void qr_append(std::vector<cd>& R, const cd* B, int nb, int cols, bool have_R) {
  const int top = have_R ? cols : 0;
  const int rows = top + nb;
  std::vector<cd> M((size_t)rows * cols);
  if (have_R) std::copy(R.begin(), R.end(), M.begin());
  std::copy(B, B + (size_t)nb * cols, M.begin() + (size_t)top * cols);
  std::vector<cd> v(rows);
  for (int c = 0; c < cols && c < rows; ++c) {
    double xn2 = 0.0;
    for (int r = c; r < rows; ++r) xn2 += std::norm(M[(size_t)r * cols + c]);
    const double xn = std::sqrt(xn2);
    if (xn == 0.0) continue;
    const cd x0 = M[(size_t)c * cols + c];
    const cd ph = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
    const cd alpha = -ph * xn;
    double vn2 = 0.0;
    for (int r = c; r < rows; ++r) {
      v[r] = M[(size_t)r * cols + c] - (r == c ? alpha : cd(0.0));
      vn2 += std::norm(v[r]);
    }
    const double vn = std::sqrt(vn2);
    if (vn == 0.0) continue;
    for (int r = c; r < rows; ++r) v[r] /= vn;
    for (int cc = c; cc < cols; ++cc) {
      cd dot(0.0);
      for (int r = c; r < rows; ++r) dot += std::conj(v[r]) * M[(size_t)r * cols + cc];
      for (int r = c; r < rows; ++r) M[(size_t)r * cols + cc] -= 2.0 * v[r] * dot;
    }
  }
  R.assign((size_t)cols * cols, cd(0.0));
  for (int r = 0; r < cols && r < rows; ++r)
    for (int c = r; c < cols; ++c) R[(size_t)r * cols + c] = M[(size_t)r * cols + c];
}

// Null vector of the 9 x 8 matrix F (row-major): the last column of the Q
// of its Householder QR, i.e. the unit vector orthogonal to all columns.
void null_vector_9x8(const cd* F, cd* out) {
  const int rows = 9, cols = 8;
  cd M[72];
  std::copy(F, F + 72, M);
  cd vs[8][9];
  for (int c = 0; c < cols; ++c) {
    double xn2 = 0.0;
    for (int r = c; r < rows; ++r) xn2 += std::norm(M[r * cols + c]);
    const double xn = std::sqrt(xn2);
    const cd x0 = M[c * cols + c];
    const cd ph = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
    const cd alpha = -ph * xn;
    double vn2 = 0.0;
    for (int r = 0; r < rows; ++r) {
      vs[c][r] = (r < c) ? cd(0.0) : M[r * cols + c] - (r == c ? alpha : cd(0.0));
      vn2 += std::norm(vs[c][r]);
    }
    const double vn = std::sqrt(vn2);
    for (int r = 0; r < rows; ++r) vs[c][r] = (vn > 0) ? vs[c][r] / vn : cd(0.0);
    for (int cc = c; cc < cols; ++cc) {
      cd dot(0.0);
      for (int r = c; r < rows; ++r) dot += std::conj(vs[c][r]) * M[r * cols + cc];
      for (int r = c; r < rows; ++r) M[r * cols + cc] -= 2.0 * vs[c][r] * dot;
    }
  }
  cd e[9] = {};
  e[8] = 1.0;
  for (int c = cols - 1; c >= 0; --c) {  // Q e_9 = H_1 (H_2 (... H_8 e_9))
    cd dot(0.0);
    for (int r = 0; r < rows; ++r) dot += std::conj(vs[c][r]) * e[r];
    for (int r = 0; r < rows; ++r) e[r] -= 2.0 * vs[c][r] * dot;
  }
  std::copy(e, e + 9, out);
}

// Reading G5: unit norm, centre coefficient real positive (else the first
// largest-modulus entry).
void normalise_phase(cd* v, int len) {
  double s = 0.0;
  for (int i = 0; i < len; ++i) s += std::norm(v[i]);
  const double inv = 1.0 / std::sqrt(s);
  for (int i = 0; i < len; ++i) v[i] *= inv;
  int j = (len - 1) / 2;
  if (std::abs(v[j]) < 1e-12) {
    j = 0;
    for (int i = 1; i < len; ++i)
      if (std::abs(v[i]) > std::abs(v[j])) j = i;
  }
  const cd c = v[j];
  const double a = std::abs(c);
  const cd rot = std::conj(c) / a;
  for (int i = 0; i < len; ++i) v[i] *= rot;
  v[j] = a;
}

// gamma of eq. gamma for one point in 2D: the null vector of the sampled
// modified plane waves, each column divided by its centre value:
//   F'_{o,r} = exp(i kappa h r.o) exp(-(kappa/omega) sum_k r_k (os_k[o_k] - os_k[0]))
// where os_k holds omega*sigma of axis k at offsets -1, 0, +1.
void pml_gamma_2d(double kappa, double omega, double h, const double os[2][3], cd* out) {
  static const int dirs_v[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};
  cd F[9 * 8];
  const double kr = kappa / omega;
  for (int r = 0; r < 8; ++r) {
    const double nv = std::sqrt((double)(dirs_v[r][0] * dirs_v[r][0] + dirs_v[r][1] * dirs_v[r][1]));
    const double r1 = dirs_v[r][0] / nv, r2 = dirs_v[r][1] / nv;
    for (int o = 0; o < 9; ++o) {
      const int d1 = o / 3 - 1, d2 = o % 3 - 1;
      const double ph = kappa * h * (r1 * d1 + r2 * d2);
      const double dmp = -kr * (r1 * (os[0][d1 + 1] - os[0][1]) + r2 * (os[1][d2 + 1] - os[1][1]));
      F[o * 8 + r] = std::exp(cd(dmp, ph));
    }
  }
  null_vector_9x8(F, out);
  normalise_phase(out, 9);
}

// Null vector of the rows x (rows - 1) matrix F (row-major): the last column
// of the Q of its Householder QR.
void null_vector_hh(const cd* F, int rows, cd* out) {
  const int cols = rows - 1;
  std::vector<cd> M(F, F + (size_t)rows * cols);
  std::vector<cd> vs((size_t)cols * rows);
  for (int c = 0; c < cols; ++c) {
    cd* v = &vs[(size_t)c * rows];
    double xn2 = 0.0;
    for (int r = c; r < rows; ++r) xn2 += std::norm(M[(size_t)r * cols + c]);
    const double xn = std::sqrt(xn2);
    const cd x0 = M[(size_t)c * cols + c];
    const cd ph = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
    const cd alpha = -ph * xn;
    double vn2 = 0.0;
    for (int r = 0; r < rows; ++r) {
      v[r] = (r < c) ? cd(0.0) : M[(size_t)r * cols + c] - (r == c ? alpha : cd(0.0));
      vn2 += std::norm(v[r]);
    }
    const double vn = std::sqrt(vn2);
    for (int r = 0; r < rows; ++r) v[r] = (vn > 0) ? v[r] / vn : cd(0.0);
    for (int cc = c; cc < cols; ++cc) {
      cd dot(0.0);
      for (int r = c; r < rows; ++r) dot += std::conj(v[r]) * M[(size_t)r * cols + cc];
      for (int r = c; r < rows; ++r) M[(size_t)r * cols + cc] -= 2.0 * v[r] * dot;
    }
  }
  std::vector<cd> e(rows, cd(0.0));
  e[rows - 1] = 1.0;
  for (int c = cols - 1; c >= 0; --c) {
    const cd* v = &vs[(size_t)c * rows];
    cd dot(0.0);
    for (int r = 0; r < rows; ++r) dot += std::conj(v[r]) * e[r];
    for (int r = 0; r < rows; ++r) e[r] -= 2.0 * v[r] * dot;
  }
  std::copy(e.begin(), e.end(), out);
}

// gamma of eq. gamma for one point in 3D (Sec. 3.1): as pml_gamma_2d over
// the 27-point neighbourhood and the 26 directions v / |v|, v in
// {-1,0,1}^3 minus 0 (lexicographic, axis 0 slowest).
void pml_gamma_3d(double kappa, double omega, double h, const double os[3][3], cd* out) {
  double dirs[26][3];
  int nd = 0;
  for (int v = 0; v < 27; ++v) {
    const int a = v / 9 - 1, c = (v / 3) % 3 - 1, e = v % 3 - 1;
    if (!a && !c && !e) continue;
    const double nv = std::sqrt((double)(a * a + c * c + e * e));
    dirs[nd][0] = a / nv;
    dirs[nd][1] = c / nv;
    dirs[nd][2] = e / nv;
    ++nd;
  }
  cd F[27 * 26];
  const double kr = kappa / omega;
  for (int r = 0; r < 26; ++r)
    for (int o = 0; o < 27; ++o) {
      const int d1 = o / 9 - 1, d2 = (o / 3) % 3 - 1, d3 = o % 3 - 1;
      const double ph = kappa * h * (dirs[r][0] * d1 + dirs[r][1] * d2 + dirs[r][2] * d3);
      const double dmp = -kr * (dirs[r][0] * (os[0][d1 + 1] - os[0][1]) + dirs[r][1] * (os[1][d2 + 1] - os[1][1]) +
                                dirs[r][2] * (os[2][d3 + 1] - os[2][1]));
      F[o * 26 + r] = std::exp(cd(dmp, ph));
    }
  null_vector_hh(F, 27, out);
  normalise_phase(out, 27);
}

// Local-frequency sample nearest to omega^2 (1 - m) (Sec. 2.3, reading G9).
int sample_index(double mp, double w2, double lo, double delta, int ns) {
  if (ns <= 1) return 0;
  const double v = w2 * (1.0 - mp);
  const double t = (v - lo) / delta + 0.5;
  const double f = std::floor(t);
  return f < 0 ? 0 : (f > ns - 1 ? ns - 1 : (int)f);
}

}  // namespace

std::vector<cd> green3_octant(int n, double omega) {
  const int Q = n + 2;
  const double h = 1.0 / (n + 1);
  std::vector<cd> kq((size_t)Q * Q * Q);
  parallel_for(Q, [&](int a) {
    for (int c = 0; c < Q; ++c)
      for (int e = 0; e < Q; ++e) {
        cd val;
        if (a == 0 && c == 0 && e == 0) {
          const double rad = h * std::cbrt(3.0 / (4.0 * kPi));
          const cd eia = std::exp(cd(0.0, omega * rad));
          val = (eia * cd(1.0, -omega * rad) - 1.0) / (omega * omega);
        } else {
          const double r = std::sqrt((double)a * a + (double)c * c + (double)e * e) * h;
          val = std::exp(cd(0.0, omega * r)) / (4.0 * kPi * r) * (h * h * h);
        }
        kq[((size_t)a * Q + c) * Q + e] = val;
      }
  });
  return kq;
}

namespace {

// The velocity-independent tables of one (d, n, omega, b, C), keys compared
// exactly. Entries are immutable once inserted; the most recent is first.
struct StencilEntry {
  int d, n, b;
  double omega, C;
  std::vector<cd> kq, gamma_glob, alpha, beta;  // alpha, beta: 3^d entries
  std::vector<double> alpha_sv;
};
std::mutex g_stencil_mu;
std::deque<std::shared_ptr<const StencilEntry>> g_stencils;
long long g_stencil_hits = 0, g_stencil_misses = 0;

std::shared_ptr<const StencilEntry> stencil_find(int d, int n, double omega, int b, double C) {
  std::lock_guard<std::mutex> lk(g_stencil_mu);
  for (size_t i = 0; i < g_stencils.size(); ++i) {
    const auto& e = g_stencils[i];
    if (e->d == d && e->n == n && e->b == b && e->omega == omega && e->C == C) {
      auto hit = e;
      g_stencils.erase(g_stencils.begin() + (long)i);
      g_stencils.push_front(hit);
      ++g_stencil_hits;
      return hit;
    }
  }
  ++g_stencil_misses;
  return nullptr;
}

void stencil_insert(std::shared_ptr<const StencilEntry> e) {
  std::lock_guard<std::mutex> lk(g_stencil_mu);
  g_stencils.push_front(std::move(e));
  while ((int)g_stencils.size() > kStencilCacheEntries) g_stencils.pop_back();
}

std::shared_ptr<const StencilEntry> make_entry(int d, int n, double omega, int b, double C,
                                               const std::vector<cd>& kq, const std::vector<cd>& gamma_glob,
                                               const cd* alpha, const cd* beta, const double* sv, int nmu) {
  auto e = std::make_shared<StencilEntry>();
  e->d = d;
  e->n = n;
  e->b = b;
  e->omega = omega;
  e->C = C;
  e->kq = kq;
  e->gamma_glob = gamma_glob;
  e->alpha.assign(alpha, alpha + nmu);
  e->beta.assign(beta, beta + nmu);
  e->alpha_sv.assign(sv, sv + nmu);
  return e;
}

}  // namespace

void stencil_cache(bool clear, long long* hits, long long* misses) {
  std::lock_guard<std::mutex> lk(g_stencil_mu);
  if (hits) *hits = g_stencil_hits;
  if (misses) *misses = g_stencil_misses;
  if (clear) {
    g_stencils.clear();
    g_stencil_hits = g_stencil_misses = 0;
  }
}

std::vector<SlicePlan> plan_slices(int n, int b, int w, int fronts) {
  std::vector<SlicePlan> out;
  const int p = fronts == 2 ? (n + 1) / (2 * w) : 0;
  if (fronts != 2 || p == 0) {
    const int nl = fronts == 2 ? 1 : std::max(1, (n + 2) / w);
    out.resize(nl);
    for (int k = 0; k < nl; ++k) {
      SlicePlan& q = out[k];
      q.lo = (k == 0) ? -b : k * w;
      q.hi = (k == nl - 1) ? n + 1 + b : (k + 1) * w - 1;
      q.first = (k == 0) ? q.lo : q.lo - b;
      q.t = q.hi - q.first + 1;
      q.naux = q.lo - q.first;
      q.org = q.first;
      q.dir = 1;
      q.prev = k - 1;
      q.next = k + 1 < nl ? k + 1 : -1;
      q.grid = k;
    }
    return out;
  }
  out.resize(2 * p + 1);
  const int mid = 2 * p;
  for (int k = 0; k < p; ++k) {  // left front, along x1
    SlicePlan& q = out[k];
    q.lo = k == 0 ? -b : k * w;
    q.hi = (k + 1) * w - 1;
    q.naux = k == 0 ? 0 : b;
    q.first = q.lo - q.naux;
    q.t = q.hi - q.first + 1;
    q.org = q.first;
    q.dir = 1;
    q.prev = k - 1;
    q.next = k + 1 < p ? k + 1 : mid;
    q.next_lam = 0;
    q.grid = k;
  }
  for (int j = 0; j < p; ++j) {  // right front, against x1
    SlicePlan& q = out[p + j];
    q.lo = n + 2 - (j + 1) * w;
    q.hi = j == 0 ? n + 1 + b : n + 1 - j * w;
    q.naux = j == 0 ? 0 : b;
    q.first = q.lo;
    q.t = q.hi - q.lo + 1 + q.naux;
    q.org = q.hi + q.naux;
    q.dir = -1;
    q.prev = j == 0 ? -1 : p + j - 1;
    q.next = j + 1 < p ? p + j + 1 : mid;
    q.next_lam = j + 1 < p ? 0 : 1;  // next to the middle slice: its last line
    q.grid = 2 * p - j;
  }
  SlicePlan& q = out[mid];  // middle: auxiliary lines on both sides
  q.lo = p * w;
  q.hi = n + 1 - p * w;
  q.naux = b;
  q.nauxr = b;
  q.first = q.lo - b;
  q.t = q.hi - q.lo + 1 + 2 * b;
  q.org = q.first;
  q.dir = 1;
  q.prev = p - 1;       // the left front's last slice (its lambda)
  q.next = 2 * p - 1;   // the right front's last slice (its lambda)
  q.next_lam = 1;
  q.grid = p;
  return out;
}

std::string build_host_setup(const double* m, int n, double omega, int b, int w, double C,
                             int freq_samples, HostSetup& S, int fronts) {
  char buf[256];
  if (n < 1) return "n must be >= 1";
  if (!(omega > 0.0) || !std::isfinite(omega)) return "omega must be finite and > 0";
  if (b < 1) return "pml_width must be >= 1";
  if (w < 1) return "layer_thickness must be >= 1";
  if (!(C >= 0.0) || !std::isfinite(C)) return "pml_C must be finite and >= 0";
  const double h = 1.0 / (n + 1);
  const double wa = omega * h / std::sqrt(kPi);
  if (wa > 2.0) return "fewer than ~2 points per wavelength (omega*h/sqrt(pi) > 2)";
  S.n = n;
  S.b = b;
  S.w = w;
  S.omega = omega;
  S.h = h;
  S.C = C;
  S.L = n + 2 + 2 * b;
  S.P = 2 * (n + 1);
  const int L = S.L;

  // ---- medium range and local-frequency samples (Sec. 2.3, reading G9) ----
  double mmax = -INFINITY, mmin = INFINITY;
  for (size_t i = 0; i < (size_t)n * n; ++i) {
    if (!std::isfinite(m[i])) return "m has a non-finite value";
    mmax = std::max(mmax, m[i]);
    mmin = std::min(mmin, m[i]);
  }
  if (!(1.0 - mmax > 0.0)) return "max m must be < 1 (the local frequency must be real)";
  const double w2 = omega * omega;
  const double lo = w2 * (1.0 - mmax);
  const double hi = w2 * (1.0 - mmin);
  int ns = freq_samples > 0 ? freq_samples : n;
  if (!(hi > lo)) ns = 1;
  const double delta = ns > 1 ? (hi - lo) / (ns - 1) : 0.0;
  S.ns = ns;
  S.freq_lo = lo;
  S.freq_delta = delta;
  S.kmap.assign((size_t)L * L, 0);
  for (int e1 = 0; e1 < L; ++e1)
    for (int e2 = 0; e2 < L; ++e2) {
      const int i1 = e1 - b, i2 = e2 - b;
      double mp = 0.0;
      if (i1 >= 1 && i1 <= n && i2 >= 1 && i2 <= n) mp = m[(size_t)(i1 - 1) * n + (i2 - 1)];
      int k = 0;
      if (ns > 1) {
        const double v = w2 * (1.0 - mp);
        const double t = (v - lo) / delta + 0.5;
        const double f = std::floor(t);
        k = f < 0 ? 0 : (f > ns - 1 ? ns - 1 : (int)f);
      }
      S.kmap[(size_t)e1 * L + e2] = k;
    }

  // ---- the velocity-independent tables: from the cache, or computed ----
  const int NC = 2 * b + 1;
  if (auto ce = stencil_find(2, n, omega, b, C)) {
    S.kq = ce->kq;
    S.gamma_glob = ce->gamma_glob;
    std::copy(ce->alpha.begin(), ce->alpha.end(), S.alpha);
    std::copy(ce->beta.begin(), ce->beta.end(), S.beta);
    std::copy(ce->alpha_sv.begin(), ce->alpha_sv.end(), S.alpha_sv);
  } else {
    // ---- Green's table k_delta, delta in [0, n+1]^2 (Sec. 1, Sec. 2.1, G1) ----
    const int Q = n + 2;
    S.kq.assign((size_t)Q * Q, cd(0.0));
    parallel_for(Q, [&](int a) {
      for (int c = 0; c <= a; ++c) {
        cd val;
        if (a == 0 && c == 0) {
          const double rad = h / std::sqrt(kPi);
          double j1, y1;
          bessel_j1y1_small(omega * rad, &j1, &y1);
          // k0 = (i pi a / (2 omega)) H1(omega a) - 1/omega^2
          val = cd(0.0, kPi * rad / (2.0 * omega)) * cd(j1, y1) - cd(1.0 / (omega * omega), 0.0);
        } else {
          const double r = std::sqrt((double)a * a + (double)c * c) * h;
          double j0, y0;
          bessel_j0y0(omega * r, &j0, &y0);
          // G = (i/4) H0(omega r) = (i/4)(J0 + i Y0), times h^2
          val = cd(-0.25 * y0, 0.25 * j0) * (h * h);
        }
        S.kq[(size_t)a * Q + c] = val;
        S.kq[(size_t)c * Q + a] = val;
      }
    });
    auto kq = [&](int d1, int d2) { return S.kq[(size_t)std::abs(d1) * Q + std::abs(d2)]; };

    // ---- alpha: streamed QR of K_{mu,mu^c}^H, then the SVD of R (eq. alpha) ----
    {
      const int nt = (int)std::min<unsigned>(worker_count(), 2 * n + 1);
      std::vector<std::vector<cd>> Rs(nt);
      std::vector<int> have(nt, 0);
      parallel_for(nt, [&](int t) {
        std::vector<cd> block;
        block.reserve(64 * 9);
        std::vector<cd> R;
        bool hv = false;
        int rows = 0;
        for (int l1 = -n + t; l1 <= n; l1 += nt)
          for (int l2 = -n; l2 <= n; ++l2) {
            if (std::abs(l1) <= 1 && std::abs(l2) <= 1) continue;
            for (int o = 0; o < 9; ++o) {
              const int j1 = o / 3 - 1, j2 = o % 3 - 1;
              block.push_back(std::conj(kq(j1 - l1, j2 - l2)));
            }
            if (++rows == 64) {
              qr_append(R, block.data(), rows, 9, hv);
              hv = true;
              rows = 0;
              block.clear();
            }
          }
        if (rows) {
          qr_append(R, block.data(), rows, 9, hv);
          hv = true;
        }
        Rs[t] = R;
        have[t] = hv;
      });
      std::vector<cd> R;
      bool hv = false;
      for (int t = 0; t < nt; ++t)
        if (have[t]) {
          qr_append(R, Rs[t].data(), 9, 9, hv);
          hv = true;
        }
      jacobi_min_right_vector(R, 9, 9, S.alpha, S.alpha_sv);
      normalise_phase(S.alpha, 9);
      // beta^* = alpha^* K_{mu,mu}:  beta_l = sum_j conj(k_{j-l}) alpha_j (eq. beta)
      for (int l = 0; l < 9; ++l) {
        cd s(0.0);
        for (int j = 0; j < 9; ++j)
          s += std::conj(kq(j / 3 - l / 3, j % 3 - l % 3)) * S.alpha[j];
        S.beta[l] = s;
      }
    }

    // ---- global PML stencils by per-axis class (eq. gamma) ----
    S.gamma_glob.assign((size_t)NC * NC * 9, cd(0.0));
    for (int c1 = 0; c1 < NC; ++c1)
      for (int c2 = 0; c2 < NC; ++c2) {
        if (c1 == 0 && c2 == 0) continue;
        double os[2][3];
        const int cls[2] = {c1, c2};
        for (int k = 0; k < 2; ++k) {
          const int i = class_index(cls[k], n, b);
          for (int o = 0; o < 3; ++o) os[k][o] = omega_sigma_global(i - 1 + o, n, b, C);
        }
        pml_gamma_2d(omega, omega, h, os, &S.gamma_glob[((size_t)c1 * NC + c2) * 9]);
      }

    stencil_insert(make_entry(2, n, omega, b, C, S.kq, S.gamma_glob, S.alpha, S.beta, S.alpha_sv, 9));
  }

  // ---- slices (readings G8, G18) ----
  if (fronts != 1 && fronts != 2) return "fronts must be 1 or 2";
  S.fronts = fronts;
  S.slices = plan_slices(n, b, w, fronts);
  const int nl = (int)S.slices.size();
  S.nslices = nl;
  for (int k = 0; k < nl; ++k)
    if (S.slices[k].t > 32) {
      std::snprintf(buf, sizeof buf, "slice %d has %d lines; at most 32 are supported (reduce w or b)",
                    S.slices[k].grid, S.slices[k].t);
      return buf;
    }

  // ---- auxiliary PML stencils at the sampled local frequencies (Sec. 2.3) ----
  // Stored for the auxiliary PML before a slice's D_k in its own (local) order;
  // lines after D_k (the two-front middle slice) take the same stencil with
  // the x1 offsets mirrored. Only (depth, class, sample) triples that some
  // auxiliary point uses are built.
  S.gamma_aux.assign((size_t)b * NC * ns * 9, cd(0.0));
  std::vector<char> used((size_t)b * NC * ns, 0);
  for (int k = 0; k < nl; ++k) {
    const SlicePlan& p = S.slices[k];
    const int tw = p.hi - p.lo + 1;
    for (int a = 0; a < p.t; ++a) {
      int q;
      if (a < p.naux)
        q = p.naux - 1 - a;
      else if (a >= p.naux + tw)
        q = a - p.naux - tw;
      else
        continue;
      const int line = p.org + p.dir * a;
      for (int e2 = 0; e2 < L; ++e2) {
        const int c2 = axis_class(e2 - b, n, b);
        const int ks = S.kmap[(size_t)(line + b) * L + e2];
        used[((size_t)q * NC + c2) * ns + ks] = 1;
      }
    }
  }
  std::vector<int> todo;
  for (size_t i = 0; i < used.size(); ++i)
    if (used[i]) todo.push_back((int)i);
  parallel_for((int)todo.size(), [&](int ii) {
    const int id = todo[ii];
    const int ks = id % ns, c2 = (id / ns) % NC, q = id / (ns * NC);
    double os[2][3];
    // x1: auxiliary profile at depths q+1, q, q-1 (offsets -1, 0, +1)
    os[0][0] = omega_sigma_aux(q + 1, b, C);
    os[0][1] = omega_sigma_aux(q, b, C);
    os[0][2] = omega_sigma_aux(q - 1, b, C);
    const int i2 = class_index(c2, n, b);
    for (int o = 0; o < 3; ++o) os[1][o] = omega_sigma_global(i2 - 1 + o, n, b, C);
    const double kappa = std::sqrt(lo + ks * delta);
    pml_gamma_2d(kappa, omega, h, os, &S.gamma_aux[(size_t)id * 9]);
  });
  return "";
}

}  // namespace lsw

namespace lsw {

std::string build_host_setup3(const double* m, int n, double omega, int b, int w, double C, int freq_samples,
                              int max_lines, int max_block, HostSetup3& S) {
  char buf[256];
  if (n < 1) return "n must be >= 1";
  if (!(omega > 0.0) || !std::isfinite(omega)) return "omega must be finite and > 0";
  if (b < 1) return "pml_width must be >= 1";
  if (w < 1) return "layer_thickness must be >= 1";
  if (!(C >= 0.0) || !std::isfinite(C)) return "pml_C must be finite and >= 0";
  const double h = 1.0 / (n + 1);
  if (omega * h / std::sqrt(kPi) > 2.0) return "fewer than ~2 points per wavelength (omega*h/sqrt(pi) > 2)";
  S.n = n;
  S.b = b;
  S.w = w;
  S.omega = omega;
  S.h = h;
  S.C = C;
  S.L = n + 2 + 2 * b;
  const int L = S.L;
  const size_t n3 = (size_t)n * n * n;

  // ---- slabs (reading G8), checked before any of the heavy setup ----
  const int nl = std::max(1, (n + 2) / w);
  S.nslices = nl;
  S.slices.resize(nl);
  for (int k = 0; k < nl; ++k) {
    SlicePlan& p = S.slices[k];
    p.lo = (k == 0) ? -b : k * w;
    p.hi = (k == nl - 1) ? n + 1 + b : (k + 1) * w - 1;
    p.first = (k == 0) ? p.lo : p.lo - b;
    p.t = p.hi - p.first + 1;
    p.naux = p.lo - p.first;
    if (p.t > max_lines) {
      std::snprintf(buf, sizeof buf, "slab %d has %d lines; at most %d are supported (reduce w or b)", k, p.t,
                    max_lines);
      return buf;
    }
    if ((long long)p.t * L > max_block) {
      std::snprintf(buf, sizeof buf,
                    "slab %d has blocks of %lld unknowns (lines x L); at most %d are supported (reduce w or b)", k,
                    (long long)p.t * L, max_block);
      return buf;
    }
  }

  // ---- medium range and local-frequency samples (Sec. 2.3, reading G9) ----
  double mmax = -INFINITY, mmin = INFINITY;
  for (size_t i = 0; i < n3; ++i) {
    if (!std::isfinite(m[i])) return "m has a non-finite value";
    mmax = std::max(mmax, m[i]);
    mmin = std::min(mmin, m[i]);
  }
  if (!(1.0 - mmax > 0.0)) return "max m must be < 1 (the local frequency must be real)";
  const double w2 = omega * omega;
  const double lo = w2 * (1.0 - mmax);
  const double hi = w2 * (1.0 - mmin);
  int ns = freq_samples > 0 ? freq_samples : n;
  if (!(hi > lo)) ns = 1;
  const double delta = ns > 1 ? (hi - lo) / (ns - 1) : 0.0;
  S.ns = ns;
  S.freq_lo = lo;
  S.freq_delta = delta;
  S.kmap.assign((size_t)L * L * L, 0);
  parallel_for(L, [&](int e1) {
    for (int e2 = 0; e2 < L; ++e2)
      for (int e3 = 0; e3 < L; ++e3) {
        const int i1 = e1 - b, i2 = e2 - b, i3 = e3 - b;
        double mp = 0.0;
        if (i1 >= 1 && i1 <= n && i2 >= 1 && i2 <= n && i3 >= 1 && i3 <= n)
          mp = m[((size_t)(i1 - 1) * n + (i2 - 1)) * n + (i3 - 1)];
        S.kmap[((size_t)e1 * L + e2) * L + e3] = sample_index(mp, w2, lo, delta, ns);
      }
  });

  // ---- the velocity-independent tables: from the cache, or computed ----
  const int NC = 2 * b + 1;
  if (auto ce = stencil_find(3, n, omega, b, C)) {
    S.kq = ce->kq;
    S.gamma_glob = ce->gamma_glob;
    std::copy(ce->alpha.begin(), ce->alpha.end(), S.alpha);
    std::copy(ce->beta.begin(), ce->beta.end(), S.beta);
    std::copy(ce->alpha_sv.begin(), ce->alpha_sv.end(), S.alpha_sv);
  } else {
    // ---- Green's table (Sec. 1, Sec. 2.1, reading G1) ----
    S.kq = green3_octant(n, omega);
    const int Q = n + 2;
    auto kq = [&](int d1, int d2, int d3) {
      return S.kq[((size_t)std::abs(d1) * Q + std::abs(d2)) * Q + std::abs(d3)];
    };

    // ---- alpha: streamed QR of K_{mu,mu^c}^H, then the SVD of R (eq. alpha) ----
    {
      const int nt = (int)std::min<unsigned>(worker_count(), 2 * n + 1);
      std::vector<std::vector<cd>> Rs(nt);
      std::vector<int> have(nt, 0);
      parallel_for(nt, [&](int t) {
        constexpr int kRows = 128;
        std::vector<cd> block;
        block.reserve((size_t)kRows * 27);
        std::vector<cd> R;
        bool hv = false;
        int rows = 0;
        for (int l1 = -n + t; l1 <= n; l1 += nt)
          for (int l2 = -n; l2 <= n; ++l2)
            for (int l3 = -n; l3 <= n; ++l3) {
              if (std::abs(l1) <= 1 && std::abs(l2) <= 1 && std::abs(l3) <= 1) continue;
              for (int o = 0; o < 27; ++o)
                block.push_back(std::conj(kq(o / 9 - 1 - l1, (o / 3) % 3 - 1 - l2, o % 3 - 1 - l3)));
              if (++rows == kRows) {
                qr_append(R, block.data(), rows, 27, hv);
                hv = true;
                rows = 0;
                block.clear();
              }
            }
        if (rows) {
          qr_append(R, block.data(), rows, 27, hv);
          hv = true;
        }
        Rs[t] = R;
        have[t] = hv;
      });
      std::vector<cd> R;
      bool hv = false;
      for (int t = 0; t < nt; ++t)
        if (have[t]) {
          qr_append(R, Rs[t].data(), 27, 27, hv);
          hv = true;
        }
      jacobi_min_right_vector(R, 27, 27, S.alpha, S.alpha_sv);
      normalise_phase(S.alpha, 27);
      // beta^* = alpha^* K_{mu,mu}:  beta_l = sum_j conj(k_{j-l}) alpha_j (eq. beta)
      for (int l = 0; l < 27; ++l) {
        cd s(0.0);
        for (int j = 0; j < 27; ++j)
          s += std::conj(kq(j / 9 - l / 9, (j / 3) % 3 - (l / 3) % 3, j % 3 - l % 3)) * S.alpha[j];
        S.beta[l] = s;
      }
    }

    // ---- global PML stencils by per-axis class (eq. gamma, Sec. 3.1) ----
    S.gamma_glob.assign((size_t)NC * NC * NC * 27, cd(0.0));
    parallel_for(NC * NC * NC, [&](int id) {
      const int cls[3] = {id / (NC * NC), (id / NC) % NC, id % NC};
      if (!cls[0] && !cls[1] && !cls[2]) return;
      double os[3][3];
      for (int k = 0; k < 3; ++k) {
        const int i = class_index(cls[k], n, b);
        for (int o = 0; o < 3; ++o) os[k][o] = omega_sigma_global(i - 1 + o, n, b, C);
      }
      pml_gamma_3d(omega, omega, h, os, &S.gamma_glob[(size_t)id * 27]);
    });
    stencil_insert(make_entry(3, n, omega, b, C, S.kq, S.gamma_glob, S.alpha, S.beta, S.alpha_sv, 27));
  }

  // ---- auxiliary PML stencils at the sampled local frequencies (Sec. 2.3) ----
  const size_t naux_keys = (size_t)b * NC * NC * ns;
  S.gamma_aux.assign(naux_keys * 27, cd(0.0));
  std::vector<char> used(naux_keys, 0);
  for (int k = 1; k < nl; ++k) {
    const SlicePlan& p = S.slices[k];
    for (int q = 0; q < b; ++q) {
      const int line = p.lo - 1 - q;
      for (int e2 = 0; e2 < L; ++e2) {
        const int c2 = axis_class(e2 - b, n, b);
        for (int e3 = 0; e3 < L; ++e3) {
          const int c3 = axis_class(e3 - b, n, b);
          const int ks = S.kmap[((size_t)(line + b) * L + e2) * L + e3];
          used[(((size_t)q * NC + c2) * NC + c3) * ns + ks] = 1;
        }
      }
    }
  }
  std::vector<size_t> todo;
  for (size_t i = 0; i < used.size(); ++i)
    if (used[i]) todo.push_back(i);
  parallel_for((int)todo.size(), [&](int ii) {
    const size_t id = todo[ii];
    const int ks = (int)(id % ns);
    const int c3 = (int)((id / ns) % NC), c2 = (int)((id / ((size_t)ns * NC)) % NC);
    const int q = (int)(id / ((size_t)ns * NC * NC));
    double os[3][3];
    os[0][0] = omega_sigma_aux(q + 1, b, C);
    os[0][1] = omega_sigma_aux(q, b, C);
    os[0][2] = omega_sigma_aux(q - 1, b, C);
    const int cls[2] = {c2, c3};
    for (int k = 0; k < 2; ++k) {
      const int i = class_index(cls[k], n, b);
      for (int o = 0; o < 3; ++o) os[k + 1][o] = omega_sigma_global(i - 1 + o, n, b, C);
    }
    const double kappa = std::sqrt(lo + ks * delta);
    pml_gamma_3d(kappa, omega, h, os, &S.gamma_aux[id * 27]);
  });
  return "";
}

}  // namespace lsw
