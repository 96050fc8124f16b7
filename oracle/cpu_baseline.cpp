// FP64 CPU destriper on all host cores: the timing baseline beside the GPU
// library (TEST INFRASTRUCTURE, like the NumPy oracle in this directory:
// only the tests and the benchmark call it; it shares no code with the GPU
// path).  C++17 + OpenMP.
//
// What it computes (Algorithm section of Zonca et al., arXiv:1309.5609):
//   data model d = A m + F a + w (Eqs. 2, 7, 8) for the streams T, q, u of
//   one channel, pointing rows A_T = (1, 0, 0), A_q = (0, cos 2psi, sin 2psi),
//   A_u = (0, -sin 2psi, cos 2psi) (Eqs. 3-6), baseline of sample t = t / L;
//   per pixel M = sum_t sum_k w_k A_k^T A_k, block diagonal T | QU; a T block
//   is valid with hits, a QU block when its eigenvalue ratio >= rcond; a
//   sample enters a stream only on a valid block;
//   the destriping equation F^T Z F a = F^T Z d (Eq. 13), Z = W (I - A M^-1
//   A^T W) on valid samples, by conjugate gradient with the Jacobi
//   preconditioner 1 / (w_k n_valid) from a = 0, stopping when
//   ||r|| <= tol ||b||; one T null vector per connected part of the
//   baseline-pixel graph is projected out of b and of every K p, and the T
//   baselines are reported with zero mean per part;
//   maps m = M^-1 A^T W (d - F a) (Eqs. 10-12).
//
// Parallel layout (the local-map / global-map scheme of the paper's MPI
// implementation, at thread level): each thread bins its share of the
// samples into a private full map, the private maps are summed pixel by
// pixel, and the rescan runs over baselines.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

struct Problem {
  int64_t n_t, n_pix, L, n_b;
  int has_T, has_QU, ns;  // stream rows: T at 0 when present, then q, u
  const int32_t* pix;
  std::vector<double> c, s;  // cos 2psi, sin 2psi per sample
  double w[3];
  // per pixel
  std::vector<int64_t> hits;
  std::vector<double> inv;  // [n_pix][4]: 1/M_TT, then the QU inverse (qq, qu, uu)
  std::vector<uint8_t> valid;  // bit 0: T block, bit 1: QU block
  // per baseline and stream row
  std::vector<double> nval;  // [ns][n_b]
  std::vector<int64_t> comp;  // component of each baseline (-1: no valid T sample)
  int64_t n_comp = 0;
  int threads = 1;
};

int row_T(const Problem& P) { return P.has_T ? 0 : -1; }
int row_q(const Problem& P) { return P.has_QU ? (P.has_T ? 1 : 0) : -1; }

bool t_ok(const Problem& P, int64_t t) {
  const int p = P.pix[t];
  return p >= 0 && (P.valid[p] & 1);
}
bool qu_ok(const Problem& P, int64_t t) {
  const int p = P.pix[t];
  return p >= 0 && (P.valid[p] & 2);
}

int64_t find(std::vector<int64_t>& par, int64_t x) {
  while (par[x] != x) {
    par[x] = par[par[x]];
    x = par[x];
  }
  return x;
}

void setup(Problem& P, const double* psi, double rcond) {
  const int64_t n = P.n_pix;
  P.hits.assign(n, 0);
  std::vector<double> M(4 * n, 0.0);  // M_TT, M_qq, M_qu, M_uu
  if (P.has_QU) {
    P.c.resize(P.n_t);
    P.s.resize(P.n_t);
#pragma omp parallel for schedule(static) num_threads(P.threads)
    for (int64_t t = 0; t < P.n_t; ++t) {
      P.c[t] = std::cos(2.0 * psi[t]);
      P.s[t] = std::sin(2.0 * psi[t]);
    }
  }
  const int nth = P.threads;
  std::vector<std::vector<double>> lm(nth);
  std::vector<std::vector<int64_t>> lh(nth);
#pragma omp parallel num_threads(nth)
  {
    const int id = omp_get_thread_num();
    std::vector<double>& m = lm[id];
    std::vector<int64_t>& h = lh[id];
    m.assign(4 * n, 0.0);
    h.assign(n, 0);
#pragma omp for schedule(static)
    for (int64_t t = 0; t < P.n_t; ++t) {
      const int p = P.pix[t];
      if (p < 0) continue;
      h[p] += 1;
      if (P.has_T) m[4 * p] += P.w[0];
      if (P.has_QU) {
        const double c = P.c[t], s = P.s[t];
        m[4 * p + 1] += P.w[1] * c * c + P.w[2] * s * s;
        m[4 * p + 2] += (P.w[1] - P.w[2]) * c * s;
        m[4 * p + 3] += P.w[1] * s * s + P.w[2] * c * c;
      }
    }
  }
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t p = 0; p < n; ++p) {
    for (int i = 0; i < nth; ++i) {
      P.hits[p] += lh[i][p];
      for (int j = 0; j < 4; ++j) M[4 * p + j] += lm[i][4 * p + j];
    }
  }
  P.inv.assign(4 * n, 0.0);
  P.valid.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) {
    if (P.hits[p] == 0) continue;
    if (P.has_T) {
      P.valid[p] |= 1;
      P.inv[4 * p] = 1.0 / M[4 * p];
    }
    if (P.has_QU) {
      const double a = M[4 * p + 1], b = M[4 * p + 2], d = M[4 * p + 3];
      const double half = 0.5 * (a - d), rad = std::sqrt(half * half + b * b);
      const double lmax = 0.5 * (a + d) + rad, lmin = 0.5 * (a + d) - rad;
      if (lmax > 0.0 && lmin > 0.0 && lmin / lmax >= rcond) {
        const double det = a * d - b * b;
        P.valid[p] |= 2;
        P.inv[4 * p + 1] = d / det;
        P.inv[4 * p + 2] = -b / det;
        P.inv[4 * p + 3] = a / det;
      }
    }
  }
  P.nval.assign(P.ns * P.n_b, 0.0);
  const int rT = row_T(P), rq = row_q(P);
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t b = 0; b < P.n_b; ++b) {
    const int64_t t1 = std::min(P.n_t, (b + 1) * P.L);
    double nT = 0.0, nQ = 0.0;
    for (int64_t t = b * P.L; t < t1; ++t) {
      nT += t_ok(P, t) ? 1.0 : 0.0;
      nQ += qu_ok(P, t) ? 1.0 : 0.0;
    }
    if (rT >= 0) P.nval[rT * P.n_b + b] = nT;
    if (rq >= 0) {
      P.nval[rq * P.n_b + b] = nQ;
      P.nval[(rq + 1) * P.n_b + b] = nQ;
    }
  }
  // connected parts of the baseline-pixel graph over T-valid samples
  P.comp.assign(P.n_b, -1);
  if (P.has_T) {
    std::vector<int64_t> par(P.n_b + n);
    std::iota(par.begin(), par.end(), 0);
    for (int64_t t = 0; t < P.n_t; ++t) {
      if (!t_ok(P, t)) continue;
      const int64_t x = find(par, t / P.L), y = find(par, P.n_b + P.pix[t]);
      if (x != y) par[std::max(x, y)] = std::min(x, y);
    }
    std::vector<int64_t> id(P.n_b + n, -1);
    for (int64_t b = 0; b < P.n_b; ++b) {
      if (P.nval[b] == 0.0) continue;
      const int64_t r = find(par, b);
      if (id[r] < 0) id[r] = P.n_comp++;
      P.comp[b] = id[r];
    }
  }
}

// s[p] = sum over valid samples of w_k A_k(t)^T x_k(t), x = (tod or 0) - F v
// (v may be NULL); thread-private maps summed per pixel.
void bin(const Problem& P, const double* tod, const double* v, std::vector<double>& s,
         std::vector<std::vector<double>>& lm) {
  const int64_t n = P.n_pix;
  const int rT = row_T(P), rq = row_q(P);
  const int nth = P.threads;
#pragma omp parallel num_threads(nth)
  {
    std::vector<double>& m = lm[omp_get_thread_num()];
    std::fill(m.begin(), m.end(), 0.0);
#pragma omp for schedule(static)
    for (int64_t t = 0; t < P.n_t; ++t) {
      const int p = P.pix[t];
      if (p < 0) continue;
      const int64_t b = t / P.L;
      if (rT >= 0 && (P.valid[p] & 1)) {
        double x = tod ? tod[rT * P.n_t + t] : 0.0;
        if (v) x -= v[rT * P.n_b + b];
        m[3 * p] += P.w[0] * x;
      }
      if (rq >= 0 && (P.valid[p] & 2)) {
        double xq = tod ? tod[rq * P.n_t + t] : 0.0, xu = tod ? tod[(rq + 1) * P.n_t + t] : 0.0;
        if (v) {
          xq -= v[rq * P.n_b + b];
          xu -= v[(rq + 1) * P.n_b + b];
        }
        const double c = P.c[t], sn = P.s[t];
        m[3 * p + 1] += P.w[1] * c * xq - P.w[2] * sn * xu;
        m[3 * p + 2] += P.w[1] * sn * xq + P.w[2] * c * xu;
      }
    }
#pragma omp for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int i = 0; i < nth; ++i) {
        a0 += lm[i][3 * p];
        a1 += lm[i][3 * p + 1];
        a2 += lm[i][3 * p + 2];
      }
      s[3 * p] = P.inv[4 * p] * a0;
      s[3 * p + 1] = P.inv[4 * p + 1] * a1 + P.inv[4 * p + 2] * a2;
      s[3 * p + 2] = P.inv[4 * p + 2] * a1 + P.inv[4 * p + 3] * a2;
    }
  }
}

// out_k[b] = sum_{t in b, valid} w_k (x_k(t) - A_k(t) m[p(t)]), x = (tod or 0) - F v.
void rescan(const Problem& P, const double* tod, const double* v, const std::vector<double>& m, double* out) {
  const int rT = row_T(P), rq = row_q(P);
#pragma omp parallel for schedule(static) num_threads(P.threads)
  for (int64_t b = 0; b < P.n_b; ++b) {
    const int64_t t1 = std::min(P.n_t, (b + 1) * P.L);
    double aT = 0.0, aq = 0.0, au = 0.0;
    for (int64_t t = b * P.L; t < t1; ++t) {
      const int p = P.pix[t];
      if (p < 0) continue;
      if (rT >= 0 && (P.valid[p] & 1)) {
        double x = tod ? tod[rT * P.n_t + t] : 0.0;
        if (v) x -= v[rT * P.n_b + b];
        aT += x - m[3 * p];
      }
      if (rq >= 0 && (P.valid[p] & 2)) {
        double xq = tod ? tod[rq * P.n_t + t] : 0.0, xu = tod ? tod[(rq + 1) * P.n_t + t] : 0.0;
        if (v) {
          xq -= v[rq * P.n_b + b];
          xu -= v[(rq + 1) * P.n_b + b];
        }
        const double c = P.c[t], sn = P.s[t];
        aq += xq - (c * m[3 * p + 1] + sn * m[3 * p + 2]);
        au += xu - (-sn * m[3 * p + 1] + c * m[3 * p + 2]);
      }
    }
    if (rT >= 0) out[rT * P.n_b + b] = P.w[0] * aT;
    if (rq >= 0) {
      out[rq * P.n_b + b] = P.w[1] * aq;
      out[(rq + 1) * P.n_b + b] = P.w[2] * au;
    }
  }
}

// Remove the T mean of each connected part (rows other than T untouched).
void project(const Problem& P, double* x) {
  if (!P.has_T || P.n_comp == 0) return;
  std::vector<double> sum(P.n_comp, 0.0), cnt(P.n_comp, 0.0);
  for (int64_t b = 0; b < P.n_b; ++b)
    if (P.comp[b] >= 0) {
      sum[P.comp[b]] += x[b];
      cnt[P.comp[b]] += 1.0;
    }
  for (int64_t b = 0; b < P.n_b; ++b)
    if (P.comp[b] >= 0) x[b] -= sum[P.comp[b]] / cnt[P.comp[b]];
}

double dot(const Problem& P, const double* a, const double* b, int64_t N) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static) num_threads(P.threads)
  for (int64_t i = 0; i < N; ++i) s += a[i] * b[i];
  return s;
}

Problem make(int64_t n_t, int64_t n_pix, int64_t L, int streams, const int32_t* pix, const double* w, int threads) {
  Problem P;
  P.n_t = n_t;
  P.n_pix = n_pix;
  P.L = L;
  P.n_b = (n_t + L - 1) / L;
  P.has_T = (streams & 1) != 0;
  P.has_QU = (streams & 6) != 0;
  P.ns = (P.has_T ? 1 : 0) + (P.has_QU ? 2 : 0);
  P.pix = pix;
  for (int k = 0; k < 3; ++k) P.w[k] = w[k];
  P.threads = threads > 0 ? threads : omp_get_max_threads();
  return P;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

// Threads OpenMP would use by default.
int cpu_destripe_max_threads(void) { return omp_get_max_threads(); }

// Full solve.  streams: 1 (T), 6 (QU) or 7 (TQU); tod [n_streams][n_t];
// w [3] (T, q, u); outputs baselines [n_streams][n_b] (canonical), map
// [n_pix][3] destriped (or NULL), hits [n_pix] (or NULL).  info [6]:
// setup seconds, loop seconds, total seconds, iterations, relative residual,
// threads.  Returns 0, or 1 when max_iter was reached.
int cpu_destripe_solve(int64_t n_t, int64_t n_pix, int64_t L, int streams, const int32_t* pix, const double* psi,
                       const double* tod, const double* w, double rcond, double tol, int max_iter, int threads,
                       double* baselines, double* map, int64_t* hits, double* info) {
  const double t0 = now();
  Problem P = make(n_t, n_pix, L, streams, pix, w, threads);
  setup(P, psi, rcond);
  const int64_t N = P.ns * P.n_b;
  std::vector<std::vector<double>> lm(P.threads, std::vector<double>(3 * n_pix));
  std::vector<double> m(3 * n_pix), b(N), a(N, 0.0), r(N), z(N), p(N), q(N), J(N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    const int64_t bb = i % P.n_b;
    const int row = (int)(i / P.n_b);
    const int k = (P.has_T && row == 0) ? 0 : (row == row_q(P) ? 1 : 2);
    const double d = P.w[k] * P.nval[i];
    J[i] = d > 0.0 ? 1.0 / d : 0.0;
    (void)bb;
  }
  bin(P, tod, nullptr, m, lm);
  rescan(P, tod, nullptr, m, b.data());
  project(P, b.data());
  const double t1 = now();
  const double bn = std::sqrt(dot(P, b.data(), b.data(), N));
  r = b;
  for (int64_t i = 0; i < N; ++i) z[i] = J[i] * r[i];
  p = z;
  double rz = dot(P, r.data(), z.data(), N);
  int it = 0;
  double rel = bn > 0.0 ? 1.0 : 0.0;
  while (bn > 0.0 && rel > tol && it < max_iter) {
    // q = P K p: bin F p (x = -F p), rescan, then negate
    bin(P, nullptr, p.data(), m, lm);
    rescan(P, nullptr, p.data(), m, q.data());
    for (int64_t i = 0; i < N; ++i) q[i] = -q[i];
    project(P, q.data());
    const double pq = dot(P, p.data(), q.data(), N);
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    for (int64_t i = 0; i < N; ++i) {
      a[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ++it;
    rel = std::sqrt(dot(P, r.data(), r.data(), N)) / bn;
    if (rel <= tol) break;
    for (int64_t i = 0; i < N; ++i) z[i] = J[i] * r[i];
    const double rz2 = dot(P, r.data(), z.data(), N);
    const double beta = rz2 / rz;
    rz = rz2;
    for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
  }
  const double t2 = now();
  // canonical T baselines: zero mean per part, zero without valid samples
  if (P.has_T) {
    project(P, a.data());
    for (int64_t i = 0; i < P.n_b; ++i)
      if (P.comp[i] < 0) a[i] = 0.0;
  }
  std::memcpy(baselines, a.data(), N * sizeof(double));
  if (map) {
    bin(P, tod, a.data(), m, lm);
    std::memcpy(map, m.data(), 3 * n_pix * sizeof(double));
  }
  if (hits) std::memcpy(hits, P.hits.data(), n_pix * sizeof(int64_t));
  const double t3 = now();
  info[0] = t1 - t0;
  info[1] = t2 - t1;
  info[2] = t3 - t0;
  info[3] = it;
  info[4] = rel;
  info[5] = P.threads;
  return rel <= tol ? 0 : 1;
}

// K v (Eq. 13 operator, no projection) repeated `reps` times after the setup;
// out [n_streams][n_b].  info [3]: setup seconds, seconds per application,
// threads.
int cpu_destripe_apply(int64_t n_t, int64_t n_pix, int64_t L, int streams, const int32_t* pix, const double* psi,
                       const double* w, double rcond, int threads, const double* v, int reps, double* out,
                       double* info) {
  const double t0 = now();
  Problem P = make(n_t, n_pix, L, streams, pix, w, threads);
  setup(P, psi, rcond);
  std::vector<std::vector<double>> lm(P.threads, std::vector<double>(3 * n_pix));
  std::vector<double> m(3 * n_pix);
  const int64_t N = P.ns * P.n_b;
  const double t1 = now();
  for (int k = 0; k < std::max(reps, 1); ++k) {
    bin(P, nullptr, v, m, lm);
    rescan(P, nullptr, v, m, out);
    for (int64_t i = 0; i < N; ++i) out[i] = -out[i];
  }
  const double t2 = now();
  info[0] = t1 - t0;
  info[1] = (t2 - t1) / std::max(reps, 1);
  info[2] = P.threads;
  return 0;
}

}  // extern "C"
