// Outer loop of ManiDSDP (Algorithm alg1), the Riemannian trust-region
// subproblem solver with truncated CG, and a Lanczos eigensolver for the
// dual certificate X = Xt + D - Diag(z).  Host C++ drives the iteration; every
// vector operation is a kernel on the problem's stream, and the host reads
// back only the scalars a decision needs (one synchronisation per tCG step).
//
// Readings of points the paper leaves open (same as the oracle's):
//  * RTR constants rho' = 0.1, kappa = 0.1, theta = 1, Delta_bar = pi sqrt(n),
//    Delta_0 = Delta_bar / 8 (Absil-Baker-Gallivan trust region);
//  * inner tolerance of subproblem k: max(gtol_min, min(gtol0, gtol_ratio ||R^k|| / (1 + ||b||)))
//    (gtol0 at k = 0), the scaled primal residual that eq. sec5:eq1 weighs
//    against ||grad||, so both sides of that rule are on one scale: sigma
//    rises when an outer step leaves the primal residual about where it was
//    and falls when RTR stops short of its tolerance.  With gtol_ratio <= 0
//    the older form max(gtol_min, min(gtol0, 0.1 eta_max, gtol_decay * previous))
//    is used.  Optional stall cap (gtol_stall > 0): after an RTR call that
//    starts below its tolerance every later tolerance is at most
//    gtol_stall ||grad||;
//  * the certificate Lanczos (deflated against range(Y), see the outer loop)
//    starts from the previous Ritz vector plus a random component and stops
//    when the error estimate of theta_min (residual, or residual^2 / certified
//    gap) is below eig_tol (1 + |theta_max|), or once theta_min minus that
//    estimate is >= 0; when it stops unconverged, eta_d uses theta_min minus
//    the estimate, and when eta_d is then at least half the largest residual
//    the step budget of the next eigensolve doubles (up to n);
//  * eq. sec5:eq1 after every outer step, except that (option sigma_hold, on
//    by default) its decrease branch is skipped after an RTR call that stopped
//    at its iteration budget: ||grad|| then measures an unfinished inner
//    solve, not a dual residual, and with a 10-step budget the printed rule
//    drives sigma down on every step of a large instance;
//  * inner budget: rtr_maxiter (10) RTR iterations of at most tcg_maxinner
//    (200) truncated-CG steps per subproblem until eta_max < polish_eta
//    (1e-4); rtr_maxiter_polish (50) of at most tcg_maxinner_polish (1000)
//    after that, when the HVPs also switch to FP64 (polish_fp64);
//  * carried direction: backtracking t = sqrt(n), sqrt(n)/2, ... along
//    R_[Y,0](t [0, v]) until Psi_k decreases, then RTR.  By default the
//    direction and its zero columns are added after every outer step whose
//    certificate curvature is below -max(1e-12, tol) (1 + |lambda_max|)
//    (step 9 of Algorithm alg1); escape_when_solved restricts that to steps
//    whose RTR call reached its tolerance;
//  * rank rule: drop singular directions of Y below tau_rank * s_1 (1e-7), then add
//    one zero column per carried negative eigenvector (at most n_neg = 15 per
//    outer step, p <= p_max): near the solution the factor is one column plus
//    the carried ones, and 16 columns fill the 16-column MFMA tiles exactly
//    (17 are staged as 32 and cost 1.8 times as much per HVP);
//  * sigma rule eq. sec5:eq1 with ||R|| = ||Q(Z)||_F and the final ||grad||;
//  * rank-one compression (Theorem thm:finite-locking, Remark
//    rem:inexact-near-locking): once eta_max < round_eta and s_2 <= round_gap
//    s_1, eq. res is also evaluated at Y1 = sign(Y v_1) with the current
//    multiplier and no multiplier step; the solve ends there when that point
//    meets the tolerance;
//  * a solve ends only on an eta_d from a verify eigensolve (random start,
//    residual error, no early stop; see certificate_spectrum).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <utility>
#include <vector>

#include "mdsdp_internal.hpp"

namespace mdsdp {

namespace {

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

#define CHK(x)                         \
  do {                                 \
    mdsdp_status st__ = (x);           \
    if (st__ != MDSDP_OK) return st__; \
  } while (0)

// ---- small host linear algebra ------------------------------------------------

// Symmetric eigen-decomposition of a k x k row-major matrix A in O(k^3):
// Householder reduction to tridiagonal form T = Q^T A Q, then the implicit-
// shift QL iteration on T with the rotations accumulated into Q.  On return
// w holds the eigenvalues and the columns of V (row-major k x k) the
// eigenvectors; A is overwritten.
void sym_eig(int k, double* A, double* w, double* V) {
  std::vector<double> e(k, 0.0), v(k), pv(k), qv(k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) V[i * k + j] = (i == j) ? 1.0 : 0.0;
  // Householder steps: zero column i below the subdiagonal
  for (int i = 0; i + 2 < k; ++i) {
    const int m = k - i - 1;  // length of x = A[i+1 .., i]
    double nx = 0.0;
    for (int r = 0; r < m; ++r) nx += A[(i + 1 + r) * k + i] * A[(i + 1 + r) * k + i];
    nx = sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = A[(i + 1) * k + i];
    const double alpha = x0 >= 0.0 ? -nx : nx;
    for (int r = 0; r < m; ++r) v[r] = A[(i + 1 + r) * k + i];
    v[0] -= alpha;
    double nv = 0.0;
    for (int r = 0; r < m; ++r) nv += v[r] * v[r];
    nv = sqrt(nv);
    if (nv == 0.0) continue;
    for (int r = 0; r < m; ++r) v[r] /= nv;
    // trailing block B -> B - 2 (v w^T + w v^T), w = B v - (v^T B v) v
    for (int r = 0; r < m; ++r) {
      double acc = 0.0;
      for (int c = 0; c < m; ++c) acc += A[(i + 1 + r) * k + (i + 1 + c)] * v[c];
      pv[r] = acc;
    }
    double K = 0.0;
    for (int r = 0; r < m; ++r) K += v[r] * pv[r];
    for (int r = 0; r < m; ++r) qv[r] = pv[r] - K * v[r];
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) A[(i + 1 + r) * k + (i + 1 + c)] -= 2.0 * (v[r] * qv[c] + qv[r] * v[c]);
    A[(i + 1) * k + i] = A[i * k + i + 1] = alpha;
    for (int r = 1; r < m; ++r) A[(i + 1 + r) * k + i] = A[i * k + i + 1 + r] = 0.0;
    // Q <- Q H on columns i+1 ..
    for (int r = 0; r < k; ++r) {
      double acc = 0.0;
      for (int c = 0; c < m; ++c) acc += V[r * k + i + 1 + c] * v[c];
      for (int c = 0; c < m; ++c) V[r * k + i + 1 + c] -= 2.0 * acc * v[c];
    }
  }
  for (int i = 0; i < k; ++i) w[i] = A[i * k + i];
  for (int i = 0; i + 1 < k; ++i) e[i] = A[(i + 1) * k + i];
  // implicit-shift QL on (w, e); e[i] couples i and i + 1
  for (int l = 0; l < k; ++l) {
    for (int iter = 0; iter < 60; ++iter) {
      int m = l;
      for (; m + 1 < k; ++m) {
        const double dd = fabs(w[m]) + fabs(w[m + 1]);
        if (fabs(e[m]) <= 1e-15 * dd) break;
      }
      if (m == l) break;
      double g = (w[l + 1] - w[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = w[m] - w[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool early = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          w[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = w[i + 1] - p;
        r = (w[i] - g) * s + 2.0 * c * b;
        p = s * r;
        w[i + 1] = g + p;
        g = c * r - b;
        for (int row = 0; row < k; ++row) {
          const double f2 = V[row * k + i + 1];
          V[row * k + i + 1] = s * V[row * k + i] + c * f2;
          V[row * k + i] = c * V[row * k + i] - s * f2;
        }
      }
      if (early) continue;
      w[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
}

// number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm)
int sturm_count(int k, const double* a, const double* b, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    if (q == 0.0) q = 1e-300;
    q = a[i] - x - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// j-th smallest eigenvalue (0-based) by bisection
double tridiag_eig(int k, const double* a, const double* b, int j) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const double span = std::max(1e-300, hi - lo);
  lo -= 1e-12 * span;
  hi += 1e-12 * span;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(k, a, b, mid) > j)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// eigenvector of the tridiagonal for eigenvalue theta by inverse iteration
void tridiag_evec(int k, const double* a, const double* b, double theta, std::vector<double>& s) {
  s.assign(k, 1.0 / sqrt((double)k));
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, fabs(a[i]) + (i + 1 < k ? fabs(b[i]) : 0.0));
  const double shift = theta - 1e-13 * std::max(scale, 1e-300);
  std::vector<double> c(k), d(k), x(k);
  for (int it = 0; it < 4; ++it) {
    // solve (T - shift I) x = s with partial-pivoting-free Thomas (shifted below
    // the spectrum edge the system is definite enough for the extreme pair)
    for (int i = 0; i < k; ++i) {
      d[i] = a[i] - shift;
      c[i] = (i + 1 < k) ? b[i] : 0.0;
    }
    x = s;
    for (int i = 1; i < k; ++i) {
      double piv = d[i - 1];
      if (fabs(piv) < 1e-300) piv = 1e-300;
      const double mlt = b[i - 1] / piv;
      d[i] -= mlt * c[i - 1];
      x[i] -= mlt * x[i - 1];
    }
    double piv = d[k - 1];
    if (fabs(piv) < 1e-300) piv = 1e-300;
    x[k - 1] /= piv;
    for (int i = k - 2; i >= 0; --i) {
      double pv = d[i];
      if (fabs(pv) < 1e-300) pv = 1e-300;
      x[i] = (x[i] - c[i] * x[i + 1]) / pv;
    }
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
    for (int i = 0; i < k; ++i) s[i] = x[i] / nrm;
  }
}

uint64_t splitmix(uint64_t& st) {
  uint64_t z = (st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void gaussian_fill(uint64_t seed, std::vector<double>& v) {
  uint64_t st = seed;
  for (size_t i = 0; i < v.size(); i += 2) {
    const double u1 = ((splitmix(st) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    v[i] = r * cos(2.0 * M_PI * u2);
    if (i + 1 < v.size()) v[i + 1] = r * sin(2.0 * M_PI * u2);
  }
}

// ---- device scalar helpers ----------------------------------------------------

mdsdp_status dots(mdsdp_problem P, int npairs, const double* const* a, const double* const* b, long long len,
                  double* host, hipStream_t s) {
  DotPtrs dp{};
  for (int i = 0; i < npairs; ++i) {
    dp.a[i] = a[i];
    dp.b[i] = b[i];
  }
  double* out_dev = P->scal + SC_DOTS;
  CHK(vec_dots(dp, npairs, len, out_dev, P->dotpart, P->dot_nblk, s));
  MDSDP_HIP(hipMemcpyAsync(P->hbuf, out_dev, npairs * sizeof(double), hipMemcpyDeviceToHost, s));
  MDSDP_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < npairs; ++i) host[i] = P->hbuf[i];
  return MDSDP_OK;
}

// pinned read-back buffer: [0, 64) scalars, [64, HBUF_LEN) small arrays
mdsdp_status read_dev(mdsdp_problem P, const double* dev, int cnt, double* host, hipStream_t s) {
  if (cnt > HBUF_LEN - 64) {
    set_error("read_dev: too many values");
    return MDSDP_EINVAL;
  }
  MDSDP_HIP(hipMemcpyAsync(P->hbuf + 64, dev, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  MDSDP_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < cnt; ++i) host[i] = P->hbuf[64 + i];
  return MDSDP_OK;
}

struct Work {
  int n = 0;
  double* buf = nullptr;
  double *Ynew, *g, *gnew, *eta, *Heta, *r, *d, *Hd, *U, *tmp, *part, *dpart, *rrb, *qc;
  TcgIter it2;  // the second truncated-CG iterate (double buffering)
  hipEvent_t ev[2] = {nullptr, nullptr};
  mdsdp_status init(int n_) {
    n = n_;
    const size_t vec = (size_t)n * PMAX;
    const size_t npart = (size_t)n / 4 + 64;  // tCG partials: one per 256 threads of 64-lane rows
    hipError_t e = hipMalloc((void**)&buf, (15 * vec + 2 * npart + 96 + PMAX) * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(solver work)");
    double* p = buf;
    Ynew = p; p += vec;
    g = p; p += vec;
    gnew = p; p += vec;
    eta = p; p += vec;
    Heta = p; p += vec;
    r = p; p += vec;
    d = p; p += vec;
    Hd = p; p += vec;
    U = p; p += vec;
    tmp = p; p += vec;
    it2.eta = p; p += vec;
    it2.Heta = p; p += vec;
    it2.r = p; p += vec;
    it2.d = p; p += vec;
    it2.Hd = p; p += vec;
    part = p; p += npart;
    dpart = p; p += npart;
    rrb = p;  // 96 doubles of tCG scalars, then PMAX of deflation coefficients
    qc = p + 96;
    for (auto& x : ev)
      if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    return MDSDP_OK;
  }
  ~Work() {
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    if (buf) (void)hipFree(buf);
  }
};

struct Counters {
  long long hvps = 0, cost_grads = 0, rtr_iters = 0, eig_iters = 0;
  double t_eval = 0, t_hvp = 0, t_eig = 0, t_update = 0;
};

// cost (and optionally Riemannian gradient) at Y; returns f on the host
mdsdp_status eval(mdsdp_problem P, int p, const double* Y, double* rgrad, double* f, Counters& C, hipStream_t s) {
  auto t0 = clk::now();
  CHK(mdsdp_cost_grad(P, p, Y, P->scal + SC_FOUT, nullptr, rgrad, s));
  CHK(read_dev(P, P->scal + SC_FOUT, 1, f, s));
  C.cost_grads++;
  C.t_eval += secs(t0, clk::now());
  return MDSDP_OK;
}

// ---- truncated CG ---------------------------------------------------------------
enum { TCG_NEG = 0, TCG_BOUND = 1, TCG_CONV = 2, TCG_MAXIT = 3 };

mdsdp_status tcg(mdsdp_problem P, int p, const double* Y, const double* g, double gn, double Delta, int prec,
                 int maxinner, Work& W, Counters& C, int* stop, hipStream_t s) {
  // Steihaug-Toint truncated CG, pipelined one step ahead.  Iterate j lives in
  // buffer j % 2 (it[0] = the caller's W.eta / W.Heta).  The device scalars
  // sc[j % 2] = {rr_j = ||r_j||^2, <d_j, H d_j>}; the update j -> j + 1 forms
  // alpha and beta from them on the device.  The host enqueues the update of
  // step j and the HVP of step j + 1 before it reads step j's scalars (one
  // event wait per step), then takes the same decisions as the plain loop
  // from host copies of the same scalars:
  //   rr_j = ||r_j||^2 <= tol^2  -> stop at eta_j (converged),
  //   <d, Hd> <= 0 or ||eta_j + alpha d_j|| >= Delta -> stop on the boundary,
  // tracking <eta, eta>, <eta, d>, <d, d> by their recurrences.  When it stops
  // at step j the work already enqueued for step j + 1 went into the other
  // buffer and is discarded; that HVP is not counted.
  const int n = P->n;
  const long long len = (long long)n * p;
  const double kappa = 0.1, theta = 1.0;
  *stop = TCG_MAXIT;
  TcgIter it[2] = {{W.eta, W.Heta, W.r, W.d, W.Hd}, W.it2};
  double* sc[2] = {W.rrb, W.rrb + 4};
  const double* hs[2] = {P->hbuf + 40, P->hbuf + 44};
  CHK(vec_fill(len, 0.0, it[0].eta, s));
  CHK(vec_fill(len, 0.0, it[0].Heta, s));
  CHK(vec_lincomb(len, 1.0, g, 0.0, nullptr, it[0].r, s));
  CHK(vec_lincomb(len, -1.0, g, 0.0, nullptr, it[0].d, s));
  double rr = gn * gn;
  CHK(vec_fill(1, rr, sc[0], s));
  if (maxinner <= 0) return MDSDP_OK;
  const double tol = gn * std::min(pow(gn, theta), kappa);
  double e_Pe = 0.0, e_Pd = 0.0, d_Pd = rr, e_part = 0.0, d_Pd_old = 0.0;
  auto t0 = clk::now();
  CHK(hvp_impl(P, p, prec, Y, it[0].d, it[0].Hd, 1, s, W.dpart, sc[0] + 1));
  C.hvps++;
  MDSDP_HIP(hipMemcpyAsync((void*)hs[0], sc[0], 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  MDSDP_HIP(hipEventRecord(W.ev[0], s));
  int cur = 0;
  // moves the result of iterate `k` into it[0]
  auto finish = [&](int k) -> mdsdp_status {
    if (k != 0) {
      CHK(vec_lincomb(len, 1.0, it[k].eta, 0.0, nullptr, it[0].eta, s));
      CHK(vec_lincomb(len, 1.0, it[k].Heta, 0.0, nullptr, it[0].Heta, s));
    }
    return MDSDP_OK;
  };
  for (int j = 0; j < maxinner; ++j) {
    const int nxt = cur ^ 1;
    // speculative: the update of step j, and the HVP of step j + 1
    CHK(launch_tcg_update(n, p, Y, sc[cur], sc[nxt], it[cur], it[nxt], W.part, s));
    if (j + 1 < maxinner) {
      CHK(hvp_impl(P, p, prec, Y, it[nxt].d, it[nxt].Hd, 1, s, W.dpart, sc[nxt] + 1));
      C.hvps++;
      MDSDP_HIP(hipMemcpyAsync((void*)hs[nxt], sc[nxt], 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      MDSDP_HIP(hipEventRecord(W.ev[nxt], s));
    }
    MDSDP_HIP(hipEventSynchronize(W.ev[cur]));
    const double rr_j = hs[cur][0], dHd = hs[cur][1];
    if (j > 0) {
      if (sqrt(rr_j) <= tol) {
        C.t_hvp += secs(t0, clk::now());
        if (j + 1 < maxinner) C.hvps--;  // the discarded speculative HVP
        *stop = TCG_CONV;
        return finish(cur);
      }
      const double beta = rr_j / rr;  // the device's beta: the same operands
      e_Pd = beta * e_part;
      d_Pd = rr_j + beta * beta * d_Pd_old;
      rr = rr_j;
    }
    const double alpha = (dHd != 0.0) ? rr / dHd : INFINITY;
    const double e_Pe_new = e_Pe + 2.0 * alpha * e_Pd + alpha * alpha * d_Pd;
    if (dHd <= 0.0 || e_Pe_new >= Delta * Delta) {
      const double tau = (-e_Pd + sqrt(std::max(0.0, e_Pd * e_Pd + d_Pd * (Delta * Delta - e_Pe)))) / d_Pd;
      CHK(vec_lincomb(len, tau, it[cur].d, 1.0, it[cur].eta, it[0].eta, s));
      CHK(vec_lincomb(len, tau, it[cur].Hd, 1.0, it[cur].Heta, it[0].Heta, s));
      C.t_hvp += secs(t0, clk::now());
      if (j + 1 < maxinner) C.hvps--;  // the discarded speculative HVP
      *stop = dHd <= 0.0 ? TCG_NEG : TCG_BOUND;
      return MDSDP_OK;
    }
    e_Pe = e_Pe_new;
    e_part = e_Pd + alpha * d_Pd;
    d_Pd_old = d_Pd;
    cur = nxt;
  }
  C.t_hvp += secs(t0, clk::now());
  return finish(cur);
}

// ---- Riemannian trust region -------------------------------------------------------
struct RTRState {
  double f = 0, gn = 0;
  int iters = 0;
  double Delta0 = 0.0;  // in: initial radius (0: Delta_bar / 8); out: the final radius
  bool stalled = false; // out: the call ended on the stall stop
};

mdsdp_status rtr(mdsdp_problem P, int p, double*& Y, double gtol, int maxiter, int maxinner, int prec,
                 Work& W, Counters& C, RTRState& st, hipStream_t s, int verbose = 0,
                 clk::time_point deadline = clk::time_point::max(), int max_stall = 0) {
  const int n = P->n;
  const long long len = (long long)n * p;
  const double Delta_bar = M_PI * sqrt((double)n);
  double Delta = st.Delta0 > 0.0 ? std::min(st.Delta0, Delta_bar) : Delta_bar / 8.0;
  double f;
  CHK(eval(P, p, Y, W.g, &f, C, s));
  double gg;
  {
    const double* a[1] = {W.g};
    CHK(dots(P, 1, a, a, len, &gg, s));
  }
  double gn = sqrt(gg);
  if (!std::isfinite(f) || !std::isfinite(gn)) {
    set_error("non-finite cost or gradient at the start of a subproblem (NaN or Inf in Y or the multiplier)");
    return MDSDP_ENONFINITE;
  }
  int it = 0;
  // stall stop (max_stall > 0): the call ends after max_stall consecutive
  // iterations that leave the gradient norm above 0.9 times the best so far
  // (the gradient has reached the level of its rounding errors)
  double gn_best = gn;
  int stall = 0;
  st.stalled = false;
  for (; it < maxiter; ++it) {
    if (gn <= gtol) break;
    if (max_stall > 0 && stall >= max_stall) {
      st.stalled = true;
      break;
    }
    int stop = 0;
    const long long hv0 = C.hvps;
    const double Delta_used = Delta;
    CHK(tcg(P, p, Y, W.g, gn, Delta, prec, maxinner, W, C, &stop, s));
    CHK(launch_retract(n, p, Y, W.eta, 1.0, W.Ynew, s));
    double fnew;
    CHK(eval(P, p, W.Ynew, W.gnew, &fnew, C, s));
    double d3[3];
    {
      const double* a[3] = {W.g, W.eta, W.gnew};
      const double* b[3] = {W.eta, W.Heta, W.gnew};
      CHK(dots(P, 3, a, b, len, d3, s));
    }
    const double model_dec = -(d3[0] + 0.5 * d3[1]);
    const double reg = std::max(1.0, fabs(f)) * 2.220446049250313e-16 * 1e3;
    const double rho = (f - fnew + reg) / (model_dec + reg);
    if (rho < 0.25)
      Delta /= 4.0;
    else if (rho > 0.75 && (stop == TCG_NEG || stop == TCG_BOUND))
      Delta = std::min(2.0 * Delta, Delta_bar);
    if (verbose >= 2)
      fprintf(stderr, "  [rtr] it=%d f=%.12e gn=%.3e Delta=%.3e rho=%.3e stop=%d inner=%lld %s\n", it, f, gn,
              Delta_used, rho, stop, C.hvps - hv0, (rho > 0.1 && std::isfinite(fnew)) ? "acc" : "REJ");
    if (rho > 0.1 && std::isfinite(fnew)) {
      std::swap(Y, W.Ynew);
      std::swap(W.g, W.gnew);
      f = fnew;
      gn = sqrt(d3[2]);
    } else {
      // restore the cached class sums / z of the current point
      double fcur;
      CHK(eval(P, p, Y, W.g, &fcur, C, s));
    }
    C.rtr_iters++;
    if (gn < 0.9 * gn_best) {
      gn_best = gn;
      stall = 0;
    } else {
      ++stall;
    }
    if (clk::now() > deadline) {
      ++it;
      break;
    }
  }
  st.f = f;
  st.gn = gn;
  st.iters = it;
  st.Delta0 = Delta;
  return MDSDP_OK;
}

}  // namespace

// ---- Lanczos ----------------------------------------------------------------------
// Lanczos with full reorthogonalisation on the certificate X = Xt + D - Diag z.
// Returns the extreme Ritz values; `evec` (nullable) receives up to `nvec`
// Ritz vectors (each n doubles, consecutive) of the smallest Ritz values; the
// first is always written, the others only for Ritz values below
// -neg_rel (1 + |theta_max|).  *nfound counts the vectors written.
static mdsdp_status lanczos(mdsdp_problem P, double tol, int maxit, uint64_t seed, double* lmin, double* lmax,
                            double* evec, int* iters, bool* converged, hipStream_t s, int nvec = 1,
                            double neg_rel = 0.0, int* nfound = nullptr, const double* warm = nullptr,
                            double* resid_out = nullptr, bool use_gap = false, int kconv = 1,
                            double* evals_out = nullptr, double* ext = nullptr, const double* Qd = nullptr,
                            int rq = 0, double* qc = nullptr, bool stop_nonneg = false,
                            double stop_above = 0.0, double reject_below = 0.0) {
  const int n = P->n;
  maxit = std::max(2, std::min(maxit, n));
  // basis V (n x (maxit + 1)), w (n), h (4 maxit + 16): the caller's fixed
  // scratch `ext` if given, else buffers of the problem (grown on demand)
  if (!ext && P->lz_cap < maxit + 1) {
    if (P->lz_V) (void)hipFree(P->lz_V);
    P->lz_V = nullptr;
    MDSDP_HIP(hipMalloc((void**)&P->lz_V, (size_t)n * (maxit + 1) * sizeof(double)));
    P->lz_cap = maxit + 1;
    if (!P->lz_w) MDSDP_HIP(hipMalloc((void**)&P->lz_w, (size_t)n * sizeof(double)));
    if (P->lz_h) (void)hipFree(P->lz_h);
    MDSDP_HIP(hipMalloc((void**)&P->lz_h, (size_t)(4 * maxit + 16) * sizeof(double)));
  }
  double* V = ext ? ext : P->lz_V;
  double* w = ext ? ext + (size_t)n * (maxit + 1) : P->lz_w;
  double* h = ext ? w + n : P->lz_h;
  std::vector<double> v0(n);
  gaussian_fill(seed ^ 0x5DEECE66Dull, v0);
  double nrm = 0.0;
  for (double x : v0) nrm += x * x;
  nrm = sqrt(nrm);
  for (double& x : v0) x /= nrm;
  if (warm) {
    // previous Ritz vector plus a 0.1-weighted random unit vector
    std::vector<double> wv(n);
    MDSDP_HIP(hipMemcpyAsync(wv.data(), warm, n * sizeof(double), hipMemcpyDeviceToHost, s));
    MDSDP_HIP(hipStreamSynchronize(s));
    double wn = 0.0;
    for (double x : wv) wn += x * x;
    wn = sqrt(wn);
    if (wn > 0.0 && std::isfinite(wn)) {
      double t = 0.0;
      for (int i = 0; i < n; ++i) {
        v0[i] = wv[i] / wn + 0.1 * v0[i];
        t += v0[i] * v0[i];
      }
      t = sqrt(t);
      for (double& x : v0) x /= t;
    }
  }
  // host-to-device copies go through the problem's pinned buffer (n doubles
  // fit: n < 65536 <= HBUF_LEN - 64), so no pageable staging is involved
  memcpy(P->hbuf + 64, v0.data(), n * sizeof(double));
  MDSDP_HIP(hipMemcpyAsync(V, P->hbuf + 64, n * sizeof(double), hipMemcpyHostToDevice, s));
  if (Qd && rq > 0) {
    // deflation (Qd = Q^T, rq x n): the Krylov space is kept orthogonal to range(Q), so the run
    // sees the compression of X to the complement of range(Q); the start is
    // projected and renormalised
    CHK(launch_deflate(n, rq, Qd, V, qc, s));
    CHK(launch_vt_w(n, 1, V, V, h, s));
    double nn;
    MDSDP_HIP(hipMemcpyAsync(P->hbuf, h, sizeof(double), hipMemcpyDeviceToHost, s));
    MDSDP_HIP(hipStreamSynchronize(s));
    nn = P->hbuf[0];
    if (!(nn > 0.0)) {
      set_error("deflated Lanczos start vector vanished");
      return MDSDP_EINVAL;
    }
    CHK(vec_lincomb(n, 1.0 / sqrt(nn), V, 0.0, nullptr, V, s));
  }
  MDSDP_HIP(hipStreamSynchronize(s));
  std::vector<double> al, be;
  std::vector<double> sv;
  double th_min = 0, th_max = 0;
  int k = 0;
  *converged = false;
  // The recurrence runs on the device: step j stores alpha_j and beta_j^2 in
  // alpha_d[j], beta2_d[j] and normalises the next basis vector by the
  // device value, so the host reads the scalars only every LZ_BATCH steps;
  // it then replays the convergence tests on those scalars, step by step for
  // the first 24 steps and at the last step of each batch after that (the
  // steps enqueued beyond a stop are discarded).
  constexpr int LZ_BATCH = 8;
  double* alpha_d = h + 2 * maxit + 8;
  double* beta2_d = alpha_d + maxit;
  bool stop = false;
  for (int j0 = 0; j0 < maxit && !stop; j0 += LZ_BATCH) {
    const int j1 = std::min(maxit, j0 + LZ_BATCH);
    for (int j = j0; j < j1; ++j) {
      double* vj = V + (size_t)j * n;
      CHK(mdsdp_certificate_matvec(P, 1, vj, w, s));
      if (Qd && rq > 0) CHK(launch_deflate(n, rq, Qd, w, qc, s));
      // full reorthogonalisation, twice (classical Gram-Schmidt with refinement)
      CHK(launch_vt_w(n, j + 1, V, w, h, s));
      CHK(launch_gemv_sub(n, j + 1, V, h, w, s));
      CHK(launch_vt_w(n, j + 1, V, w, h + maxit + 2, s));
      CHK(launch_gemv_sub(n, j + 1, V, h + maxit + 2, w, s));
      CHK(launch_vt_w(n, 1, w, w, h + 2 * maxit + 6, s));
      CHK(launch_lanczos_step(n, j, h, h + maxit + 2, h + 2 * maxit + 6, alpha_d, beta2_d, w,
                              V + (size_t)(j + 1) * n, j + 1 < maxit, s));
    }
    const int cnt = j1 - j0;
    MDSDP_HIP(hipMemcpyAsync(P->hbuf, alpha_d + j0, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    MDSDP_HIP(hipMemcpyAsync(P->hbuf + LZ_BATCH, beta2_d + j0, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    MDSDP_HIP(hipStreamSynchronize(s));
    for (int j = j0; j < j1; ++j) {
      al.push_back(P->hbuf[j - j0]);
      const double bj = sqrt(std::max(0.0, P->hbuf[LZ_BATCH + j - j0]));
      k = j + 1;
      // the tests cost O(k) host work per Ritz value (bisection, inverse
      // iteration): every step while k is small, then at the end of each batch
      // (and at a vanishing beta_j, where the run must stop)
      if (k >= 24 && j != j1 - 1 && !(bj <= 1e-14 * (1.0 + fabs(th_max)))) {
        be.push_back(bj);
        continue;
      }
      th_min = tridiag_eig(k, al.data(), be.data(), 0);
      th_max = tridiag_eig(k, al.data(), be.data(), k - 1);
      tridiag_evec(k, al.data(), be.data(), th_min, sv);
      // error estimate of theta_min: the residual, or residual^2 / gap when the
      // gap to the rest of the spectrum is certified: theta_2 minus its own
      // residual still lies above theta_min (then the interval of theta_2
      // excludes theta_min's eigenvalue and resid^2 / gap bounds its error)
      const double resid = bj * fabs(sv[k - 1]);
      double err = resid;
      if (use_gap && k >= 2) {
        const double th2 = tridiag_eig(k, al.data(), be.data(), 1);
        std::vector<double> s2;
        tridiag_evec(k, al.data(), be.data(), th2, s2);
        const double gap = th2 - bj * fabs(s2[k - 1]) - th_min;
        if (gap > 0.0) err = std::min(resid, resid * resid / gap);
      }
      // the other pairs that must converge (kconv > 1): their residuals
      double err_all = err;
      for (int i = 1; i < std::min(kconv, k); ++i) {
        std::vector<double> si;
        tridiag_evec(k, al.data(), be.data(), tridiag_eig(k, al.data(), be.data(), i), si);
        err_all = std::max(err_all, bj * fabs(si[k - 1]));
      }
      if (resid_out) *resid_out = err;
      if (k >= std::max(3, kconv + 2) && err_all <= tol * (1.0 + fabs(th_max))) {
        *converged = true;
        stop = true;
        break;
      }
      // certified: theta_min - err >= stop_above puts the smallest eigenvalue
      // (of the operator the run sees) at or above stop_above, which is all
      // the dual residual and the curvature test need
      if (stop_nonneg && k >= 3 && th_min - err >= stop_above * (1.0 + fabs(th_max))) {
        *converged = true;
        stop = true;
        break;
      }
      // rejection (reject_below < 0): lambda_min <= theta_min < reject_below
      // (1 + |theta_max|) already decides the test the caller makes
      if (reject_below < 0.0 && k >= 3 && th_min < reject_below * (1.0 + fabs(th_max))) {
        stop = true;
        break;
      }
      if (bj <= 1e-14 * (1.0 + fabs(th_max))) {
        *converged = true;  // invariant subspace
        stop = true;
        break;
      }
      be.push_back(bj);
    }
  }
  *lmin = th_min;
  *lmax = th_max;
  *iters = k;
  if (evals_out)
    for (int i = 0; i < kconv; ++i) evals_out[i] = i < k ? tridiag_eig(k, al.data(), be.data(), i) : NAN;
  int found = 0;
  if (evec && nvec >= 1) {
    // Ritz vectors V s_i for the smallest Ritz values (the first always; with
    // neg_rel >= 0 the others only while negative)
    for (int i = 0; i < std::min(nvec, k); ++i) {
      const double th = i == 0 ? th_min : tridiag_eig(k, al.data(), be.data(), i);
      if (i > 0 && neg_rel >= 0.0 && !(th < -neg_rel * (1.0 + fabs(th_max)))) break;
      if (i > 0) tridiag_evec(k, al.data(), be.data(), th, sv);
      memcpy(P->hbuf + 64, sv.data(), k * sizeof(double));
      MDSDP_HIP(hipMemcpyAsync(h, P->hbuf + 64, k * sizeof(double), hipMemcpyHostToDevice, s));
      CHK(launch_gemv(n, k, V, h, evec + (size_t)i * n, s));
      MDSDP_HIP(hipStreamSynchronize(s));
      ++found;
    }
  }
  if (nfound) *nfound = found;
  return MDSDP_OK;
}

// Bounds on the spectrum of the certificate X = Xt + D - Diag(z) (z of the
// last multiplier update) for eta_d of eq. res and the curvature test of
// Theorem sec5:thm1.  With Q an orthonormal basis of range(Y) and
// A = Q^T X Q, B = (I - Q Q^T) X Q, C = the compression of X to the complement
// of range(Q): X = [[A, B^T], [B, C]] in [Q, Q_perp], and lambda_min(X) is at
// least the smaller eigenvalue of [[lambda_min(A), -||B||_2], [-||B||_2,
// lambda_min(C)]] (a sharpening of Weyl's min(lambda_min(A), lambda_min(C)) -
// ||B||_2; ||B||_2 from the rq x rq matrix B^T B for rq <= 64, else the
// Frobenius norm, which bounds it).  X Y = grad / 2
// is small at a solved subproblem, so A and B are small and the Lanczos run on
// C does not have to resolve the cluster of eigenvalues near zero that
// range(Y) carries.  An unconverged Lanczos run only certifies an eigenvalue
// within its error estimate of theta_min, so lo uses theta_min minus that
// estimate then.  wv / Vv: eigen-decomposition of Y^T Y, idx its order by
// decreasing eigenvalue.  Qb, XQb: n x p buffers; qc: p doubles.
// Neither a residual nor a gap estimate can show that the Krylov space has
// reached the bottom of the spectrum: a run warm-started near an eigenvector
// that is not the lowest can meet its stopping test within a few steps.  The
// fast mode (warm start, gap-based error, stop once theta_min minus the error
// is at least stop_above) steers the iteration; every eta_d that ends a solve
// comes from a verify run (random start, residual error, no early stop).
struct CertSpectrum {
  double lo = 0.0;    // certified lower bound of lambda_min(X)
  double lmin = 0.0;  // smallest Ritz value of the run
  double lmax = 0.0;  // largest Ritz value (of the run and of A)
  int iters = 0, nfound = 0;
  bool conv = false;
};

static mdsdp_status certificate_spectrum(mdsdp_problem P, int p, const double* Y, const std::vector<double>& wv,
                                         const std::vector<double>& Vv, const std::vector<int>& idx, bool deflate,
                                         double eig_tol, int budget, uint64_t seed, int nvec, const double* warm,
                                         double* evec, double* Qb, double* XQb, double* qc, double stop_above,
                                         CertSpectrum* out, hipStream_t s, bool verify = false,
                                         double reject_below = 0.0) {
  const int n = P->n;
  double lmin = 0, lmax = 0, lres = 0.0;
  double lmin_A = 0.0, lmax_A = 0.0, nB = 0.0;
  int eit = 0, nfound = 0;
  bool conv = false;
  int rq = 0;
  {
    const double w0 = std::max(0.0, wv[idx[0]]);
    for (int i = 0; i < p; ++i)
      if (wv[idx[i]] > 1e-14 * w0) ++rq;
    rq = std::min(rq, n - 2);
  }
  if (deflate && rq > 0) {
    // Q = Y V_r diag(w_r)^{-1/2}  (n x rq, in Qb); X Q in XQb, then Q^T there
    std::vector<double> Mq((size_t)p * rq);
    for (int i = 0; i < p; ++i)
      for (int c = 0; c < rq; ++c) Mq[(size_t)i * rq + c] = Vv[i * p + idx[c]] / sqrt(wv[idx[c]]);
    memcpy(P->hbuf + 64, Mq.data(), Mq.size() * sizeof(double));
    MDSDP_HIP(hipMemcpyAsync(P->gpart + GP_M, P->hbuf + 64, Mq.size() * sizeof(double), hipMemcpyHostToDevice, s));
    CHK(launch_rightmul(n, p, rq, Y, P->gpart + GP_M, false, Qb, s));
    CHK(mdsdp_certificate_matvec(P, rq, Qb, XQb, s));
    CHK(launch_gram(P, rq, Qb, XQb, s));
    const int pw = P->gram_pw;
    std::vector<double> G((size_t)pw * pw), Aq((size_t)rq * rq), wa(rq), Va((size_t)rq * rq);
    CHK(read_dev(P, P->gram + GRAM_U, pw * pw, G.data(), s));
    double a2 = 0.0;
    for (int i = 0; i < rq; ++i)
      for (int j = 0; j < rq; ++j) {
        Aq[i * rq + j] = 0.5 * (G[(size_t)i * pw + j] + G[(size_t)j * pw + i]);
        a2 += Aq[i * rq + j] * Aq[i * rq + j];
      }
    if (rq <= 64) {
      // ||B||_2^2 = lambda_max(B^T B), B^T B = (X Q)^T (X Q) - A^2 (rq x rq)
      CHK(launch_gram(P, rq, XQb, XQb, s, false));
      std::vector<double> G2((size_t)pw * pw), M((size_t)rq * rq), wm(rq), Vm((size_t)rq * rq);
      CHK(read_dev(P, P->gram + GRAM_U, pw * pw, G2.data(), s));
      for (int i = 0; i < rq; ++i)
        for (int j = 0; j < rq; ++j) {
          double aa = 0.0;
          for (int l = 0; l < rq; ++l) aa += Aq[i * rq + l] * Aq[l * rq + j];
          M[i * rq + j] = 0.5 * (G2[(size_t)i * pw + j] + G2[(size_t)j * pw + i]) - aa;
        }
      sym_eig(rq, M.data(), wm.data(), Vm.data());
      nB = sqrt(std::max(0.0, *std::max_element(wm.begin(), wm.end())));
    } else {
      double xq2;
      const double* a1[1] = {XQb};
      CHK(dots(P, 1, a1, a1, (long long)n * rq, &xq2, s));
      nB = sqrt(std::max(0.0, xq2 - a2));  // ||X Q - Q A||_F >= ||B||_2
    }
    sym_eig(rq, Aq.data(), wa.data(), Va.data());
    lmin_A = *std::min_element(wa.begin(), wa.end());
    lmax_A = *std::max_element(wa.begin(), wa.end());
    CHK(launch_transpose(n, rq, Qb, XQb, s));  // Q^T (rq x n) for the projections
  } else {
    rq = 0;
  }
  // verify: a fresh random start, the residual alone as the error estimate
  // and no early stop, i.e. the run stops only once theta_min has converged
  // (or at the budget)
  CHK(lanczos(P, eig_tol, budget, seed, &lmin, &lmax, evec, &eit, &conv, s, nvec, 1e-12, &nfound,
              verify ? nullptr : warm, &lres, !verify, 1, nullptr, nullptr, rq > 0 ? XQb : nullptr, rq, qc, !verify,
              stop_above, reject_below));
  double lo = conv ? lmin : lmin - lres;
  if (rq > 0) {
    // for a unit x = (u, w) in [Q, Q_perp]: x^T X x >= a |u|^2 - 2 b |u| |w| + c |w|^2
    // with a = lambda_min(A), c = lambda_min(C), b = ||B||_2, whose minimum over
    // |u|^2 + |w|^2 = 1 is the smaller eigenvalue of [[a, -b], [-b, c]]
    // (at least min(a, c) - b, and a - b^2 / (c - a) when c - a >> b)
    const double a_ = lmin_A, c_ = lo;
    lo = 0.5 * (a_ + c_) - sqrt(0.25 * (a_ - c_) * (a_ - c_) + nB * nB);
    lmax = std::max(lmax, lmax_A);
  }
  out->lo = lo;
  out->lmin = lmin;
  out->lmax = lmax;
  out->iters = eit;
  out->nfound = nfound;
  out->conv = conv;
  return MDSDP_OK;
}

}  // namespace mdsdp

using namespace mdsdp;

extern "C" {

void mdsdp_default_options(mdsdp_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_outer = 200;
  o->sigma0 = 1.0;
  o->sigma_min = 1e-3;
  o->sigma_max = 1e6;
  o->gamma = 2.0;
  o->kappa1 = 0.1;
  o->kappa2 = 10.0;
  o->p_max = PMAX;
  o->n_neg = 15;
  o->tau_rank = 1e-7;
  o->gtol0 = 1e-2;
  o->gtol_min = 1e-10;
  o->gtol_decay = 1.0;
  o->gtol_ratio = 0.1;
  o->gtol_stall = 0.0;
  o->sigma_hold = 1;
  o->escape_when_solved = 0;
  o->rtr_maxiter = 10;
  o->tcg_maxinner = 200;
  o->hvp_prec = MDSDP_FP64;
  o->polish_fp64 = 1;
  o->polish_eta = 1e-4;
  o->deflate = 1;
  o->direct_admm = 0;
  o->rtr_warm_radius = 1;
  o->rtr_maxiter_polish = 50;
  o->tcg_maxinner_polish = 1000;
  o->rtr_stall = 0;
  o->round_rank_one = 1;
  o->round_eta = 1e-3;
  o->round_gap = 0.1;
  o->eig_tol = 1e-10;
  o->eig_maxit = 300;
  o->time_limit_s = 0.0;
  o->verbose = 0;
  o->seed = 1;
}

mdsdp_status mdsdp_min_eigpair(mdsdp_problem P, int32_t k, double tol, int32_t maxit, uint64_t seed,
                               double* evals, double* lambda_max, double* evecs, int32_t* iters, void* stream) {
  if (!P || !evals || !lambda_max) {
    set_error("NULL argument");
    return MDSDP_EINVAL;
  }
  if (k < 1 || maxit < 2 || !(tol > 0.0)) {
    set_error("need k >= 1, maxit >= 2 and tol > 0");
    return MDSDP_EINVAL;
  }
  if (k > P->n || k + 2 > maxit) {
    set_error("need k <= n and k + 2 <= maxit");
    return MDSDP_EINVAL;
  }
  bool conv = false;
  int it = 0;
  double lmin = 0.0;
  mdsdp_status st = lanczos(P, tol, maxit, seed, &lmin, lambda_max, evecs, &it, &conv, (hipStream_t)stream, k,
                            -1.0, nullptr, nullptr, nullptr, false, k, evals);
  if (iters) *iters = it;
  if (st != MDSDP_OK) return st;
  if (!conv) {
    set_error("Lanczos reached maxit before the residual tolerance");
    return MDSDP_ENOCONV;
  }
  return MDSDP_OK;
}

mdsdp_status mdsdp_min_eigpair_noalloc(mdsdp_problem P, int32_t k, double tol, int32_t maxit, uint64_t seed,
                                       double* evals, double* lambda_max, double* evecs, int32_t* iters,
                                       void* stream) {
  if (!P || !evals || !lambda_max) {
    set_error("NULL argument");
    return MDSDP_EINVAL;
  }
  if (k < 1 || maxit < 2 || !(tol > 0.0) || k > P->n || k + 2 > maxit) {
    set_error("need 1 <= k <= n, maxit >= k + 2 and tol > 0");
    return MDSDP_EINVAL;
  }
  const int n = P->n;
  const int mx = std::min(maxit, n);
  const long long need = (long long)n * (mx + 1) + n + 4LL * mx + 16;
  if (need > SCRATCH_DOUBLES) {
    set_error("n * (maxit + 1) + n + 4 maxit + 16 = " + std::to_string(need) + " doubles exceeds the fixed scratch of " +
              std::to_string(SCRATCH_DOUBLES) + " doubles; lower maxit or use mdsdp_min_eigpair");
    return MDSDP_EINVAL;
  }
  int dev = -1;
  MDSDP_HIP(hipGetDevice(&dev));
  if (dev != P->device) {
    set_error("the current device is not the problem's device");
    return MDSDP_EINVAL;
  }
  double* ext = nullptr;
  CHK(scratch_buffer(&ext));
  bool conv = false;
  int it = 0;
  double lmin = 0.0;
  mdsdp_status st = lanczos(P, tol, maxit, seed, &lmin, lambda_max, evecs, &it, &conv, (hipStream_t)stream, k,
                            -1.0, nullptr, nullptr, nullptr, false, k, evals, ext);
  if (iters) *iters = it;
  if (st != MDSDP_OK) return st;
  if (!conv) {
    set_error("Lanczos reached maxit before the residual tolerance");
    return MDSDP_ENOCONV;
  }
  return MDSDP_OK;
}

mdsdp_status mdsdp_certificate_estimate(mdsdp_problem P, double tol, int32_t maxit, uint64_t seed,
                                       const double* warm, double* out, double* evec, int32_t* iters,
                                       void* stream) {
  if (!P || !out) {
    set_error("NULL argument");
    return MDSDP_EINVAL;
  }
  if (maxit < 3 || !(tol > 0.0)) {
    set_error("need maxit >= 3 and tol > 0");
    return MDSDP_EINVAL;
  }
  bool conv = false;
  int it = 0;
  double err = 0.0;
  mdsdp_status st = lanczos(P, tol, maxit, seed, out, out + 1, evec, &it, &conv, (hipStream_t)stream, 1, 0.0,
                            nullptr, warm, &err, true);
  if (iters) *iters = it;
  out[2] = err;
  out[3] = conv ? 1.0 : 0.0;
  return st;
}

mdsdp_status mdsdp_certificate_bound(mdsdp_problem P, int32_t p, const double* Y, double tol, int32_t maxit,
                                    uint64_t seed, double* out, void* stream) {
  if (!P || !Y || !out) {
    set_error("NULL argument");
    return MDSDP_EINVAL;
  }
  if (p < 1 || p > PMAX || p > P->n - 2 || maxit < 3 || !(tol > 0.0)) {
    set_error("need 1 <= p <= min(512, n - 2), maxit >= 3 and tol > 0");
    return MDSDP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int n = P->n;
  CHK(launch_gram(P, p, Y, Y, s));
  P->gram_yy_valid = false;
  std::vector<double> wv(p), Vv((size_t)p * p);
  {
    const int pw = P->gram_pw;
    std::vector<double> G((size_t)pw * pw), A((size_t)p * p);
    CHK(read_dev(P, P->gram, pw * pw, G.data(), s));
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) A[i * p + j] = G[(size_t)i * pw + j];
    sym_eig(p, A.data(), wv.data(), Vv.data());
  }
  std::vector<int> idx(p);
  for (int i = 0; i < p; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return wv[x] > wv[y]; });
  double* buf = nullptr;
  const size_t len = 3 * (size_t)n * p + n + PMAX;
  MDSDP_HIP(hipMalloc((void**)&buf, len * sizeof(double)));
  CertSpectrum sp;
  const mdsdp_status st = certificate_spectrum(P, p, Y, wv, Vv, idx, true, tol, maxit, seed, 1, nullptr, buf,
                                               buf + n, buf + n + (size_t)n * p, buf + n + 2 * (size_t)n * p, 0.0,
                                               &sp, s, true);
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (st != MDSDP_OK) return st;
  out[0] = sp.lo;
  out[1] = sp.lmax;
  out[2] = sp.iters;
  out[3] = sp.conv ? 1.0 : 0.0;
  return MDSDP_OK;
}

mdsdp_status mdsdp_solve(mdsdp_problem P, const mdsdp_options* opt, int32_t p0, double* Ybuf, mdsdp_result* res,
                         double* hist, int32_t hist_cap, void* stream) {
  if (!opt) {
    set_error("NULL options");
    return MDSDP_EINVAL;
  }
  // options first, so that a bad option is reported whatever else is wrong
  if (!(opt->tol > 0.0) || opt->max_outer < 1) {
    set_error("need tol > 0 and max_outer >= 1");
    return MDSDP_EINVAL;
  }
  if (!(opt->sigma_min > 0.0 && opt->sigma_min <= opt->sigma_max && std::isfinite(opt->sigma_max))) {
    set_error("need 0 < sigma_min <= sigma_max < inf");
    return MDSDP_EINVAL;
  }
  if (!(opt->sigma0 >= opt->sigma_min && opt->sigma0 <= opt->sigma_max)) {
    set_error("need sigma_min <= sigma0 <= sigma_max");
    return MDSDP_EINVAL;
  }
  if (!(opt->gamma > 1.0 && opt->kappa1 > 0.0 && opt->kappa1 <= opt->kappa2 && std::isfinite(opt->kappa2))) {
    set_error("need gamma > 1 and 0 < kappa1 <= kappa2 (eq. sec5:eq1)");
    return MDSDP_EINVAL;
  }
  if (!(opt->time_limit_s >= 0.0) || opt->rtr_maxiter < 1 || opt->tcg_maxinner < 1 || opt->eig_maxit < 2 ||
      !(opt->eig_tol > 0.0) || !(opt->gtol0 > 0.0) || !(opt->gtol_min >= 0.0)) {
    set_error("need time_limit_s >= 0, rtr_maxiter >= 1, tcg_maxinner >= 1, eig_maxit >= 2, eig_tol > 0, "
              "gtol0 > 0, gtol_min >= 0");
    return MDSDP_EINVAL;
  }
  if (opt->hvp_prec != MDSDP_FP64 && opt->hvp_prec != MDSDP_FP32) {
    set_error("hvp_prec must be MDSDP_FP64 or MDSDP_FP32");
    return MDSDP_EINVAL;
  }
  if (!(opt->round_eta >= 0.0 && opt->round_gap >= 0.0 && opt->round_gap <= 1.0)) {
    set_error("need round_eta >= 0 and 0 <= round_gap <= 1");
    return MDSDP_EINVAL;
  }
  if (!P || !Ybuf || !res) {
    set_error("NULL argument");
    return MDSDP_EINVAL;
  }
  if (opt->p_max < 1 || opt->p_max > PMAX || p0 < 1 || p0 > opt->p_max) {
    set_error("need 1 <= p0 <= p_max <= " + std::to_string(PMAX));
    return MDSDP_EINVAL;
  }
  if (!(opt->gtol_decay > 0.0 && opt->gtol_decay <= 1.0)) {
    set_error("need 0 < gtol_decay <= 1");
    return MDSDP_EINVAL;
  }
  if (opt->n_neg < 0 || opt->n_neg > PMAX) {
    set_error("need 0 <= n_neg <= " + std::to_string(PMAX));
    return MDSDP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int n = P->n;
  const auto t_start = clk::now();
  memset(res, 0, sizeof(*res));
  Work W;
  CHK(W.init(n));
  Counters C;
  int p = p0;
  // the caller's buffer holds Y; we alternate between it and W.Ynew, so keep
  // a pointer and copy back at the end.
  double* Y = Ybuf;
  // normalise rows of the start point
  CHK(launch_retract(n, p, Y, Y, 0.0, Y, s));
  if (opt->resume) {
    CHK(mdsdp_set_sigma(P, opt->sigma0));
    CHK(vec_fill(1, 0.0, P->scal + SC_NONFIN, s));
  } else {
    CHK(mdsdp_set_multiplier(P, nullptr, opt->sigma0, s));
  }
  // direct-DSDP ablation: stale y^0 = class averages at the start point
  CHK(mdsdp_set_direct(P, opt->direct_admm ? 1 : 0, p, opt->direct_admm ? Y : nullptr, s));
  double sigma = opt->sigma0;
  double eta_max = 1.0;
  bool carry = false;
  int p_maxr = p;
  double eta[3] = {INFINITY, INFINITY, INFINITY};
  double value = 0.0;
  int k = 0;
  mdsdp_status final_status = MDSDP_ENOCONV;
  double* evec = W.tmp;
  double gtol = opt->gtol0 / opt->gtol_decay;
  double prim_ratio = INFINITY;  // ||R|| / (1 + ||b||) of the last outer step
  double stall_cap = INFINITY;   // tolerance cap after an RTR call that took no step
  bool have_evec = false;
  int eig_budget = opt->eig_maxit;
  const int verify_budget = std::min(n, std::max(4 * opt->eig_maxit, 64));
  double warm_delta = 0.0;
  int rounded = 0;
  for (k = 0; k < opt->max_outer; ++k) {
    CHK(mdsdp_set_sigma(P, sigma));
    // polishing phase (eta_max < polish_eta): FP64 HVPs and the larger RTR budget
    const bool polish = eta_max < opt->polish_eta;
    const int prec = (opt->polish_fp64 && polish) ? MDSDP_FP64 : opt->hvp_prec;
    const int rtr_budget = polish ? std::max(opt->rtr_maxiter, opt->rtr_maxiter_polish) : opt->rtr_maxiter;
    const int tcg_budget = polish ? std::max(opt->tcg_maxinner, opt->tcg_maxinner_polish) : opt->tcg_maxinner;
    if (carry) {
      // backtracking along the carried negative-curvature direction
      double f0;
      CHK(eval(P, p, Y, nullptr, &f0, C, s));
      double t = sqrt((double)n);
      while (t > 1e-8) {
        CHK(launch_retract(n, p, Y, W.U, t, W.Ynew, s));
        double ft;
        CHK(eval(P, p, W.Ynew, nullptr, &ft, C, s));
        if (ft < f0) {
          std::swap(Y, W.Ynew);
          break;
        }
        t *= 0.5;
      }
    }
    {
      double g;
      if (opt->gtol_ratio > 0.0)
        g = std::isfinite(prim_ratio) ? std::min(opt->gtol0, opt->gtol_ratio * prim_ratio) : opt->gtol0;
      else
        g = std::min(std::min(opt->gtol0, 0.1 * eta_max), opt->gtol_decay * gtol);
      g = std::min(g, stall_cap);
      gtol = std::max(opt->gtol_min, g);
    }
    RTRState rs;
    // warm radius: the previous call's final radius (at most Delta_bar / 8),
    // so that a call does not spend its first steps shrinking Delta_bar / 8
    if (opt->rtr_warm_radius && warm_delta > 0.0) rs.Delta0 = std::min(warm_delta, M_PI * sqrt((double)n) / 8.0);
    const clk::time_point deadline =
        opt->time_limit_s > 0 ? t_start + std::chrono::duration_cast<clk::duration>(
                                              std::chrono::duration<double>(opt->time_limit_s))
                              : clk::time_point::max();
    mdsdp_status rst = rtr(P, p, Y, gtol, rtr_budget, tcg_budget, prec, W, C, rs, s, opt->verbose,
                           deadline, opt->rtr_stall);
    if (rst == MDSDP_ENONFINITE) {
      final_status = MDSDP_ENONFINITE;
      ++k;
      break;
    }
    CHK(rst);
    warm_delta = rs.Delta0;
    if (opt->gtol_stall > 0.0 && rs.iters == 0 && rs.gn > 0.0) stall_cap = std::min(stall_cap, opt->gtol_stall * rs.gn);
    // multiplier update (Algorithm alg1 steps 5-8)
    auto tu = clk::now();
    CHK(mdsdp_update_multiplier(P, p, Y, nullptr, nullptr, P->scal + SC_KKT, s));
    double kk[4];
    CHK(read_dev(P, P->scal + SC_KKT, 4, kk, s));
    C.t_update += secs(tu, clk::now());
    if (!(std::isfinite(kk[0]) && std::isfinite(kk[1]) && std::isfinite(kk[2]) && std::isfinite(kk[3]))) {
      set_error("non-finite value in the multiplier update (||Q(Z)||, b^T y or sum z)");
      final_status = MDSDP_ENONFINITE;
      ++k;
      break;
    }
    // Gram matrix of Y and its eigen-decomposition (p x p, host): the rank
    // update below and the deflation of the certificate eigensolve
    CHK(launch_gram(P, p, Y, Y, s));
    P->gram_yy_valid = false;  // the Gram buffer is reused below and Y changes
    std::vector<double> wv(p), Vv((size_t)p * p);
    {
      const int pw = P->gram_pw;
      std::vector<double> G((size_t)pw * pw), A((size_t)p * p);
      CHK(read_dev(P, P->gram, pw * pw, G.data(), s));
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) A[i * p + j] = G[(size_t)i * pw + j];
      sym_eig(p, A.data(), wv.data(), Vv.data());
    }
    std::vector<int> idx(p);
    for (int i = 0; i < p; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return wv[x] > wv[y]; });
    auto te = clk::now();
    CertSpectrum sp;
    CHK(certificate_spectrum(P, p, Y, wv, Vv, idx, opt->deflate != 0, opt->eig_tol, eig_budget,
                             opt->seed + (uint64_t)k, std::max(1, opt->n_neg), have_evec ? evec : nullptr, evec, W.r,
                             W.Hd, W.qc, -0.5 * opt->tol, &sp, s));
    have_evec = true;
    C.eig_iters += sp.iters;
    C.t_eig += secs(te, clk::now());
    const double lmin = sp.lmin, lmax = sp.lmax, lo = sp.lo;
    const bool conv = sp.conv;
    const int nfound = sp.nfound, eit = sp.iters;
    const double normR = kk[0], bty = kk[1], sumz = kk[2], cx = kk[3];
    eta[0] = normR / (1.0 + P->normC);
    eta[1] = std::max(0.0, -lo) / (1.0 + fabs(lmax));
    const double prim = cx + sumz;
    eta[2] = fabs(prim - bty) / (1.0 + fabs(prim) + fabs(bty));
    eta_max = std::max(eta[0], std::max(eta[1], eta[2]));
    if (eta_max <= opt->tol) {
      // acceptance: eta_d again from a verify run
      const auto tv = clk::now();
      CertSpectrum spv;
      CHK(certificate_spectrum(P, p, Y, wv, Vv, idx, opt->deflate != 0, opt->eig_tol, verify_budget,
                               opt->seed + (uint64_t)k + 0x632BE59BD9B4E019ull, 1, nullptr, W.it2.d, W.r, W.Hd,
                               W.qc, 0.0, &spv, s, true, -2.0 * opt->tol));
      C.eig_iters += spv.iters;
      C.t_eig += secs(tv, clk::now());
      eta[1] = std::max(0.0, -spv.lo) / (1.0 + fabs(spv.lmax));
      eta_max = std::max(eta[0], std::max(eta[1], eta[2]));
      if (opt->verbose)
        fprintf(stderr, "[mdsdp] k=%d verified eta_d=%.2e (%d steps%s)\n", k, eta[1], spv.iters,
                spv.conv ? "" : ", unconverged");
      if (eta_max > opt->tol) eig_budget = std::min(n, 2 * eig_budget);
    }
    // when the dual residual (an unconverged Lanczos estimate) is among the
    // largest residuals, give the next eigensolve more steps (it restarts
    // from the current Ritz vector)
    if (!conv && eta[1] > opt->tol && eta[1] >= 0.5 * eta_max) eig_budget = std::min(n, 2 * eig_budget);
    value = bty;
    if (hist && k < hist_cap) {
      double* hrow = hist + (size_t)k * 8;
      hrow[0] = k;
      hrow[1] = p;
      hrow[2] = sigma;
      hrow[3] = eta[0];
      hrow[4] = eta[1];
      hrow[5] = eta[2];
      hrow[6] = value;
      hrow[7] = (double)C.hvps;
    }
    if (opt->verbose)
      fprintf(stderr,
              "[mdsdp] k=%d p=%d sigma=%.3g eta=(%.2e %.2e %.2e) value=%.10f gnorm=%.2e rtr=%d hvps=%lld eig=%d "
              "s2/s1=%.2e\n",
              k, p, sigma, eta[0], eta[1], eta[2], value, rs.gn, rs.iters, C.hvps, eit,
              p > 1 ? sqrt(std::max(0.0, wv[idx[1]]) / std::max(1e-300, wv[idx[0]])) : 0.0);
    if (eta_max <= opt->tol) {
      final_status = MDSDP_OK;
      ++k;
      break;
    }
    // rank-one compression test (Theorem thm:finite-locking, Remark
    // rem:inexact-near-locking): once Y is close to rank one, eq. res is
    // evaluated at S1 = Y1 Y1^T, Y1 = sign(Y v_1) (v_1 the leading right
    // singular vector), with the current multiplier and no multiplier step
    // (sigma 0 in the update pass: Xt stays, z becomes z(S1)).  The solve
    // stops there when that point meets the tolerance; otherwise nothing of
    // the iteration changes (the next multiplier update recomputes z).
    if (opt->round_rank_one && !opt->direct_admm && eta_max < opt->round_eta &&
        (p == 1 || wv[idx[1]] <= opt->round_gap * opt->round_gap * wv[idx[0]])) {
      const auto tr = clk::now();
      for (int i = 0; i < p; ++i) P->hbuf[64 + i] = Vv[i * p + idx[0]];
      MDSDP_HIP(hipMemcpyAsync(P->gpart + GP_M, P->hbuf + 64, p * sizeof(double), hipMemcpyHostToDevice, s));
      double* Y1 = W.it2.eta;
      CHK(launch_sign_col(n, p, Y, P->gpart + GP_M, Y1, s));
      const double sigma_keep = P->sigma;
      P->sigma = 0.0;
      const mdsdp_status ust = mdsdp_update_multiplier(P, 1, Y1, nullptr, nullptr, P->scal + SC_KKT, s);
      P->sigma = sigma_keep;
      CHK(ust);
      double k1[4];
      CHK(read_dev(P, P->scal + SC_KKT, 4, k1, s));
      double eta1[3] = {k1[0] / (1.0 + P->normC), INFINITY,
                        fabs(k1[3] + k1[2] - k1[1]) / (1.0 + fabs(k1[3] + k1[2]) + fabs(k1[1]))};
      // the eigensolve only for a point that is feasible and has no gap
      if (eta1[0] <= opt->tol && eta1[2] <= opt->tol) {
        const std::vector<double> w1(1, (double)n), V1(1, 1.0);
        const std::vector<int> i1(1, 0);
        CertSpectrum sp1;
        CHK(certificate_spectrum(P, 1, Y1, w1, V1, i1, opt->deflate != 0, opt->eig_tol,
                                 std::max(eig_budget, verify_budget), opt->seed + (uint64_t)k + 0x9E3779B97F4A7C15ull,
                                 1, nullptr, W.it2.d, W.it2.Heta, W.it2.r, W.qc, 0.0, &sp1, s, true,
                                 -2.0 * opt->tol));
        C.eig_iters += sp1.iters;
        eta1[1] = std::max(0.0, -sp1.lo) / (1.0 + fabs(sp1.lmax));
      }
      C.t_eig += secs(tr, clk::now());
      if (opt->verbose)
        fprintf(stderr, "[mdsdp] k=%d rank-one compression eta=(%.2e %.2e %.2e)\n", k, eta1[0], eta1[1], eta1[2]);
      if (std::max(eta1[0], std::max(eta1[1], eta1[2])) <= opt->tol) {
        MDSDP_HIP(hipMemcpyAsync(Y, Y1, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        p = 1;
        for (int i = 0; i < 3; ++i) eta[i] = eta1[i];
        value = k1[1];
        rounded = 1;
        final_status = MDSDP_OK;
        ++k;
        break;
      }
    }
    if (opt->time_limit_s > 0 && secs(t_start, clk::now()) > opt->time_limit_s) {
      ++k;
      break;
    }
    // rank update: singular values of Y from its Gram matrix (computed above)
    const double s1 = sqrt(std::max(0.0, wv[idx[0]]));
    int r = 0;
    for (int i = 0; i < p; ++i)
      if (sqrt(std::max(0.0, wv[idx[i]])) > opt->tau_rank * s1) ++r;
    r = std::max(1, r);
    const bool unsolved = rs.gn > gtol;  // RTR stopped at its iteration cap
    // curvature below the stopping tolerance's scale is not worth new columns
    const bool neg = lmin < -std::max(1e-12, opt->tol) * (1.0 + fabs(lmax));
    // negative-curvature directions: Ritz vectors of the negative Ritz values
    int nneg = 0;
    if (neg && opt->n_neg > 0 && !(opt->escape_when_solved && unsolved)) nneg = std::min(nfound, opt->n_neg);
    const int dadd = std::max(0, std::min(nneg, opt->p_max - r));
    const int pnew = r + dadd;
    // M = [V_r, 0] (p x pnew)
    std::vector<double> M((size_t)p * pnew);
    for (int i = 0; i < p; ++i)
      for (int c = 0; c < pnew; ++c) M[(size_t)i * pnew + c] = (c < r) ? Vv[i * p + idx[c]] : 0.0;
    MDSDP_HIP(hipMemcpyAsync(P->gpart + GP_M, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice, s));
    CHK(launch_rightmul(n, p, pnew, Y, P->gpart + GP_M, true, W.Ynew, s));
    MDSDP_HIP(hipStreamSynchronize(s));
    std::swap(Y, W.Ynew);
    p = pnew;
    p_maxr = std::max(p_maxr, p);
    carry = false;
    if (dadd) {
      // U = [0, v_1, ..., v_dadd]: launch_set_col zeroes the other columns on the first call only
      for (int j = 0; j < dadd; ++j) CHK(launch_set_col(n, p, r + j, evec + (size_t)j * n, W.U, s, j == 0));
      carry = true;
    }
    // sigma rule, eq. sec5:eq1
    const double ratio = normR / (1.0 + P->normb);
    prim_ratio = ratio;
    if (ratio < opt->kappa1 * rs.gn && !(opt->sigma_hold && unsolved))
      sigma = std::max(sigma / opt->gamma, opt->sigma_min);
    else if (ratio > opt->kappa2 * rs.gn)
      sigma = std::min(opt->gamma * sigma, opt->sigma_max);
  }
  MDSDP_HIP(hipStreamSynchronize(s));
  if (opt->direct_admm) CHK(mdsdp_set_direct(P, 0, p, nullptr, s));
  if (Y != Ybuf) MDSDP_HIP(hipMemcpy(Ybuf, Y, (size_t)n * p * sizeof(double), hipMemcpyDeviceToDevice));
  res->status = final_status;
  res->outer_iters = k;
  res->rtr_iters = C.rtr_iters;
  res->hvps = C.hvps;
  res->cost_grads = C.cost_grads;
  res->eig_iters = C.eig_iters;
  res->p_final = p;
  res->p_max_reached = p_maxr;
  res->value = value;
  res->eta_p = eta[0];
  res->eta_d = eta[1];
  res->eta_g = eta[2];
  res->sigma = sigma;
  res->seconds = secs(t_start, clk::now());
  res->t_eval = C.t_eval;
  res->t_hvp = C.t_hvp;
  res->t_eig = C.t_eig;
  res->t_update = C.t_update;
  res->rank_one_round = rounded;
  if (final_status == MDSDP_ENONFINITE) return MDSDP_ENONFINITE;
  return final_status == MDSDP_OK ? MDSDP_OK : MDSDP_ENOCONV;
}

mdsdp_status mdsdp_solve_batch(int32_t nprob, mdsdp_problem* probs, const mdsdp_options* opt, const int32_t* p0,
                               double* const* Ybufs, mdsdp_result* results, int32_t nworkers) {
  if (nprob < 1 || !probs || !opt || !p0 || !Ybufs || !results) {
    set_error("NULL argument or nprob < 1");
    return MDSDP_EINVAL;
  }
  if (nworkers < 1 || nworkers > 64) {
    set_error("need 1 <= nworkers <= 64");
    return MDSDP_EINVAL;
  }
  int dev = 0;
  MDSDP_HIP(hipGetDevice(&dev));
  for (int i = 0; i < nprob; ++i)
    if (!probs[i] || !Ybufs[i] || probs[i]->device != dev) {
      set_error("problem " + std::to_string(i) + " is NULL, has no Y buffer or lives on another device");
      return MDSDP_EINVAL;
    }
  // work queue: largest problems first (longest-processing-time order)
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a]->n > probs[b]->n; });
  const int nw = std::min(nworkers, nprob);
  std::vector<hipStream_t> streams(nw, nullptr);
  for (int w = 0; w < nw; ++w) {
    hipError_t e = hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int u = 0; u < w; ++u) (void)hipStreamDestroy(streams[u]);
      return hip_fail(e, "hipStreamCreate");
    }
  }
  std::atomic<int> next(0);
  std::vector<mdsdp_status> worker_status(nw, MDSDP_OK);
  std::vector<std::string> worker_err(nw);
  auto work = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= nprob) break;
      const int i = order[t];
      const mdsdp_status st = mdsdp_solve(probs[i], opt, p0[i], Ybufs[i], &results[i], nullptr, 0, streams[w]);
      results[i].status = st;
      if (st != MDSDP_OK && st != MDSDP_ENOCONV && worker_status[w] == MDSDP_OK) {
        worker_status[w] = st;
        worker_err[w] = std::string("problem ") + std::to_string(i) + ": " + mdsdp_last_error();
      }
    }
  };
  std::vector<std::thread> threads;
  for (int w = 1; w < nw; ++w) threads.emplace_back(work, w);
  work(0);
  for (auto& th : threads) th.join();
  for (int w = 0; w < nw; ++w) (void)hipStreamDestroy(streams[w]);
  for (int w = 0; w < nw; ++w)
    if (worker_status[w] != MDSDP_OK) {
      set_error(worker_err[w]);
      return worker_status[w];
    }
  for (int i = 0; i < nprob; ++i)
    if (results[i].status != MDSDP_OK) {
      set_error("problem " + std::to_string(i) + " did not reach the tolerance");
      return MDSDP_ENOCONV;
    }
  return MDSDP_OK;
}

}  // extern "C"
