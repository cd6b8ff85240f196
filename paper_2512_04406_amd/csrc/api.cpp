// C ABI entry points: problem construction (host), layout, and the
// subproblem evaluations, each a short sequence of kernel launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "mdsdp_internal.hpp"

namespace mdsdp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

mdsdp_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return e == hipErrorOutOfMemory ? MDSDP_ENOMEM : MDSDP_EHIP;
}

static mdsdp_status einval(const std::string& m) {
  g_err = m;
  return MDSDP_EINVAL;
}

// ---------------------------------------------------------------------------
// BQP relaxation builder (host)
// ---------------------------------------------------------------------------
static long long binom(long long a, int k) {
  if (k < 0 || a < k) return 0;
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (a - k + i) / i;
  return r;
}

struct Mono {
  int a, b;  // sorted variable indices, -1 = absent
};

static std::vector<Mono> bqp_basis(int q, int order) {
  std::vector<Mono> v;
  v.reserve(1 + q + (size_t)q * (q - 1) / 2);
  v.push_back({-1, -1});
  for (int i = 0; i < q; ++i) v.push_back({i, -1});
  if (order == MDSDP_ORDER_LEX) {
    for (int i = 0; i < q; ++i)
      for (int j = i + 1; j < q; ++j) v.push_back({i, j});
  } else {
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < j; ++i) v.push_back({i, j});
  }
  return v;
}

// class id of x^u x^v: symmetric difference of the index sets, ranked by
// degree, then colex (off[d] + sum_i C(c_i, i)).
static long long bqp_class(const Mono& u, const Mono& v, const long long* off) {
  int e[4];
  int k = 0;
  const int in[4] = {u.a, u.b, v.a, v.b};
  for (int t = 0; t < 4; ++t)
    if (in[t] >= 0) e[k++] = in[t];
  std::sort(e, e + k);
  int out[4];
  int d = 0;
  for (int t = 0; t < k;) {
    if (t + 1 < k && e[t] == e[t + 1]) {
      t += 2;  // x_i^2 = 1
    } else {
      out[d++] = e[t++];
    }
  }
  long long id = off[d];
  for (int i = 0; i < d; ++i) id += binom(out[i], i + 1);
  return id;
}

static void bqp_offsets(int q, long long* off) {
  off[0] = 0;
  for (int d = 0; d < 5; ++d) off[d + 1] = off[d] + binom(q, d);
}

}  // namespace mdsdp

using namespace mdsdp;

extern "C" {

const char* mdsdp_last_error(void) { return g_err.c_str(); }
const char* mdsdp_version(void) { return "manidsdp-gfx950 0.1"; }

mdsdp_status mdsdp_bqp_sizes(int32_t q, int32_t* n_out, int64_t* m_out) {
  if (q < 1 || q > 362) return einval("q must be in [1, 362] (n < 65536)");
  long long off[6];
  bqp_offsets(q, off);
  if (n_out) *n_out = (int32_t)(1 + q + (long long)q * (q - 1) / 2);
  if (m_out) *m_out = off[5];
  return MDSDP_OK;
}

mdsdp_status mdsdp_bqp_classmap(int32_t q, int32_t order, int32_t* cls_out) {
  if (q < 1 || q > 362) return einval("q must be in [1, 362]");
  if (order != MDSDP_ORDER_LEX && order != MDSDP_ORDER_COLEX) return einval("bad basis order");
  if (!cls_out) return einval("cls_out is NULL");
  long long off[6];
  bqp_offsets(q, off);
  std::vector<Mono> B = bqp_basis(q, order);
  const long long n = (long long)B.size();
  long long idx = 0;
  for (long long r = 0; r < n; ++r)
    for (long long c = r; c < n; ++c) cls_out[idx++] = (int32_t)bqp_class(B[r], B[c], off);
  return MDSDP_OK;
}

// ---- Hermitian UCQP relaxation (real embedding) -----------------------------
// An exponent difference alpha - beta of two basis monomials (at most two
// units each) has at most four nonzero components: kept as (index, value)
// pairs sorted by index.  Class representatives have their first nonzero
// component positive; classes are numbered in the ascending order of the
// representatives as dense integer vectors (the comparator below walks the
// sparse pairs in that order).
namespace {
struct UDiff {
  int8_t cnt = 0;
  int16_t idx[4];
  int8_t val[4];
};
bool udiff_less(const UDiff& a, const UDiff& b) {
  int ia = 0, ib = 0;
  while (ia < a.cnt || ib < b.cnt) {
    const int xa = ia < a.cnt ? a.idx[ia] : 1 << 30, xb = ib < b.cnt ? b.idx[ib] : 1 << 30;
    const int i = std::min(xa, xb);
    const int va = xa == i ? a.val[ia] : 0, vb = xb == i ? b.val[ib] : 0;
    if (va != vb) return va < vb;
    if (xa == i) ++ia;
    if (xb == i) ++ib;
  }
  return false;
}
bool udiff_eq(const UDiff& a, const UDiff& b) { return !udiff_less(a, b) && !udiff_less(b, a); }
// basis monomial t: 1 (t = 0), z_i (t = 1 + i), z_i z_j with i <= j (lex order)
std::vector<std::pair<int, int>> ucqp_basis(int q) {
  std::vector<std::pair<int, int>> B{{-1, -1}};
  for (int i = 0; i < q; ++i) B.push_back({i, -1});
  for (int i = 0; i < q; ++i)
    for (int j = i; j < q; ++j) B.push_back({i, j});
  return B;
}
UDiff ucqp_diff(const std::pair<int, int>& a, const std::pair<int, int>& b, int* sign) {
  int idx[4], val[4], k = 0;
  auto add = [&](int i, int v) {
    if (i < 0) return;
    for (int t = 0; t < k; ++t)
      if (idx[t] == i) {
        val[t] += v;
        return;
      }
    idx[k] = i;
    val[k++] = v;
  };
  add(a.first, 1);
  add(a.second, 1);
  add(b.first, -1);
  add(b.second, -1);
  UDiff d;
  for (int t = 0; t < k; ++t)
    if (val[t] != 0) {
      int u = d.cnt;  // insertion sort by index
      while (u > 0 && d.idx[u - 1] > idx[t]) {
        d.idx[u] = d.idx[u - 1];
        d.val[u] = d.val[u - 1];
        --u;
      }
      d.idx[u] = (int16_t)idx[t];
      d.val[u] = (int8_t)val[t];
      ++d.cnt;
    }
  *sign = (d.cnt > 0 && d.val[0] < 0) ? -1 : 1;
  if (*sign < 0)
    for (int t = 0; t < d.cnt; ++t) d.val[t] = (int8_t)-d.val[t];
  return d;
}
struct UcqpMap {
  int nc = 0;
  long long m_re = 0;
  std::vector<int32_t> rep;  // nc x nc: rank of the representative of (a, c)
  std::vector<int8_t> sgn;   // nc x nc: +-1
};
mdsdp_status ucqp_map(int q, UcqpMap& M) {
  const auto B = ucqp_basis(q);
  const int nc = (int)B.size();
  M.nc = nc;
  std::vector<UDiff> all;
  all.reserve((size_t)nc * nc);
  M.sgn.resize((size_t)nc * nc);
  for (int a = 0; a < nc; ++a)
    for (int c = 0; c < nc; ++c) {
      int sg = 1;
      all.push_back(ucqp_diff(B[a], B[c], &sg));
      M.sgn[(size_t)a * nc + c] = (int8_t)sg;
    }
  std::vector<UDiff> reps = all;
  std::sort(reps.begin(), reps.end(), udiff_less);
  reps.erase(std::unique(reps.begin(), reps.end(), udiff_eq), reps.end());
  M.m_re = (long long)reps.size();
  M.rep.resize((size_t)nc * nc);
  for (size_t e = 0; e < all.size(); ++e) {
    const auto it = std::lower_bound(reps.begin(), reps.end(), all[e], udiff_less);
    M.rep[e] = (int32_t)(it - reps.begin());
  }
  return MDSDP_OK;
}
}  // namespace

mdsdp_status mdsdp_ucqp_sizes(int32_t q, int32_t* n_out, int64_t* m_out) {
  if (q < 1 || q > 60) return einval("q must be in [1, 60]");
  const int nc = 1 + q + q * (q + 1) / 2;
  if (n_out) *n_out = 2 * nc;
  if (m_out) {
    UcqpMap M;
    mdsdp_status st = ucqp_map(q, M);
    if (st != MDSDP_OK) return st;
    *m_out = 2 * M.m_re - 1;
  }
  return MDSDP_OK;
}

mdsdp_status mdsdp_ucqp_structure(int32_t q, int32_t* cls_out, int8_t* coef_out) {
  if (q < 1 || q > 60) return einval("q must be in [1, 60]");
  if (!cls_out || !coef_out) return einval("NULL argument");
  UcqpMap M;
  mdsdp_status st = ucqp_map(q, M);
  if (st != MDSDP_OK) return st;
  const int nc = M.nc;
  const long long n = 2LL * nc;
  long long idx = 0;
  for (long long r = 0; r < n; ++r)
    for (long long c = r; c < n; ++c, ++idx) {
      const int a = (int)(r % nc), b = (int)(c % nc);
      const bool rim = r >= nc, cim = c >= nc;
      const int k = M.rep[(size_t)a * nc + b];
      if (rim == cim) {  // Re M in both diagonal blocks
        cls_out[idx] = k;
        coef_out[idx] = 1;
      } else if (k == 0) {  // imaginary part of a diagonal-class entry: no class
        cls_out[idx] = 0;
        coef_out[idx] = 0;
      } else {  // (nc + a, b): +s Im M[a][b];  (a, nc + b): -s Im M[a][b]
        const int s = M.sgn[(size_t)a * nc + b];
        cls_out[idx] = (int32_t)(M.m_re + k - 1);
        coef_out[idx] = (int8_t)(rim ? s : -s);
      }
    }
  return MDSDP_OK;
}

mdsdp_status mdsdp_ucqp_b(int32_t q, const double* Qre, const double* Qim, double* b) {
  if (q < 1 || q > 60) return einval("q must be in [1, 60]");
  if (!Qre || !Qim || !b) return einval("NULL argument");
  UcqpMap M;
  mdsdp_status st = ucqp_map(q, M);
  if (st != MDSDP_OK) return st;
  const long long m = 2 * M.m_re - 1;
  for (long long g = 0; g < m; ++g) b[g] = 0.0;
  for (int i = 0; i < q; ++i) b[0] += Qre[(size_t)i * q + i];
  // class of e_i - e_j (i < j): the pair (z_i, z_j) of basis rows 1 + i, 1 + j
  for (int i = 0; i < q; ++i)
    for (int j = i + 1; j < q; ++j) {
      const int k = M.rep[(size_t)(1 + i) * M.nc + (1 + j)];
      b[k] += 2.0 * Qre[(size_t)i * q + j];
      b[M.m_re + k - 1] += 2.0 * Qim[(size_t)i * q + j];
    }
  return MDSDP_OK;
}

mdsdp_status mdsdp_bqp_b(int32_t q, const double* Q, const double* c, double* b) {
  if (q < 1 || q > 362) return einval("q must be in [1, 362]");
  if (!Q || !c || !b) return einval("NULL argument");
  long long off[6];
  bqp_offsets(q, off);
  for (long long g = 0; g < off[5]; ++g) b[g] = 0.0;
  double tr = 0.0;
  for (int i = 0; i < q; ++i) tr += Q[(size_t)i * q + i];
  b[0] = tr;
  for (int i = 0; i < q; ++i) b[off[1] + i] = c[i];
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < j; ++i) b[off[2] + binom(i, 1) + binom(j, 2)] = Q[(size_t)i * q + j] + Q[(size_t)j * q + i];
  return MDSDP_OK;
}

}  // extern "C"

namespace mdsdp {

static void free_problem(mdsdp_problem P) {
  if (!P) return;
  void* ptrs[] = {P->cls,      P->cls32,  P->Xt,     P->Xt32,    P->Ct,      P->segs,   P->seg_start, P->cy,
                  P->Cavg,     P->ab64,   P->ab32,    P->invc,    P->bvec,    P->sacc,   P->Yp,        P->Up,
                  P->bqp4_items, P->bqp1_items, P->bqp2_items, P->bqpP1, P->bqpT, P->bqpStar,
                  P->zvec,     P->zmult,  P->rowpart, P->colpart, P->wgpart, P->zpart,     P->gram,
                  P->gpart,    P->scal,   P->bound,   P->dotpart, (void*)P->dotptr, P->lz_V, P->lz_w,
                  P->lz_h,     P->lz_hpart, P->work,   P->Xt2,     P->lrbuf};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (P->hbuf) (void)hipHostFree(P->hbuf);
  for (auto& r : P->timer.recs) {
    if (r.ev0) (void)hipEventDestroy(r.ev0);
    if (r.ev1) (void)hipEventDestroy(r.ev1);
  }
  delete P;
}

template <typename T>
static mdsdp_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  return MDSDP_OK;
}

#define TRY(x)                        \
  do {                                \
    mdsdp_status st__ = (x);          \
    if (st__ != MDSDP_OK) {           \
      free_problem(P);                \
      return st__;                    \
    }                                 \
  } while (0)

static mdsdp_status check_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    return MDSDP_EUNSUPPORTED;
  }
  return MDSDP_OK;
}

// Builds the device problem from a packed-upper class map (row-major).
// coef (nullable = all +1): coefficient of each packed entry in its A_gamma,
// +1, -1, or 0 for an entry in no class (its class id is then ignored)
static mdsdp_status create_from_packed(int n, long long m, const int32_t* cls, const int8_t* coef,
                                       const double* b, const double* C, mdsdp_problem* out) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  if (n < 1 || n >= 65536) return einval("n must be in [1, 65535]");
  if (m < 1 || m > (long long)CLS_MASK) return einval("m out of range");
  if (!cls || !b) return einval("cls and b are required");
  for (long long g = 0; g < m; ++g)
    if (!std::isfinite(b[g])) {
      set_error("b has a non-finite entry at " + std::to_string(g));
      return MDSDP_ENONFINITE;
    }
  if (C)
    for (long long i = 0; i < (long long)n * n; ++i)
      if (!std::isfinite(C[i])) {
        set_error("C has a non-finite entry at " + std::to_string(i));
        return MDSDP_ENONFINITE;
      }

  const long long ne = (long long)n * (n + 1) / 2;
  std::vector<long long> cnt(m, 0);
  {
    long long idx = 0;
    for (long long r = 0; r < n; ++r)
      for (long long c = r; c < n; ++c, ++idx) {
        if (coef && coef[idx] == 0) continue;
        const long long g = cls[idx];
        if (g < 0 || g >= m) return einval("class id out of range at packed index " + std::to_string(idx));
        cnt[g] += (r == c) ? 1 : 2;  // sum of w_e^2 over the ordered entries, w_e = +-1
      }
  }
  long long kmax = 0;
  for (long long g = 0; g < m; ++g) {
    if (cnt[g] == 0) return einval("class " + std::to_string(g) + " is empty (AA* singular)");
    kmax = std::max(kmax, cnt[g]);
  }
  mdsdp_status st = check_device();
  if (st != MDSDP_OK) return st;

  mdsdp_problem P = new mdsdp_problem_s();
  (void)hipGetDevice(&P->device);
  P->n = n;
  P->m = m;
  P->nb = (n + TS - 1) / TS;
  P->npad = P->nb * TS;
  P->ntiles = P->nb * (P->nb + 1) / 2;
  P->nslots = (long long)P->ntiles * TSLOTS;
  P->kmax = kmax;
  P->hasC = C != nullptr;
  double nb2 = 0.0;
  for (long long g = 0; g < m; ++g) nb2 += b[g] * b[g];
  P->normb = sqrt(nb2);

  // tile-major class words and C
  std::vector<uint32_t> hcls(P->nslots);
  std::vector<double> hC;
  if (C) hC.assign(P->nslots, 0.0);
  std::vector<char> seen(m, 0);
  double nC2 = 0.0;
  for (int J = 0; J < P->nb; ++J)
    for (int I = 0; I <= J; ++I) {
      const long long t = (long long)J * (J + 1) / 2 + I;
      for (int sb = 0; sb < 16; ++sb)
        for (int e = 0; e < 256; ++e) {
          const long long s = t * TSLOTS + sb * 256 + e;
          const int r = I * TS + (sb >> 2) * SB + (e >> 4);
          const int c = J * TS + (sb & 3) * SB + (e & 15);
          if (r >= n || c >= n) {
            hcls[s] = 0xFFFFFFFFu;
            continue;
          }
          const long long rr = std::min(r, c), cc = std::max(r, c);
          const long long pidx = rr * n - rr * (rr - 1) / 2 + (cc - rr);
          const int8_t we = coef ? coef[pidx] : (int8_t)1;
          const uint32_t g = we == 0 ? 0u : (uint32_t)cls[pidx];
          uint32_t wv = g | (we == 0 ? FREE_BIT : (we < 0 ? NEG_BIT : 0u));
          // owner: first slot of the class in slot order (diagonal tiles hold
          // both (r, c) and (c, r); either may own)
          if (we != 0 && !seen[g]) {
            seen[g] = 1;
            wv |= OWNER_BIT;
          }
          hcls[s] = wv;
          if (C) hC[s] = C[(size_t)r * n + c];
        }
    }
  if (C)
    for (long long i = 0; i < (long long)n * n; ++i) nC2 += C[i] * C[i];
  P->normC = sqrt(nC2);

  // per-class constants
  std::vector<double2> hcy(m);
  std::vector<double> hinvc(m);
  for (long long g = 0; g < m; ++g) {
    hcy[g] = make_double2(b[g] / (double)cnt[g], 0.0);
    hinvc[g] = 1.0 / (double)cnt[g];
  }
  long long last_b = 0;
  for (long long g = 0; g < m; ++g)
    if (b[g] != 0.0) last_b = g + 1;
  P->bty_range = last_b;
  std::vector<double> hCavg;
  if (C) {
    hCavg.assign(m, 0.0);
    long long idx = 0;
    for (long long r = 0; r < n; ++r)
      for (long long c = r; c < n; ++c, ++idx) {
        const double we = coef ? (double)coef[idx] : 1.0;
        if (we != 0.0) hCavg[cls[idx]] += we * (r == c ? 1.0 : 2.0) * C[(size_t)r * n + c];
      }
    for (long long g = 0; g < m; ++g) hCavg[g] /= (double)cnt[g];
  }

  // segments: column block J, row blocks in chunks of SEGLEN
  const int SEGLEN = 4;
  std::vector<Seg> hseg;
  std::vector<int> hstart(P->nb + 1, 0);
  for (int J = 0; J < P->nb; ++J) {
    hstart[J] = (int)hseg.size();
    for (int I0 = 0; I0 <= J; I0 += SEGLEN) hseg.push_back({J, I0, std::min(J, I0 + SEGLEN - 1)});
  }
  hstart[P->nb] = (int)hseg.size();
  P->nseg = (int)hseg.size();

  TRY(dalloc(&P->cls, P->nslots));
  TRY(dalloc(&P->Xt, P->nslots));
  TRY(dalloc(&P->Xt32, P->nslots));
  TRY(dalloc(&P->cls32, P->nslots));
  if (C) TRY(dalloc(&P->Ct, P->nslots));
  TRY(dalloc(&P->segs, P->nseg));
  TRY(dalloc(&P->seg_start, P->nb + 1));
  TRY(dalloc(&P->cy, m));
  TRY(dalloc(&P->ab64, m));
  TRY(dalloc(&P->ab32, m));
  TRY(dalloc(&P->invc, m));
  TRY(dalloc(&P->bvec, m));
  TRY(dalloc(&P->sacc, m));
  if (C) TRY(dalloc(&P->Cavg, m));
  TRY(dalloc((double**)&P->Yp, (size_t)P->npad * PMAX));
  TRY(dalloc((double**)&P->Up, (size_t)P->npad * PMAX));
  TRY(dalloc(&P->zvec, n));
  TRY(dalloc(&P->zmult, n));
  TRY(dalloc(&P->rowpart, (size_t)P->ntiles * 64 * PMAX));
  TRY(dalloc(&P->colpart, (size_t)P->nseg * 64 * PMAX));
  TRY(dalloc(&P->wgpart, (size_t)P->nseg * 4));
  TRY(dalloc(&P->zpart, (size_t)(n * PMAX + 255) / 256 + 1));
  TRY(dalloc(&P->lrbuf, (size_t)n * PMAX));
  TRY(dalloc(&P->gram, 2 * GRAM_U));
  TRY(dalloc(&P->gpart, GP_SIZE));
  TRY(dalloc(&P->scal, SC_COUNT));
  TRY(dalloc(&P->bound, 2));
  P->dot_nblk = 256;
  TRY(dalloc(&P->dotpart, (size_t)P->dot_nblk * 8));
  TRY(dalloc((double**)&P->dotptr, 16));
  {
    hipError_t eh = hipHostMalloc((void**)&P->hbuf, HBUF_LEN * sizeof(double), hipHostMallocDefault);
    if (eh != hipSuccess) {
      mdsdp_status s2 = hip_fail(eh, "hipHostMalloc");
      free_problem(P);
      return s2;
    }
  }

  hipError_t e;
#define CP(dst, src, bytes)                                      \
  e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);         \
  if (e != hipSuccess) {                                         \
    mdsdp_status s2 = hip_fail(e, "hipMemcpy");                  \
    free_problem(P);                                             \
    return s2;                                                   \
  }
  CP(P->cls, hcls.data(), P->nslots * sizeof(uint32_t));
  {
    std::vector<uint32_t> h32(P->nslots);
    for (long long q = 0; q < P->nslots; ++q) h32[slot32((size_t)q)] = hcls[q];
    CP(P->cls32, h32.data(), P->nslots * sizeof(uint32_t));
  }
  if (C) CP(P->Ct, hC.data(), P->nslots * sizeof(double));
  CP(P->segs, hseg.data(), hseg.size() * sizeof(Seg));
  CP(P->seg_start, hstart.data(), hstart.size() * sizeof(int));
  CP(P->cy, hcy.data(), m * sizeof(double2));
  CP(P->invc, hinvc.data(), m * sizeof(double));
  CP(P->bvec, b, m * sizeof(double));
  if (C) CP(P->Cavg, hCavg.data(), m * sizeof(double));
#undef CP
  TRY(hipMemset(P->sacc, 0, m * sizeof(long long)) == hipSuccess ? MDSDP_OK : MDSDP_EHIP);
  TRY(hipMemset(P->ab64, 0, m * sizeof(double2)) == hipSuccess ? MDSDP_OK : MDSDP_EHIP);
  TRY(hipMemset(P->scal, 0, SC_COUNT * sizeof(double)) == hipSuccess ? MDSDP_OK : MDSDP_EHIP);
  TRY(hipMemset(P->zvec, 0, n * sizeof(double)) == hipSuccess ? MDSDP_OK : MDSDP_EHIP);
  TRY(hipMemset(P->zmult, 0, n * sizeof(double)) == hipSuccess ? MDSDP_OK : MDSDP_EHIP);
  TRY(launch_set_dense(P, nullptr, nullptr));
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    mdsdp_status s2 = hip_fail(e, "hipDeviceSynchronize");
    free_problem(P);
    return s2;
  }
  P->sigma = 1.0;
  *out = P;
  return MDSDP_OK;
}

static mdsdp_status check_p(mdsdp_problem P, int p) {
  if (!P) return einval("problem is NULL");
  if (p < 1 || p > PMAX) {
    set_error("p must be in [1, " + std::to_string(PMAX) + "]");
    return p < 1 ? MDSDP_EINVAL : MDSDP_EUNSUPPORTED;
  }
  return MDSDP_OK;
}

mdsdp_status hvp_impl(mdsdp_problem P, int p, int prec, const double* Y, const double* U, double* HU, int riem,
                      hipStream_t s, double* dotpart, double* dot_out) {
  mdsdp_status st = check_p(P, p);
  if (st != MDSDP_OK) return st;
  if (!Y || !U || !HU) return einval("NULL argument");
  if (prec != MDSDP_FP64 && prec != MDSDP_FP32) return einval("bad precision");
  const bool fp32 = prec == MDSDP_FP32;
  if ((st = launch_stage(P, p, Y, U, fp32, s)) != MDSDP_OK) return st;
  if ((st = launch_classsum_Z(P, fp32, s)) != MDSDP_OK) return st;
  if ((st = fp32 ? launch_hvp32(P, s) : launch_resid(P, M_HVP, false, s)) != MDSDP_OK) return st;
  P->last_hvp_prec = prec;
  // the Gram matrices feed only the row finaliser: launched after the long
  // passes, the host enqueues them while those run
  const bool need_yy = !(P->gram_yy_valid && P->gram_yy_p == p);
  if ((st = launch_gram(P, p, Y, U, s, need_yy)) != MDSDP_OK) return st;
  P->gram_yy_valid = true;
  P->gram_yy_p = p;
  return launch_rowfinal_hvp(P, p, fp32, Y, U, HU, riem ? 1 : 0, s, dotpart, dot_out);
}

}  // namespace mdsdp

extern "C" {

mdsdp_status mdsdp_create_classmap(int32_t n, int64_t m, const int32_t* cls, const double* b, const double* C,
                                   mdsdp_problem* out) {
  return create_from_packed(n, m, cls, nullptr, b, C, out);
}

mdsdp_status mdsdp_create_bqp(int32_t q, int32_t order, const double* Q, const double* c, mdsdp_problem* out) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  mdsdp_status st = mdsdp_bqp_sizes(q, &n, &m);
  if (st != MDSDP_OK) return st;
  if (order != MDSDP_ORDER_LEX && order != MDSDP_ORDER_COLEX) return einval("bad basis order");
  if (!Q || !c) return einval("Q and c are required");
  for (long long i = 0; i < (long long)q * q; ++i)
    if (!std::isfinite(Q[i])) {
      set_error("Q has a non-finite entry at " + std::to_string(i));
      return MDSDP_ENONFINITE;
    }
  for (int i = 0; i < q; ++i)
    if (!std::isfinite(c[i])) {
      set_error("c has a non-finite entry at " + std::to_string(i));
      return MDSDP_ENONFINITE;
    }
  std::vector<int32_t> cls((size_t)n * (n + 1) / 2);
  std::vector<double> b(m);
  if ((st = mdsdp_bqp_classmap(q, order, cls.data())) != MDSDP_OK) return st;
  if ((st = mdsdp_bqp_b(q, Q, c, b.data())) != MDSDP_OK) return st;
  mdsdp_problem P = nullptr;
  if ((st = create_from_packed(n, m, cls.data(), nullptr, b.data(), nullptr, &P)) != MDSDP_OK) return st;
  if (order == MDSDP_ORDER_COLEX && q >= 1) {
    // structured class-sum kernels.  Degree-4 pass 1: items (d, c0, t0), a
    // 16-block of c < d and 64 pair rows t below C(c0 + 15, 2); pass 2: one
    // item per (c, d), 2 <= c < d < q, the largest c (most work) first.
    P->bqp_q = q;
    bqp_offsets(q, P->bqp_off);
    std::vector<int4> items1;
    for (int d = 3; d < q; ++d)
      for (int c0 = 0; c0 < d; c0 += 16) {
        const long long cm = std::min(c0 + 15, d - 1);
        if (cm < 2) continue;
        const long long nt = cm * (cm - 1) / 2;
        for (long long t0 = 0; t0 < nt; t0 += 64) items1.push_back(make_int4(d, c0, (int)t0, 0));
      }
    std::vector<int4> items4;  // single-pass items: 16-blocks of d > c, of b < c and of a <= b
    for (int cc = 2; cc <= q - 2; ++cc)
      for (int d0 = cc + 1; d0 < q; d0 += 16)
        for (int b0 = 0; b0 < cc; b0 += 16)
          for (int a0 = 0; a0 <= b0; a0 += 16) items4.push_back(make_int4(cc, d0, a0, b0));
    std::vector<int2> items2;
    for (int cc = q - 2; cc >= 2; --cc)
      for (int d = cc + 1; d < q; ++d) items2.push_back(make_int2(cc, d));
    P->bqp4_n = (int)items4.size();
    P->bqp1_n = (int)items1.size();
    P->bqp2_n = (int)items2.size();
    const long long n4 = std::max<long long>(1, (long long)q * (q - 1) * (q - 2) * (q - 3) / 24);
    hipError_t e = hipSuccess;
    if (!items4.empty()) {
      e = hipMalloc((void**)&P->bqp4_items, items4.size() * sizeof(int4));
      if (e == hipSuccess)
        e = hipMemcpy(P->bqp4_items, items4.data(), items4.size() * sizeof(int4), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !items1.empty()) {
      e = hipMalloc((void**)&P->bqp1_items, items1.size() * sizeof(int4));
      if (e == hipSuccess)
        e = hipMemcpy(P->bqp1_items, items1.data(), items1.size() * sizeof(int4), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !items2.empty()) {
      e = hipMalloc((void**)&P->bqp2_items, items2.size() * sizeof(int2));
      if (e == hipSuccess)
        e = hipMemcpy(P->bqp2_items, items2.data(), items2.size() * sizeof(int2), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&P->bqpP1, (size_t)n4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&P->bqpT, (size_t)n * (q + 1) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&P->bqpStar, (size_t)STAR_LG * q * q * sizeof(double));
    if (e != hipSuccess) {
      st = hip_fail(e, "bqp tables");
      free_problem(P);
      return st;
    }
  }
  *out = P;
  return MDSDP_OK;
}

mdsdp_status mdsdp_create_ucqp(int32_t q, const double* Qre, const double* Qim, mdsdp_problem* out) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  if (q < 1 || q > 60) return einval("q must be in [1, 60]");
  if (!Qre || !Qim) return einval("Qre and Qim are required");
  for (long long i = 0; i < (long long)q * q; ++i)
    if (!std::isfinite(Qre[i]) || !std::isfinite(Qim[i])) {
      set_error("Q has a non-finite entry at " + std::to_string(i));
      return MDSDP_ENONFINITE;
    }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      if (Qre[(size_t)i * q + j] != Qre[(size_t)j * q + i] || Qim[(size_t)i * q + j] != -Qim[(size_t)j * q + i])
        return einval("Q must be Hermitian");
  int32_t n = 0;
  int64_t m = 0;
  mdsdp_status st = mdsdp_ucqp_sizes(q, &n, &m);
  if (st != MDSDP_OK) return st;
  const long long ne = (long long)n * (n + 1) / 2;
  std::vector<int32_t> cls(ne);
  std::vector<int8_t> coef(ne);
  std::vector<double> b(m);
  if ((st = mdsdp_ucqp_structure(q, cls.data(), coef.data())) != MDSDP_OK) return st;
  if ((st = mdsdp_ucqp_b(q, Qre, Qim, b.data())) != MDSDP_OK) return st;
  return create_from_packed(n, m, cls.data(), coef.data(), b.data(), nullptr, out);
}

mdsdp_status mdsdp_create_sparse_A(int32_t n, int64_t m, int64_t nnz, const int32_t* cls, const int32_t* row,
                                   const int32_t* col, const double* val, const double* b, const double* C,
                                   mdsdp_problem* out) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  if (n < 1 || n >= 65536) return einval("n must be in [1, 65535]");
  if (nnz < 0 || !cls || !row || !col || !val) return einval("sparse A arrays required");
  const long long ne = (long long)n * (n + 1) / 2;
  std::vector<int32_t> packed(ne, -1);
  std::vector<int8_t> coef(ne, 0);  // entries no triplet covers stay in no class
  bool unit = true;
  for (long long t = 0; t < nnz; ++t) {
    const long long r = row[t], c = col[t];
    if (r < 0 || c < r || c >= n) return einval("sparse A entry not in the upper triangle");
    if (cls[t] < 0 || cls[t] >= m) return einval("sparse A class out of range");
    if (!std::isfinite(val[t])) {
      set_error("sparse A has a non-finite value at triplet " + std::to_string(t));
      return MDSDP_ENONFINITE;
    }
    if (val[t] != 1.0 && val[t] != -1.0) {
      set_error("only coefficients +1 and -1 are supported in the A_gamma (value " + std::to_string(val[t]) +
                " at triplet " + std::to_string(t) + ")");
      return MDSDP_EUNSUPPORTED;
    }
    if (val[t] != 1.0) unit = false;
    const long long pidx = r * n - r * (r - 1) / 2 + (c - r);
    if (packed[pidx] >= 0) {
      set_error("sparse A supports overlap at (" + std::to_string(r) + ", " + std::to_string(c) + ")");
      return MDSDP_ENOTORTH;
    }
    packed[pidx] = cls[t];
    coef[pidx] = val[t] > 0.0 ? 1 : -1;
  }
  bool covered = true;
  for (long long i = 0; i < ne; ++i)
    if (packed[i] < 0) {
      covered = false;
      packed[i] = 0;
    }
  return create_from_packed(n, m, packed.data(), (unit && covered) ? nullptr : coef.data(), b, C, out);
}

mdsdp_status mdsdp_destroy(mdsdp_problem P) {
  if (!P) return einval("problem is NULL");
  (void)hipDeviceSynchronize();
  free_problem(P);
  return MDSDP_OK;
}

mdsdp_status mdsdp_problem_info(mdsdp_problem P, int32_t* n, int64_t* m, int64_t* n_slots, int32_t* n_tiles) {
  if (!P) return einval("problem is NULL");
  if (n) *n = P->n;
  if (m) *m = P->m;
  if (n_slots) *n_slots = P->nslots;
  if (n_tiles) *n_tiles = P->ntiles;
  return MDSDP_OK;
}

mdsdp_status mdsdp_set_multiplier(mdsdp_problem P, const double* Xt_dev, double sigma, void* stream) {
  if (!P) return einval("problem is NULL");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return einval("sigma must be positive and finite");
  if (sigma != P->sigma) P->a32_valid = P->a64_valid = false;
  P->sigma = sigma;
  // a new multiplier starts a new state: clear the sticky non-finite flag
  // (a fill kernel, so that the call can be recorded into a HIP graph)
  mdsdp_status st = vec_fill(1, 0.0, P->scal + SC_NONFIN, (hipStream_t)stream);
  if (st != MDSDP_OK) return st;
  return launch_set_dense(P, Xt_dev, (hipStream_t)stream);
}

mdsdp_status mdsdp_set_direct(mdsdp_problem P, int32_t on, int32_t p, const double* Y_dev, void* stream) {
  if (!P) return einval("problem is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (on && Y_dev) {
    // y^k = class averages of Z^k = Y Y^T + C (the ADMM y-update at Y)
    mdsdp_status st = check_p(P, p);
    if (st != MDSDP_OK) return st;
    P->frozen = false;
    if ((st = launch_stage(P, p, Y_dev, nullptr, false, s)) != MDSDP_OK) return st;
    if ((st = launch_classsum_S(P, s)) != MDSDP_OK) return st;
  }
  P->frozen = on != 0;
  P->ycoef_zero = false;
  P->a32_valid = P->a64_valid = false;
  return MDSDP_OK;
}

mdsdp_status mdsdp_sync_status(mdsdp_problem P, void* stream) {
  if (!P) return einval("problem is NULL");
  hipStream_t s = (hipStream_t)stream;
  double flag = 0.0;
  MDSDP_HIP(hipMemcpyAsync(P->hbuf + 56, P->scal + SC_NONFIN, sizeof(double), hipMemcpyDeviceToHost, s));
  MDSDP_HIP(hipStreamSynchronize(s));
  flag = P->hbuf[56];
  if (flag != 0.0) {
    set_error("a non-finite value was met (multiplier, cost, Hessian-vector product or multiplier update) "
              "since the last mdsdp_set_multiplier");
    return MDSDP_ENONFINITE;
  }
  return MDSDP_OK;
}

mdsdp_status mdsdp_get_multiplier(mdsdp_problem P, double* Xt_dev, void* stream) {
  if (!P || !Xt_dev) return einval("NULL argument");
  return launch_get_dense(P, Xt_dev, false, (hipStream_t)stream);
}

mdsdp_status mdsdp_set_sigma(mdsdp_problem P, double sigma) {
  if (!P) return einval("problem is NULL");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return einval("sigma must be positive and finite");
  if (sigma != P->sigma) P->a32_valid = P->a64_valid = false;
  P->sigma = sigma;
  return MDSDP_OK;
}

mdsdp_status mdsdp_cost_grad(mdsdp_problem P, int32_t p, const double* Y, double* f, double* egrad,
                             double* rgrad, void* stream) {
  mdsdp_status st = check_p(P, p);
  if (st != MDSDP_OK) return st;
  if (!Y) return einval("Y is NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = launch_stage(P, p, Y, nullptr, false, s)) != MDSDP_OK) return st;
  if (!P->frozen) {  // the direct-DSDP subproblem keeps the stale class averages y^k
    if ((st = launch_classsum_S(P, s)) != MDSDP_OK) return st;
    if ((st = launch_bty(P, s)) != MDSDP_OK) return st;
  }
  if ((st = launch_resid(P, M_GRAD, false, s)) != MDSDP_OK) return st;
  return launch_rowfinal_grad(P, p, Y, egrad, rgrad, f, s);
}

mdsdp_status mdsdp_hvp(mdsdp_problem P, int32_t p, int32_t prec, const double* Y, const double* U, double* HU,
                       int32_t riemannian, void* stream) {
  return hvp_impl(P, p, prec, Y, U, HU, riemannian, (hipStream_t)stream);
}

mdsdp_status mdsdp_class_average(mdsdp_problem P, int32_t p, const double* Y, double* y, void* stream) {
  mdsdp_status st = check_p(P, p);
  if (st != MDSDP_OK) return st;
  if (!Y || !y) return einval("NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if ((st = launch_stage(P, p, Y, nullptr, false, s)) != MDSDP_OK) return st;
  if ((st = launch_classsum_S(P, s)) != MDSDP_OK) return st;
  return launch_y_export(P, y, s);
}

mdsdp_status mdsdp_retract(int32_t n, int32_t p, const double* Y, const double* V, double t, double* Yout,
                           void* stream) {
  if (n < 1 || p < 1) return einval("bad sizes");
  if (!Y || !V || !Yout) return einval("NULL argument");
  return launch_retract(n, p, Y, V, t, Yout, (hipStream_t)stream);
}

mdsdp_status mdsdp_project_tangent(int32_t n, int32_t p, const double* Y, const double* U, double* out,
                                   void* stream) {
  if (n < 1 || p < 1) return einval("bad sizes");
  if (!Y || !U || !out) return einval("NULL argument");
  return launch_project(n, p, Y, U, out, (hipStream_t)stream);
}

mdsdp_status mdsdp_update_multiplier(mdsdp_problem P, int32_t p, const double* Y, double* y, double* z,
                                     double* kkt, void* stream) {
  mdsdp_status st = check_p(P, p);
  if (st != MDSDP_OK) return st;
  if (!Y) return einval("Y is NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((st = launch_stage(P, p, Y, nullptr, false, s)) != MDSDP_OK) return st;
  if ((st = launch_classsum_S(P, s)) != MDSDP_OK) return st;
  if ((st = launch_bty(P, s)) != MDSDP_OK) return st;
  if (y && (st = launch_y_export(P, y, s)) != MDSDP_OK) return st;
  if ((st = launch_resid(P, M_MULT, false, s)) != MDSDP_OK) return st;
  return launch_rowfinal_mult(P, p, Y, z, kkt, s);
}

mdsdp_status mdsdp_certificate_matvec(mdsdp_problem P, int32_t k, const double* V, double* XV, void* stream) {
  mdsdp_status st = check_p(P, k);
  if (st != MDSDP_OK) return st;
  if (!V || !XV) return einval("NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if ((st = launch_stage(P, k, V, V, false, s)) != MDSDP_OK) return st;
  if ((st = launch_resid(P, M_XMV, false, s)) != MDSDP_OK) return st;
  return launch_rowfinal_xmv(P, k, V, XV, s);
}

mdsdp_status mdsdp_adjoint_C(mdsdp_problem P, double* dC, void* stream) {
  if (!P || !dC) return einval("NULL argument");
  return launch_get_dense(P, dC, true, (hipStream_t)stream);
}

mdsdp_status mdsdp_export_classmap(mdsdp_problem P, int32_t* out) {
  if (!P || !out) return einval("NULL argument");
  std::vector<uint32_t> h(P->nslots);
  MDSDP_HIP(hipMemcpy(h.data(), P->cls, P->nslots * sizeof(uint32_t), hipMemcpyDeviceToHost));
  const int n = P->n;
  for (int J = 0; J < P->nb; ++J)
    for (int I = 0; I <= J; ++I) {
      const long long t = (long long)J * (J + 1) / 2 + I;
      for (int sb = 0; sb < 16; ++sb)
        for (int e = 0; e < 256; ++e) {
          const int r = I * TS + (sb >> 2) * SB + (e >> 4);
          const int c = J * TS + (sb & 3) * SB + (e & 15);
          if (r >= n || c >= n || r > c) continue;
          const long long pidx = (long long)r * n - (long long)r * (r - 1) / 2 + (c - r);
          out[pidx] = (int32_t)(h[t * TSLOTS + sb * 256 + e] & CLS_MASK);
        }
    }
  return MDSDP_OK;
}

mdsdp_status mdsdp_export_multiplier_packed(mdsdp_problem P, double* out) {
  if (!P || !out) return einval("NULL argument");
  std::vector<double> h(P->nslots);
  MDSDP_HIP(hipMemcpy(h.data(), P->Xt, P->nslots * sizeof(double), hipMemcpyDeviceToHost));
  const int n = P->n;
  for (int J = 0; J < P->nb; ++J)
    for (int I = 0; I <= J; ++I) {
      const long long t = (long long)J * (J + 1) / 2 + I;
      for (int sb = 0; sb < 16; ++sb)
        for (int e = 0; e < 256; ++e) {
          const int r = I * TS + (sb >> 2) * SB + (e >> 4);
          const int c = J * TS + (sb & 3) * SB + (e & 15);
          if (r >= n || c >= n || r > c) continue;
          const long long pidx = (long long)r * n - (long long)r * (r - 1) / 2 + (c - r);
          out[pidx] = h[t * TSLOTS + sb * 256 + e];
        }
    }
  return MDSDP_OK;
}

mdsdp_status mdsdp_time_product_pass(mdsdp_problem P, int32_t reps, double* us_out, void* stream) {
  if (!P || !us_out) return einval("NULL argument");
  if (reps < 1) return einval("reps must be >= 1");
  if (P->last_hvp_prec < 0) return einval("call mdsdp_hvp first");
  hipStream_t s = (hipStream_t)stream;
  const bool fp32 = P->last_hvp_prec == MDSDP_FP32;
  const bool was_on = P->timer.on;
  P->timer.on = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MDSDP_HIP(hipEventCreate(&e0));
  MDSDP_HIP(hipEventCreate(&e1));
  mdsdp_status st = MDSDP_OK;
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps && st == MDSDP_OK; ++i) st = fp32 ? launch_hvp32(P, s) : launch_resid(P, M_HVP, false, s);
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->timer.on = was_on;
  if (st != MDSDP_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
  *us_out = 1e3 * (double)ms / reps;
  return MDSDP_OK;
}

mdsdp_status mdsdp_enable_timing(mdsdp_problem P, int32_t on) {
  if (!P) return einval("problem is NULL");
  P->timer.on = on != 0;
  for (auto& r : P->timer.recs) {
    if (r.ev0) (void)hipEventDestroy(r.ev0);
    if (r.ev1) (void)hipEventDestroy(r.ev1);
  }
  P->timer.recs.clear();
  P->timer.open.clear();
  return MDSDP_OK;
}

// Returns, per timed kernel launch since the last call, the elapsed time in
// ms (synchronises).  Names are concatenated as "name;name;..." in the error
// buffer for diagnostics.
mdsdp_status mdsdp_kernel_times(mdsdp_problem P, double* ms_out, int32_t cap, int32_t* count) {
  if (!P || !count) return einval("NULL argument");
  MDSDP_HIP(hipDeviceSynchronize());
  std::string names;
  int k = 0;
  auto& T = P->timer;
  for (auto& r : T.recs) {
    if (!r.ev0 || !r.ev1) continue;
    float ms = 0.f;
    MDSDP_HIP(hipEventElapsedTime(&ms, r.ev0, r.ev1));
    if (k < cap && ms_out) ms_out[k] = ms;
    names += r.name + ";";
    ++k;
  }
  for (auto& r : T.recs) {
    if (r.ev0) (void)hipEventDestroy(r.ev0);
    if (r.ev1) (void)hipEventDestroy(r.ev1);
  }
  T.recs.clear();
  T.open.clear();
  *count = k;
  g_err = names;
  return MDSDP_OK;
}

}  // extern "C"
