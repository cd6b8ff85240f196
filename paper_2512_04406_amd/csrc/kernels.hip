// HIP kernels (gfx950) of the ManiDSDP subproblem library.
//
// Passes over the tile-major packed upper triangle (layout in mdsdp_internal.hpp):
//
//  k_classsum<T, ZMODE>  class sums of Z = Y Y^T (ZMODE = 0) or of
//      Z' = Y U^T + U Y^T (ZMODE = 1): the A(.) of the variable projection
//      y(S) = (AA*)^{-1} A(S + C) (section 3) and of the HVP's Q(Y U^T + U Y^T)
//      (Proposition prop).  16 x 16 blocks of Z come from MFMA 16x16x4 on
//      LDS-staged 64-row slices of Y and U; every entry is added to its class
//      with a 64-bit fixed-point atomic (integer addition is associative, so
//      the sums are bit-reproducible whatever the scheduling).  Sums are
//      double-buffered; the class's "owner" slot clears the other buffer.
//
//  k_resid<T, MODE>  per-entry coefficient and symmetric product pass:
//      GRAD: r = Z - y, G = Xt + D + sigma r (Lemma lm:suboptimality), cost
//            terms sum w r^2, sum w Xt Z, b^T y (eq. reduced-ALM-subproblem);
//            out = G Y.
//      MULT: Xt <- Xt + sigma (Z - y) in place (Algorithm alg1 step 6),
//            out = (Xt + D) Y for z = diag((Xt + D) S) (step 7).
//      XMV : out = (Xt + D) V (certificate matvec without -Diag(z)).
//      HVP : a = coefficient of U, b = coefficient of Y per entry, out = A U + B Y
//            (the entry-wise part of 2 G U + 2 sigma Q(Y U^T + U Y^T) Y).
//      Each 16 x 16 coefficient block is written to LDS once and read back in
//      the two MFMA operand layouts, giving both the row-side product
//      (rows of the tile) and the column-side product (columns) of the packed
//      symmetric matrix from one read of the entry data.  Row-side results go
//      to one partial per tile, column-side results are accumulated in
//      registers over a segment of tiles of one column block; k_row* kernels
//      add the partials in a fixed order.
//
// Workgroup -> segment mapping is XCD-aware: consecutive segments (same
// column block, hence overlapping class ids and Y rows) land on one XCD.

#include <math.h>

#include "mdsdp_internal.hpp"

namespace mdsdp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct V4;
template <>
struct V4<double> {
  typedef v4d type;
};
template <>
struct V4<float> {
  typedef v4f type;
};

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct KArgs {
  const uint32_t* cls;
  double* Xt;
  float* Xt32;
  const double* Ct;
  const Seg* segs;
  int nseg, seg_per_xcd, nb;
  int nk;  // number of 4-wide K chunks covering p
  const void* Yp;
  const void* Up;
  const double2* cinf;  // {D, 1/|gamma|}
  const double* Cavg;   // A(C)/|gamma| or null
  long long* sS_acc;    // S-sum buffer being accumulated
  long long* sS_clr;    // S-sum buffer to clear
  const long long* sS;  // S-sums to read (residual passes)
  long long* sZ_acc;
  long long* sZ_clr;
  const long long* sZ;
  const unsigned long long* bound;  // [ymax, umax] bit patterns
  double* scal;
  double kmax;
  double sigma;
  void* rowpart;
  void* colpart;
  double* wgpart;
};

constexpr int NWP = 4;  // scalar partials per workgroup

__device__ __forceinline__ double fx_scale(double kmax, double bnd) {
  // largest power of two 2^F with kmax * bnd * 2^F <= 2^61
  double lim = kmax * bnd;
  if (!(lim > 0.0)) return 1.0;
  int e;
  (void)frexp(lim, &e);
  return ldexp(1.0, 61 - e);
}

__device__ __forceinline__ double bound_val(const unsigned long long* b, int i) {
  return __longlong_as_double((long long)b[i]);
}

__device__ __forceinline__ int seg_of_block(int b, int per, int nseg) {
  int s = (b & 7) * per + (b >> 3);
  return s < nseg ? s : -1;
}

template <typename T>
__device__ __forceinline__ void load_rows(T* sdst, const T* src, int row0, int tid) {
  // 64 rows x 16 cols, padded source (npad x 16), LDS pitch LP
  for (int i = tid; i < 64 * 16; i += 256) {
    int r = i >> 4, c = i & 15;
    sdst[r * LP + c] = src[(size_t)(row0 + r) * 16 + c];
  }
}

// ---------------------------------------------------------------------------
// staging: FP64 n x p (ld = p) -> padded npad x 16 in T; max row norms
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_stage(int n, int p, int npad, const double* __restrict__ Y,
                                               const double* __restrict__ U, T* __restrict__ Yp,
                                               T* __restrict__ Up, unsigned long long* bound) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int r = idx >> 4, c = idx & 15;
  bool in = idx < npad * 16;
  double y = (in && r < n && c < p) ? Y[(size_t)r * p + c] : 0.0;
  double u = (U && in && r < n && c < p) ? U[(size_t)r * p + c] : 0.0;
  if (in) {
    Yp[idx] = (T)y;
    if (U) Up[idx] = (T)u;
  }
  double ny = y * y, nu = u * u;
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) {
    ny += __shfl_xor(ny, off, 16);
    nu += __shfl_xor(nu, off, 16);
  }
  if (in && c == 0 && r < n) {
    atomicMax(&bound[0], (unsigned long long)__double_as_longlong(sqrt(ny)));
    if (U) atomicMax(&bound[1], (unsigned long long)__double_as_longlong(sqrt(nu)));
  }
}

// ---------------------------------------------------------------------------
// class sums
// ---------------------------------------------------------------------------
template <typename T, bool ZMODE>
__global__ __launch_bounds__(256) void k_classsum(KArgs a) {
  typedef typename V4<T>::type v4;
  const int sidx = seg_of_block(blockIdx.x, a.seg_per_xcd, a.nseg);
  if (sidx < 0) return;
  const Seg sg = a.segs[sidx];
  __shared__ T sYc[64 * LP], sYr[64 * LP];
  __shared__ T sUc[ZMODE ? 64 * LP : 1], sUr[ZMODE ? 64 * LP : 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const T* Yp = (const T*)a.Yp;
  const T* Up = (const T*)a.Up;
  load_rows(sYc, Yp, sg.J * 64, tid);
  if (ZMODE) load_rows(sUc, Up, sg.J * 64, tid);
  const double ymax = bound_val(a.bound, 0);
  const double scale = ZMODE ? fx_scale(a.kmax, 2.0 * ymax * bound_val(a.bound, 1))
                             : fx_scale(a.kmax, ymax * ymax);
  if (sidx == 0 && tid == 0) a.scal[ZMODE ? 8 : 7] = scale;
  long long* acc_t = ZMODE ? a.sZ_acc : a.sS_acc;
  long long* clr_t = ZMODE ? a.sZ_clr : a.sS_clr;
  const int li = lane & 15, lk = lane >> 4;
  for (int I = sg.I0; I <= sg.I1; ++I) {
    __syncthreads();
    load_rows(sYr, Yp, I * 64, tid);
    if (ZMODE) load_rows(sUr, Up, I * 64, tid);
    __syncthreads();
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    const double wgt = (I == sg.J) ? 1.0 : 2.0;
    for (int sc = 0; sc < 4; ++sc) {
      v4 acc = {0, 0, 0, 0};
      for (int j = 0; j < a.nk; ++j) {
        const int k = 4 * j + lk;
        T ya = sYr[(w * 16 + li) * LP + k];
        T yb = sYc[(sc * 16 + li) * LP + k];
        if (ZMODE) {
          T ub = sUc[(sc * 16 + li) * LP + k];
          T ua = sUr[(w * 16 + li) * LP + k];
          acc = mfma(ya, ub, acc);
          acc = mfma(ua, yb, acc);
        } else {
          acc = mfma(ya, yb, acc);
        }
      }
      const uint32_t* cb = a.cls + t * TSLOTS + (w * 4 + sc) * 256 + lk * 64 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t cw = cb[v * 16];
        if (!(cw & 0x80000000u)) {
          uint32_t id = cw & CLS_MASK;
          long long qv = llrint(wgt * (double)acc[v] * scale);
          atomicAdd((unsigned long long*)&acc_t[id], (unsigned long long)qv);
          if (cw & OWNER_BIT) clr_t[id] = 0;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// residual / product pass
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_resid(KArgs a) {
  typedef typename V4<T>::type v4;
  constexpr bool HAS_S = (MODE == M_GRAD || MODE == M_MULT || (MODE == M_HVP && sizeof(T) == 4));
  constexpr bool HAS_B = (MODE == M_HVP);
  constexpr bool SEPARATE_U = (MODE == M_HVP || MODE == M_XMV);
  constexpr bool NEED_Y = (MODE != M_XMV);
  const int sidx = seg_of_block(blockIdx.x, a.seg_per_xcd, a.nseg);
  if (sidx < 0) return;
  const Seg sg = a.segs[sidx];
  __shared__ T sYc[NEED_Y ? 64 * LP : 1], sYr[NEED_Y ? 64 * LP : 1];
  __shared__ T sUc[SEPARATE_U ? 64 * LP : 1], sUr[SEPARATE_U ? 64 * LP : 1];
  __shared__ T tA[4][16 * LP];
  __shared__ T tB[HAS_B ? 4 : 1][HAS_B ? 16 * LP : 1];
  __shared__ double red[256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const T* Yp = (const T*)a.Yp;
  const T* Up = (const T*)a.Up;
  const T* cY = sYc;
  const T* rY = sYr;
  const T* cU = SEPARATE_U ? sUc : sYc;
  const T* rU = SEPARATE_U ? sUr : sYr;
  if (NEED_Y) load_rows(sYc, Yp, sg.J * 64, tid);
  if (SEPARATE_U) load_rows(sUc, Up, sg.J * 64, tid);

  const double sigma = a.sigma;
  double inv_sS = 1.0, inv_sZ = 1.0;
  if (MODE == M_GRAD || MODE == M_MULT || MODE == M_HVP) {
    const double ymax = bound_val(a.bound, 0);
    inv_sS = 1.0 / fx_scale(a.kmax, ymax * ymax);
    if (MODE == M_HVP) inv_sZ = 1.0 / fx_scale(a.kmax, 2.0 * ymax * bound_val(a.bound, 1));
  }
  if (MODE == M_HVP) {
    // the S-sums were taken at the cost/grad point with the same Y
    inv_sS = 1.0 / a.scal[7];
  }
  v4 accC[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) accC[i] = v4{0, 0, 0, 0};
  double p_r2 = 0.0, p_xz = 0.0, p_bty = 0.0, p_cx = 0.0;
  T* tAw = tA[w];
  T* tBw = HAS_B ? tB[w] : tA[w];

  for (int I = sg.I0; I <= sg.I1; ++I) {
    __syncthreads();
    if (NEED_Y) load_rows(sYr, Yp, I * 64, tid);
    if (SEPARATE_U) load_rows(sUr, Up, I * 64, tid);
    __syncthreads();
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    const bool diag = (I == sg.J);
    const double wgt = diag ? 1.0 : 2.0;
    v4 accR = {0, 0, 0, 0};
    for (int sc = 0; sc < 4; ++sc) {
      v4 Sb = {0, 0, 0, 0};
      if (HAS_S) {
        for (int j = 0; j < a.nk; ++j) {
          const int k = 4 * j + lk;
          Sb = mfma(rY[(w * 16 + li) * LP + k], cY[(sc * 16 + li) * LP + k], Sb);
        }
      }
      const size_t base = (size_t)t * TSLOTS + (w * 4 + sc) * 256 + lk * 64 + li;
      // D layout: element v <-> (row 4*lk + v, col li) of the sub-block
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t off = base + v * 16;
        const uint32_t cw = a.cls[off];
        const bool valid = !(cw & 0x80000000u);
        const uint32_t id = valid ? (cw & CLS_MASK) : 0u;
        T av = 0, bv = 0;
        if (valid) {
          const double2 ci = a.cinf[id];
          const double Ce = a.Ct ? a.Ct[off] : 0.0;
          if (MODE == M_GRAD || MODE == M_MULT) {
            double y = (double)a.sS[id] * inv_sS * ci.y;
            if (a.Cavg) y += a.Cavg[id];
            const double Zv = (double)Sb[v] + Ce;
            const double r = Zv - y;
            const double x = a.Xt[off];
            p_r2 += wgt * r * r;
            if (MODE == M_GRAD) {
              p_xz += wgt * x * Zv;
              av = (T)(x + ci.x + sigma * r);
            } else {
              const double xn = x + sigma * r;
              a.Xt[off] = xn;
              a.Xt32[off] = (float)xn;
              p_cx += wgt * Ce * (xn + ci.x);
              av = (T)(xn + ci.x);
            }
            if (cw & OWNER_BIT) p_bty += ci.x / ci.y * y;
          } else if (MODE == M_XMV) {
            av = (T)(a.Xt[off] + ci.x);
          } else {  // HVP
            double y = (double)a.sS[id] * inv_sS * ci.y;
            if (a.Cavg) y += a.Cavg[id];
            const double yz = (double)a.sZ[id] * inv_sZ * ci.y;
            bv = (T)(-sigma * yz);
            if (sizeof(T) == 8) {
              av = (T)(a.Xt[off] + (ci.x - sigma * y) + sigma * Ce);
            } else {
              const float rS = (float)Sb[v] + (float)(Ce - y);
              av = (T)(a.Xt32[off] + (float)ci.x + (float)sigma * rS);
            }
          }
        }
        tAw[(4 * lk + v) * LP + li] = av;
        if (HAS_B) tBw[(4 * lk + v) * LP + li] = bv;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // row side: out_R[row][pcol] += sum_c A[row][c] U_C[c][pcol] (+ B Y_C)
      // column side: out_C^T[pcol][c] += sum_r U_R[r][pcol] A[r][c] (+ Y_R B)
      for (int j = 0; j < 4; ++j) {
        const T a1 = tAw[li * LP + 4 * j + lk];
        const T a2 = tAw[(4 * j + lk) * LP + li];
        const T uc = cU[(sc * 16 + 4 * j + lk) * LP + li];
        const T ur = rU[(w * 16 + 4 * j + lk) * LP + li];
        accR = mfma(a1, uc, accR);
        if (!diag) accC[sc] = mfma(ur, a2, accC[sc]);
        if (HAS_B) {
          const T b1 = tBw[li * LP + 4 * j + lk];
          const T b2 = tBw[(4 * j + lk) * LP + li];
          const T yc = cY[(sc * 16 + 4 * j + lk) * LP + li];
          const T yr = rY[(w * 16 + 4 * j + lk) * LP + li];
          accR = mfma(b1, yc, accR);
          if (!diag) accC[sc] = mfma(yr, b2, accC[sc]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // row-side partial of this tile: rows w*16 + 4*lk + v, pcol li
    T* rp = (T*)a.rowpart + ((size_t)t * 64 + w * 16 + 4 * lk) * 16 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) rp[v * 16] = accR[v];
  }
  // column-side partial of the segment: sum the four waves (rows sub-blocks)
  __syncthreads();
  T* cred = &tA[0][0];  // reuse: need 4 waves x 4 sc x 256 values -> do sc by sc
  T* cp = (T*)a.colpart + (size_t)sidx * 64 * 16;
  for (int sc = 0; sc < 4; ++sc) {
    // accC[sc]: lane (lk, li), v -> pcol 4*lk + v, col li
    __syncthreads();
    if (w > 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) cred[(w - 1) * 256 + (4 * lk + v) * 16 + li] = accC[sc][v];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pc = 4 * lk + v;
        T s = accC[sc][v];
        s += cred[0 * 256 + pc * 16 + li];
        s += cred[1 * 256 + pc * 16 + li];
        s += cred[2 * 256 + pc * 16 + li];
        cp[(sc * 16 + li) * 16 + pc] = s;
      }
    }
  }
  if (MODE == M_GRAD || MODE == M_MULT) {
    double vals[NWP] = {p_r2, p_xz, p_bty, p_cx};
    for (int q = 0; q < NWP; ++q) {
      __syncthreads();
      red[tid] = vals[q];
      __syncthreads();
      for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
      }
      if (tid == 0) a.wgpart[(size_t)sidx * NWP + q] = red[0];
    }
  }
}

// ---------------------------------------------------------------------------
// row finalisers: thread per (row, pcol); 16 lanes per row
// ---------------------------------------------------------------------------
struct RowArgs {
  int n, p, nb, nseg;
  const int* seg_start;  // nb + 1
  const void* rowpart;
  const void* colpart;
};

template <typename T>
__device__ __forceinline__ double row_sum(const RowArgs& ra, int r, int k) {
  const int I = r >> 6, rr = r & 63;
  const T* rp = (const T*)ra.rowpart;
  const T* cp = (const T*)ra.colpart;
  double s = 0.0;
  for (int J = I; J < ra.nb; ++J) {
    const long long t = (long long)J * (J + 1) / 2 + I;
    s += (double)rp[((size_t)t * 64 + rr) * 16 + k];
  }
  for (int q = ra.seg_start[I]; q < ra.seg_start[I + 1]; ++q) s += (double)cp[((size_t)q * 64 + rr) * 16 + k];
  return s;
}

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 16);
  return v;
}

__global__ __launch_bounds__(256) void k_row_grad(RowArgs ra, const double* __restrict__ Y,
                                                  double* __restrict__ egrad, double* __restrict__ rgrad,
                                                  double* __restrict__ zvec) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx >> 4, k = idx & 15;
  const bool in = r < ra.n;
  const bool kin = in && k < ra.p;
  double gy = in ? row_sum<double>(ra, r, k) : 0.0;
  double y = kin ? Y[(size_t)r * ra.p + k] : 0.0;
  if (!kin) gy = 0.0;
  const double z = sum16(gy * y);
  if (in && k == 0) zvec[r] = z;
  if (kin) {
    if (egrad) egrad[(size_t)r * ra.p + k] = 2.0 * gy;
    if (rgrad) rgrad[(size_t)r * ra.p + k] = 2.0 * (gy - z * y);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_row_hvp(RowArgs ra, const double* __restrict__ Y,
                                                 const double* __restrict__ U, const double* __restrict__ gram,
                                                 const double* __restrict__ zvec, double sigma, int fp32, int riem,
                                                 double* __restrict__ HU) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx >> 4, k = idx & 15;
  const bool in = r < ra.n;
  const bool kin = in && k < ra.p;
  double h = in ? row_sum<T>(ra, r, k) : 0.0;
  // low-rank terms: sigma [Y (Y^T U + U^T Y) + U (Y^T Y)] (FP64 tiles) or
  // sigma [Y (U^T Y) + U (Y^T Y)] (FP32 tiles carry S U entry-wise)
  const double* YtY = gram;
  const double* YtU = gram + 256;
  double lr = 0.0;
  if (in) {
    for (int i = 0; i < ra.p; ++i) {
      const double yi = Y[(size_t)r * ra.p + i];
      const double ui = U[(size_t)r * ra.p + i];
      double w1 = YtU[k * 16 + i];
      if (!fp32) w1 += YtU[i * 16 + k];
      lr += yi * w1 + ui * YtY[i * 16 + k];
    }
  }
  double Ht = kin ? 2.0 * (h + sigma * lr) : 0.0;
  const double y = kin ? Y[(size_t)r * ra.p + k] : 0.0;
  const double u = kin ? U[(size_t)r * ra.p + k] : 0.0;
  if (riem) {
    const double d = sum16(Ht * y);
    Ht = Ht - d * y - 2.0 * (in ? zvec[r] : 0.0) * u;
  }
  if (kin) HU[(size_t)r * ra.p + k] = Ht;
}

__global__ __launch_bounds__(256) void k_row_mult(RowArgs ra, const double* __restrict__ Y,
                                                  double* __restrict__ zmult, double* __restrict__ zout,
                                                  double* __restrict__ zpart) {
  __shared__ double red[256];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx >> 4, k = idx & 15;
  const bool in = r < ra.n;
  const bool kin = in && k < ra.p;
  double o = kin ? row_sum<double>(ra, r, k) : 0.0;
  const double y = kin ? Y[(size_t)r * ra.p + k] : 0.0;
  const double z = sum16(o * y);
  if (in && k == 0) {
    zmult[r] = z;
    if (zout) zout[r] = z;
  }
  red[threadIdx.x] = (in && k == 0) ? z : 0.0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) zpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_row_xmv(RowArgs ra, const double* __restrict__ V,
                                                 const double* __restrict__ zmult, double* __restrict__ XV) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx >> 4, k = idx & 15;
  if (r >= ra.n || k >= ra.p) return;
  const double o = row_sum<double>(ra, r, k);
  XV[(size_t)r * ra.p + k] = o - zmult[r] * V[(size_t)r * ra.p + k];
}

// scalar reduction (single block, fixed order)
__global__ __launch_bounds__(256) void k_scalars(int mode, const double* __restrict__ wgpart, int nseg,
                                                 const double* __restrict__ zpart, int nz, double sigma,
                                                 double* scal, double* f_out, double* kkt_out) {
  __shared__ double red[256];
  double acc[NWP + 1];
  for (int q = 0; q < NWP; ++q) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nseg; i += 256) s += wgpart[(size_t)i * NWP + q];
    acc[q] = s;
  }
  double sz = 0.0;
  if (zpart)
    for (int i = threadIdx.x; i < nz; i += 256) sz += zpart[i];
  acc[NWP] = sz;
  double tot[NWP + 1];
  for (int q = 0; q <= NWP; ++q) {
    __syncthreads();
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    tot[q] = red[0];
  }
  if (threadIdx.x == 0) {
    const double r2 = tot[0], xz = tot[1], bty = tot[2], cx = tot[3];
    scal[SC_R2] = r2;
    scal[SC_XZ] = xz;
    scal[SC_BTY] = bty;
    if (mode == M_GRAD) {
      const double f = bty + xz + 0.5 * sigma * r2;
      scal[SC_F] = f;
      if (!isfinite(f)) scal[SC_NONFIN] = 1.0;
      if (f_out) *f_out = f;
    } else {
      scal[SC_SUMZ] = tot[NWP];
      scal[SC_CXZ] = cx;
      if (kkt_out) {
        kkt_out[0] = sqrt(r2);
        kkt_out[1] = bty;
        kkt_out[2] = tot[NWP];
        kkt_out[3] = cx;
      }
      if (!isfinite(r2) || !isfinite(tot[NWP])) scal[SC_NONFIN] = 1.0;
    }
  }
}

// Gram matrices Y^T Y and Y^T U (16 x 16, FP64), two-stage fixed order.
__global__ __launch_bounds__(256) void k_gram_part(int n, int p, const double* __restrict__ Y,
                                                   const double* __restrict__ U, double* __restrict__ part) {
  const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
  const int r0 = blockIdx.x * 64;
  double syy = 0.0, syu = 0.0;
  if (i < p && j < p) {
    for (int r = r0; r < min(n, r0 + 64); ++r) {
      const double yi = Y[(size_t)r * p + i];
      syy += yi * Y[(size_t)r * p + j];
      syu += yi * U[(size_t)r * p + j];
    }
  }
  part[(size_t)blockIdx.x * 512 + threadIdx.x] = syy;
  part[(size_t)blockIdx.x * 512 + 256 + threadIdx.x] = syu;
}

__global__ __launch_bounds__(512) void k_gram_final(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ gram) {
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * 512 + threadIdx.x];
  gram[threadIdx.x] = s;
}

// retraction and tangent projection: one thread per row, any p
__global__ __launch_bounds__(256) void k_retract(int n, int p, const double* __restrict__ Y,
                                                 const double* __restrict__ V, double t, double* Yout) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double nrm = 0.0;
  for (int k = 0; k < p; ++k) {
    const double v = Y[(size_t)r * p + k] + t * V[(size_t)r * p + k];
    nrm += v * v;
  }
  const double inv = 1.0 / sqrt(nrm);
  for (int k = 0; k < p; ++k) {
    const double v = Y[(size_t)r * p + k] + t * V[(size_t)r * p + k];
    Yout[(size_t)r * p + k] = v * inv;
  }
}

__global__ __launch_bounds__(256) void k_project(int n, int p, const double* __restrict__ Y,
                                                 const double* U, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double d = 0.0;
  for (int k = 0; k < p; ++k) d += U[(size_t)r * p + k] * Y[(size_t)r * p + k];
  for (int k = 0; k < p; ++k) out[(size_t)r * p + k] = U[(size_t)r * p + k] - d * Y[(size_t)r * p + k];
}

// y export: y_gamma = S-sum / scale / |gamma| (+ A(C)/|gamma|)
__global__ __launch_bounds__(256) void k_y_export(long long m, const long long* __restrict__ sS,
                                                  const double2* __restrict__ cinf, const double* __restrict__ Cavg,
                                                  const double* __restrict__ scal, double* __restrict__ y) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  double v = (double)sS[g] / scal[7] * cinf[g].y;
  if (Cavg) v += Cavg[g];
  y[g] = v;
}

// dense <-> tile layout for Xt
__global__ __launch_bounds__(256) void k_set_dense(int n, int nb, long long nslots, const double* __restrict__ X,
                                                   double* __restrict__ Xt, float* __restrict__ Xt32) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const long long t = s / TSLOTS;
  const int in = (int)(s % TSLOTS);
  // invert t = J(J+1)/2 + I
  int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((long long)(J + 1) * (J + 2) / 2 <= t) ++J;
  while ((long long)J * (J + 1) / 2 > t) --J;
  const int I = (int)(t - (long long)J * (J + 1) / 2);
  const int sb = in >> 8, e = in & 255;
  const int r = I * 64 + (sb >> 2) * 16 + (e >> 4);
  const int c = J * 64 + (sb & 3) * 16 + (e & 15);
  double v = 0.0;
  if (r < n && c < n) v = X ? X[(size_t)r * n + c] : 0.0;
  Xt[s] = v;
  Xt32[s] = (float)v;
}

__global__ __launch_bounds__(256) void k_get_dense(int n, int nb, long long nslots, const double* __restrict__ Xt,
                                                   const uint32_t* __restrict__ cls, const double2* __restrict__ cinf,
                                                   int add_D, double* __restrict__ X) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const long long t = s / TSLOTS;
  const int in = (int)(s % TSLOTS);
  int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((long long)(J + 1) * (J + 2) / 2 <= t) ++J;
  while ((long long)J * (J + 1) / 2 > t) --J;
  const int I = (int)(t - (long long)J * (J + 1) / 2);
  const int sb = in >> 8, e = in & 255;
  const int r = I * 64 + (sb >> 2) * 16 + (e >> 4);
  const int c = J * 64 + (sb & 3) * 16 + (e & 15);
  if (r >= n || c >= n) return;
  double v = Xt[s];
  if (add_D) v += cinf[cls[s] & CLS_MASK].x;
  X[(size_t)r * n + c] = v;
  X[(size_t)c * n + r] = v;
}

// vector helpers for the solver (deterministic two-stage dot products)
__global__ __launch_bounds__(256) void k_dots(const double* const* __restrict__ a, const double* const* __restrict__ b,
                                              int npairs, long long len, double* __restrict__ part) {
  __shared__ double red[256];
  for (int q = 0; q < npairs; ++q) {
    double s = 0.0;
    const double* x = a[q];
    const double* y = b[q];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < len; i += (long long)gridDim.x * 256)
      s += x[i] * y[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_dots_final(int npairs, int nblk, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q >= npairs) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)q * nblk + b];
  out[q] = s;
}

__global__ __launch_bounds__(256) void k_lincomb(long long len, double alpha, const double* __restrict__ x,
                                                 double beta, const double* y, double* out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  double v = alpha * x[i];
  if (y) v += beta * y[i];
  out[i] = v;
}

__global__ __launch_bounds__(256) void k_fill(long long len, double v, double* out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < len) out[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long count, int per) { return (unsigned)((count + per - 1) / per); }

static KArgs make_args(mdsdp_problem P) {
  KArgs a{};
  a.cls = P->cls;
  a.Xt = P->Xt;
  a.Xt32 = P->Xt32;
  a.Ct = P->Ct;
  a.segs = P->segs;
  a.nseg = P->nseg;
  a.seg_per_xcd = (P->nseg + 7) / 8;
  a.nb = P->nb;
  a.nk = (P->last_p + 3) / 4;
  a.Yp = P->Yp;
  a.Up = P->Up;
  a.cinf = P->cinf;
  a.Cavg = P->Cavg;
  a.bound = P->bound;
  a.scal = P->scal;
  a.kmax = (double)P->kmax;
  a.sigma = P->sigma;
  a.rowpart = P->rowpart;
  a.colpart = P->colpart;
  a.wgpart = P->wgpart;
  return a;
}

static unsigned seg_grid(mdsdp_problem P) { return (unsigned)(8 * ((P->nseg + 7) / 8)); }

void timer_begin(mdsdp_problem P, hipStream_t s, const char* name) {
  if (!P->timer.on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, s);
  P->timer.ev.push_back(e);
  P->timer.names.push_back(name);
}
void timer_end(mdsdp_problem P, hipStream_t s) {
  if (!P->timer.on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, s);
  P->timer.ev.push_back(e);
  P->timer.names.push_back("");
}

mdsdp_status launch_stage(mdsdp_problem P, int p, const double* Y, const double* U, bool fp32,
                          hipStream_t s) {
  P->last_p = p;
  MDSDP_HIP(hipMemsetAsync(P->bound, 0, 2 * sizeof(unsigned long long), s));
  const long long cnt = (long long)P->npad * 16;
  if (fp32)
    k_stage<float><<<blocks_for(cnt, 256), 256, 0, s>>>(P->n, p, P->npad, Y, U, (float*)P->Yp, (float*)P->Up,
                                                         P->bound);
  else
    k_stage<double><<<blocks_for(cnt, 256), 256, 0, s>>>(P->n, p, P->npad, Y, U, (double*)P->Yp,
                                                          (double*)P->Up, P->bound);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_classsum_S(mdsdp_problem P, hipStream_t s) {
  KArgs a = make_args(P);
  P->spar ^= 1;
  const int par = P->spar;
  a.sS_acc = P->sS[par];
  a.sS_clr = P->sS[par ^ 1];
  timer_begin(P, s, "classsum_S");
  k_classsum<double, false><<<seg_grid(P), 256, 0, s>>>(a);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_classsum_Z(mdsdp_problem P, bool fp32, hipStream_t s) {
  KArgs a = make_args(P);
  P->zpar ^= 1;
  const int par = P->zpar;
  a.sZ_acc = P->sZ[par];
  a.sZ_clr = P->sZ[par ^ 1];
  timer_begin(P, s, fp32 ? "classsum_Z32" : "classsum_Z64");
  if (fp32)
    k_classsum<float, true><<<seg_grid(P), 256, 0, s>>>(a);
  else
    k_classsum<double, true><<<seg_grid(P), 256, 0, s>>>(a);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_resid(mdsdp_problem P, int mode, bool fp32, hipStream_t s) {
  KArgs a = make_args(P);
  a.sS = P->sS[P->spar];
  a.sZ = P->sZ[P->zpar];
  const unsigned g = seg_grid(P);
  switch (mode) {
    case M_GRAD:
      timer_begin(P, s, "resid_grad");
      k_resid<double, M_GRAD><<<g, 256, 0, s>>>(a);
      break;
    case M_MULT:
      timer_begin(P, s, "resid_mult");
      k_resid<double, M_MULT><<<g, 256, 0, s>>>(a);
      break;
    case M_XMV:
      timer_begin(P, s, "resid_xmv");
      k_resid<double, M_XMV><<<g, 256, 0, s>>>(a);
      break;
    default:
      if (fp32) {
        timer_begin(P, s, "resid_hvp32");
        k_resid<float, M_HVP><<<g, 256, 0, s>>>(a);
      } else {
        timer_begin(P, s, "resid_hvp64");
        k_resid<double, M_HVP><<<g, 256, 0, s>>>(a);
      }
  }
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

static RowArgs row_args(mdsdp_problem P, int p) {
  RowArgs ra;
  ra.n = P->n;
  ra.p = p;
  ra.nb = P->nb;
  ra.nseg = P->nseg;
  ra.seg_start = P->seg_start;
  ra.rowpart = P->rowpart;
  ra.colpart = P->colpart;
  return ra;
}

mdsdp_status launch_gram(mdsdp_problem P, int p, const double* Y, const double* U, hipStream_t s) {
  const int nblk = (P->n + 63) / 64;
  k_gram_part<<<nblk, 256, 0, s>>>(P->n, p, Y, U, P->gpart);
  k_gram_final<<<1, 512, 0, s>>>(nblk, P->gpart, P->gram);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_grad(mdsdp_problem P, int p, const double* Y, double* egrad, double* rgrad,
                                  double* f, hipStream_t s) {
  RowArgs ra = row_args(P, p);
  timer_begin(P, s, "row_grad");
  k_row_grad<<<blocks_for((long long)P->n * 16, 256), 256, 0, s>>>(ra, Y, egrad, rgrad, P->zvec);
  k_scalars<<<1, 256, 0, s>>>(M_GRAD, P->wgpart, P->nseg, nullptr, 0, P->sigma, P->scal, f, nullptr);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_hvp(mdsdp_problem P, int p, bool fp32, const double* Y, const double* U,
                                 double* HU, int riem, hipStream_t s) {
  RowArgs ra = row_args(P, p);
  timer_begin(P, s, "row_hvp");
  if (fp32)
    k_row_hvp<float><<<blocks_for((long long)P->n * 16, 256), 256, 0, s>>>(ra, Y, U, P->gram, P->zvec, P->sigma,
                                                                            1, riem, HU);
  else
    k_row_hvp<double><<<blocks_for((long long)P->n * 16, 256), 256, 0, s>>>(ra, Y, U, P->gram, P->zvec,
                                                                             P->sigma, 0, riem, HU);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_mult(mdsdp_problem P, int p, const double* Y, double* z, double* kkt,
                                  hipStream_t s) {
  RowArgs ra = row_args(P, p);
  const unsigned nblk = blocks_for((long long)P->n * 16, 256);
  k_row_mult<<<nblk, 256, 0, s>>>(ra, Y, P->zmult, z, P->zpart);
  k_scalars<<<1, 256, 0, s>>>(M_MULT, P->wgpart, P->nseg, P->zpart, (int)nblk, P->sigma, P->scal, nullptr, kkt);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_xmv(mdsdp_problem P, int k, const double* V, double* XV, hipStream_t s) {
  RowArgs ra = row_args(P, k);
  k_row_xmv<<<blocks_for((long long)P->n * 16, 256), 256, 0, s>>>(ra, V, P->zmult, XV);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_retract(int n, int p, const double* Y, const double* V, double t, double* Yout,
                            hipStream_t s) {
  k_retract<<<blocks_for(n, 256), 256, 0, s>>>(n, p, Y, V, t, Yout);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_project(int n, int p, const double* Y, const double* U, double* out, hipStream_t s) {
  k_project<<<blocks_for(n, 256), 256, 0, s>>>(n, p, Y, U, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_y_export(mdsdp_problem P, double* y, hipStream_t s) {
  k_y_export<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->sS[P->spar], P->cinf, P->Cavg, P->scal, y);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_set_dense(mdsdp_problem P, const double* X, hipStream_t s) {
  k_set_dense<<<blocks_for(P->nslots, 256), 256, 0, s>>>(P->n, P->nb, P->nslots, X, P->Xt, P->Xt32);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_get_dense(mdsdp_problem P, double* X, bool add_D, hipStream_t s) {
  k_get_dense<<<blocks_for(P->nslots, 256), 256, 0, s>>>(P->n, P->nb, P->nslots, P->Xt, P->cls, P->cinf,
                                                         add_D ? 1 : 0, X);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_dots(const double* const* a, const double* const* b, int npairs, long long len, double* out_dev,
                      double* part, int nblk, hipStream_t s) {
  k_dots<<<nblk, 256, 0, s>>>(a, b, npairs, len, part);
  k_dots_final<<<1, 256, 0, s>>>(npairs, nblk, part, out_dev);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_lincomb(long long len, double alpha, const double* x, double beta, const double* y, double* out,
                         hipStream_t s) {
  k_lincomb<<<blocks_for(len, 256), 256, 0, s>>>(len, alpha, x, beta, y, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_fill(long long len, double v, double* out, hipStream_t s) {
  k_fill<<<blocks_for(len, 256), 256, 0, s>>>(len, v, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

}  // namespace mdsdp
