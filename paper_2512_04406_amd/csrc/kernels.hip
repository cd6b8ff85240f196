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
//      the sums are bit-reproducible whatever the scheduling); k_final_*
//      turns them into class averages and clears the accumulator.  This is
//      the path for any class map; BQP relaxations in colex order use the
//      structured kernels k_bqp_pass1 / k_bqp_pass2 / k_bqpFin instead (no class-map reads,
//      no atomics).
//
//  k_resid<T, MODE, SW>  per-entry coefficient and symmetric product pass
//      (FP64 tiles; slices of SW <= 64 factor columns):
//      GRAD: r = Z - y, G = Xt + D + sigma r (Lemma lm:suboptimality), cost
//            terms sum w r^2, sum w Xt Z, b^T y (eq. reduced-ALM-subproblem);
//            out = G Y.
//      MULT: Xt <- Xt + sigma (Z - y) in place (Algorithm alg1 step 6),
//            out = (Xt + D) Y for z = diag((Xt + D) S) (step 7).
//      XMV : out = (Xt + D) V (certificate matvec without -Diag(z)).
//      HVP : a = coefficient of U, b = coefficient of Y per entry, out = A U + B Y
//            (the entry-wise part of 2 G U + 2 sigma Q(Y U^T + U Y^T) Y); the
//            FP32-tile version of this mode is k_hvp32.
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

#include <algorithm>
#include <mutex>
#include <type_traits>


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

// Result layout of the 16x16x4 MFMA: lane l = 16 * lk + li holds column li;
// its element v is row lk + 4 v for the FP64 instruction and row 4 lk + v for
// the FP32 one (measured on gfx950).  The operand layouts are the same for
// both: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k.
template <typename T>
__device__ __forceinline__ int drow(int lk, int v) {
  return sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v;
}

struct KArgs {
  const uint32_t* cls;
  double* Xt;
  double* Xt_out;       // multiplier update target (Xt itself, or a second buffer when sliced)
  float* Xt32;
  const double* Ct;
  const Seg* segs;
  int nseg, seg_per_xcd, nb;
  int nk;  // number of 4-wide K chunks covering p
  int pw;  // row pitch of the staged factors (16, 32, 64 or a multiple of 64)
  int nsl; // column slices of width min(pw, 64)
  const void* Yp;
  const void* Up;
  const double2* cy;    // {D, y}
  const double2* ab64;  // FP64 HVP class coefficients {D - sigma y, -sigma y'}
  const double* Cavg;   // A(C)/|gamma| or null
  long long* sacc;      // generic fixed-point accumulator
  const unsigned long long* bound;  // [ymax, umax] bit patterns
  double* scal;
  double kmax;
  double sigma;
  void* rowpart;
  void* colpart;
  double* wgpart;
  int frozen;  // direct-DSDP (ADMM) subproblem: y is the stale y^k, and sum D Z is accumulated
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

// coefficient w_e of a slot in its A_gamma: +1, -1, or 0 (no class)
__device__ __forceinline__ double coef_of(uint32_t cw) {
  return (cw & FREE_BIT) ? 0.0 : ((cw & NEG_BIT) ? -1.0 : 1.0);
}

__device__ __forceinline__ int seg_of_block(int b, int per, int nseg) {
  int s = (b & 7) * per + (b >> 3);
  return s < nseg ? s : -1;
}

// 64 rows x W columns (from column col0) of a staged factor with row pitch SP
// into LDS (row pitch W + 1)
template <int W, int SP, typename T>
__device__ __forceinline__ void load_rows(T* sdst, const T* src, int row0, int col0, int tid) {
  for (int i = tid; i < 64 * W; i += 256) {
    const int r = i / W, c = i % W;
    sdst[r * (W + 1) + c] = src[(size_t)(row0 + r) * SP + col0 + c];
  }
}

// ---------------------------------------------------------------------------
// staging: FP64 n x p (ld = p) -> zero-padded npad x pw in T; max row norms
// (the latter only for the fixed-point class sums of generic class maps)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_stage(int n, int p, int npad, int pw, const double* __restrict__ Y,
                                               const double* __restrict__ U, T* __restrict__ Yp,
                                               T* __restrict__ Up, unsigned long long* bound) {
  // lanes per row L = min(pw, 64); each lane stages pw / L columns
  __shared__ double smax[2][256];
  const int L = pw < 64 ? pw : 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx / L, c0 = idx % L;
  const bool in = r < npad;
  double ny = 0.0, nu = 0.0;
  for (int c = c0; c < pw; c += L) {
    const double y = (in && r < n && c < p) ? Y[(size_t)r * p + c] : 0.0;
    const double u = (U && in && r < n && c < p) ? U[(size_t)r * p + c] : 0.0;
    if (in) {
      Yp[(size_t)r * pw + c] = (T)y;
      if (U) Up[(size_t)r * pw + c] = (T)u;
    }
    ny += y * y;
    nu += u * u;
  }
  if (!bound) return;
  for (int off = L >> 1; off >= 1; off >>= 1) {
    ny += __shfl_xor(ny, off, L);
    nu += __shfl_xor(nu, off, L);
  }
  smax[0][threadIdx.x] = (in && r < n) ? sqrt(ny) : 0.0;
  smax[1][threadIdx.x] = (in && r < n) ? sqrt(nu) : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m0 = 0.0, m1 = 0.0;
    for (int i = 0; i < 256; i += L) {
      m0 = fmax(m0, smax[0][i]);
      m1 = fmax(m1, smax[1][i]);
    }
    atomicMax(&bound[0], (unsigned long long)__double_as_longlong(m0));
    if (U) atomicMax(&bound[1], (unsigned long long)__double_as_longlong(m1));
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
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const T* Yp = (const T*)a.Yp;
  const T* Up = (const T*)a.Up;
  const int pw = a.pw;
  const double ymax = bound_val(a.bound, 0);
  const double scale = ZMODE ? fx_scale(a.kmax, 2.0 * ymax * bound_val(a.bound, 1))
                             : fx_scale(a.kmax, ymax * ymax);
  if (sidx == 0 && tid == 0) a.scal[ZMODE ? SC_SCALE_Z : SC_SCALE_S] = scale;
  long long* acc_t = a.sacc;
  const int li = lane & 15, lk = lane >> 4;
  const int nk = a.nk;
  for (int I = sg.I0; I <= sg.I1; ++I) {
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    const double wgt = (I == sg.J) ? 1.0 : 2.0;
    const size_t ra = (size_t)(I * 64 + w * 16 + li) * pw;
    for (int sc = 0; sc < 4; ++sc) {
      const size_t rb = (size_t)(sg.J * 64 + sc * 16 + li) * pw;
      v4 acc = {0, 0, 0, 0};
      for (int j = 0; j < nk; ++j) {
        const int k = 4 * j + lk;
        const T ya = Yp[ra + k], yb = Yp[rb + k];
        if (ZMODE) {
          acc = mfma(ya, Up[rb + k], acc);
          acc = mfma(Up[ra + k], yb, acc);
        } else {
          acc = mfma(ya, yb, acc);
        }
      }
      const uint32_t* cb = a.cls + t * TSLOTS + (w * 4 + sc) * 256 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t cw = cb[drow<T>(lk, v) * 16];
        if (!(cw & (0x80000000u | FREE_BIT))) {
          const uint32_t id = cw & CLS_MASK;
          const long long qv = llrint(coef_of(cw) * wgt * (double)acc[v] * scale);
          atomicAdd((unsigned long long*)&acc_t[id], (unsigned long long)qv);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// residual / product pass
// ---------------------------------------------------------------------------
// Factor columns are cut into slices of SW = min(pw, 64) columns
// (blockIdx.y); a workgroup forms the products of one slice.  The S tile needs
// the whole contraction over p: with one slice it comes from the staged slabs
// themselves, with several the rows are staged chunk by chunk (64 columns) and
// the S tile is accumulated before the slice is staged for the products.  With
// several slices the multiplier update writes a second buffer (Xt_out, slice 0
// only) while every slice reads the old Xt, and only slice 0 adds the cost
// and KKT partial sums.
template <typename T, int MODE, int SW>
struct ResidLds {
  static constexpr bool NEED_Y = (MODE != M_XMV);
  static constexpr bool SEPARATE_U = (MODE == M_HVP || MODE == M_XMV);
  static constexpr bool HAS_B = (MODE == M_HVP);
  static constexpr int LPW = SW + 1;
  static constexpr size_t slab = 64 * LPW;  // one 64-row slice
  static constexpr size_t nslab = (NEED_Y ? 2 : 0) + (SEPARATE_U ? 2 : 0);
  static constexpr size_t tbuf = 16 * LP;    // one 16 x 16 transpose buffer
  static constexpr size_t bytes = (nslab * slab + (HAS_B ? 8 : 4) * tbuf) * sizeof(T) + 256 * sizeof(double);
};

// 64 rows x SW columns (from column col0, row pitch pw) into LDS (row pitch SW + 1)
template <int SW, typename T>
__device__ __forceinline__ void load_slab(T* sdst, const T* src, int row0, int col0, int pw, int tid) {
  for (int i = tid; i < 64 * SW; i += 256) {
    const int r = i / SW, c = i % SW;
    sdst[r * (SW + 1) + c] = src[(size_t)(row0 + r) * pw + col0 + c];
  }
}

template <typename T, int MODE, int SW>
__global__ __launch_bounds__(256) void k_resid(KArgs a) {
  typedef typename V4<T>::type v4;
  typedef ResidLds<T, MODE, SW> L;
  constexpr bool HAS_S = (MODE == M_GRAD || MODE == M_MULT);
  constexpr bool HAS_B = L::HAS_B;
  constexpr bool SEPARATE_U = L::SEPARATE_U;
  constexpr bool NEED_Y = L::NEED_Y;
  constexpr int NC = SW / 16, LPW = L::LPW;
  const int pw = a.pw, nsl = a.nsl;
  const int col0 = (int)blockIdx.y * SW;
  const bool lead = blockIdx.y == 0;  // the slice that owns writes of entry data and scalar partials
  const bool chunked = HAS_S && nsl > 1;
  const int sidx = seg_of_block(blockIdx.x, a.seg_per_xcd, a.nseg);
  if (sidx < 0) return;
  const Seg sg = a.segs[sidx];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* red = (double*)smem_raw;
  T* sp = (T*)(smem_raw + 256 * sizeof(double));
  T* sYc = nullptr;
  T* sYr = nullptr;
  T* sUc = nullptr;
  T* sUr = nullptr;
  if (NEED_Y) {
    sYc = sp;
    sp += L::slab;
    sYr = sp;
    sp += L::slab;
  }
  if (SEPARATE_U) {
    sUc = sp;
    sp += L::slab;
    sUr = sp;
    sp += L::slab;
  }
  T* tA = sp;                               // 4 waves x (16 x LP)
  T* tB = HAS_B ? sp + 4 * L::tbuf : sp;    // 4 more for the B coefficients
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const T* Yp = (const T*)a.Yp;
  const T* Up = (const T*)a.Up;
  const T* cY = sYc;
  const T* rY = sYr;
  const T* cU = SEPARATE_U ? sUc : sYc;
  const T* rU = SEPARATE_U ? sUr : sYr;
  if (!chunked) {
    if (NEED_Y) load_slab<SW>(sYc, Yp, sg.J * 64, col0, pw, tid);
    if (SEPARATE_U) load_slab<SW>(sUc, Up, sg.J * 64, col0, pw, tid);
  }

  const double sigma = a.sigma;
  v4 accC[4][NC];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) accC[i][c] = v4{0, 0, 0, 0};
  double p_r2 = 0.0, p_xz = 0.0, p_cx = 0.0, p_dz = 0.0;
  T* tAw = tA + w * L::tbuf;
  T* tBw = tB + w * L::tbuf;

  for (int I = sg.I0; I <= sg.I1; ++I) {
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    const bool diag = (I == sg.J);
    const double wgt = diag ? 1.0 : 2.0;
    // ---- memory phase for this wave's 16 x 64 slab of the tile, in two
    // halves of two 16 x 16 sub-blocks each (half the registers of one batch
    // of sixteen entries per lane: more waves per SIMD hide the latency) ----
    typedef typename std::conditional<sizeof(T) == 8 || MODE != M_HVP, double, float>::type XT;
    const size_t tb = (size_t)t * TSLOTS + (size_t)(w * 4) * 256 + li;
    uint32_t cwv[2][4];
    XT xv[2][4];
    double2 dyv[2][4];  // {D, y}, or for the HVP {D - sigma y, -sigma y'}
    auto load_half = [&](int h) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t off = tb + (2 * h + s2) * 256 + drow<T>(lk, v) * 16;
          cwv[s2][v] = a.cls[off];
          if (sizeof(XT) == 8)
            xv[s2][v] = (XT)a.Xt[off];
          else
            xv[s2][v] = (XT)a.Xt32[slot32(off)];
        }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t cw = cwv[s2][v];
          const bool valid = !(cw & 0x80000000u);
          const uint32_t id = valid ? (cw & CLS_MASK) : 0u;
          dyv[s2][v] = (MODE == M_HVP) ? a.ab64[id] : a.cy[id];
        }
    };
    load_half(0);
    // S blocks of the four sub-blocks (MFMA from LDS, K = p)
    v4 Sbv[4];
#pragma unroll
    for (int sc = 0; sc < 4; ++sc) Sbv[sc] = v4{0, 0, 0, 0};
    if (HAS_S && chunked) {
      for (int kc = 0; kc < nsl; ++kc) {
        __syncthreads();
        load_slab<SW>(sYc, Yp, sg.J * 64, kc * SW, pw, tid);
        load_slab<SW>(sYr, Yp, I * 64, kc * SW, pw, tid);
        __syncthreads();
#pragma unroll
        for (int sc = 0; sc < 4; ++sc)
          for (int j = 0; j < SW / 4; ++j) {
            const int k = 4 * j + lk;
            Sbv[sc] = mfma(rY[(w * 16 + li) * LPW + k], cY[(sc * 16 + li) * LPW + k], Sbv[sc]);
          }
      }
      __syncthreads();
      load_slab<SW>(sYc, Yp, sg.J * 64, col0, pw, tid);
      load_slab<SW>(sYr, Yp, I * 64, col0, pw, tid);
      __syncthreads();
    } else {
      __syncthreads();
      if (NEED_Y) load_slab<SW>(sYr, Yp, I * 64, col0, pw, tid);
      if (SEPARATE_U) load_slab<SW>(sUr, Up, I * 64, col0, pw, tid);
      __syncthreads();
      if (HAS_S) {
        const int nk = min(SW / 4, a.nk);
#pragma unroll
        for (int sc = 0; sc < 4; ++sc)
          for (int j = 0; j < nk; ++j) {
            const int k = 4 * j + lk;
            Sbv[sc] = mfma(rY[(w * 16 + li) * LPW + k], cY[(sc * 16 + li) * LPW + k], Sbv[sc]);
          }
      }
    }
    v4 accR[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) accR[c] = v4{0, 0, 0, 0};
#pragma unroll
    for (int sc = 0; sc < 4; ++sc) {
      if (sc == 2) load_half(1);
      const int s2 = sc & 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rv = drow<T>(lk, v);
        const size_t off = tb + sc * 256 + rv * 16;
        const uint32_t cw = cwv[s2][v];
        const bool valid = !(cw & 0x80000000u);
        T av = 0, bv = 0;
        if (valid) {
          // class data times the slot's coefficient w_e: {w D, w y} (or the HVP pair)
          const double we = coef_of(cw);
          const double2 dy = make_double2(we * dyv[s2][v].x, we * dyv[s2][v].y);
          const double Ce = a.Ct ? a.Ct[off] : 0.0;
          if (MODE == M_GRAD || MODE == M_MULT) {
            const double Zv = (double)Sbv[sc][v] + Ce;
            const double r = Zv - dy.y;
            const double x = (double)xv[s2][v];
            p_r2 += wgt * r * r;
            if (MODE == M_GRAD) {
              p_xz += wgt * x * Zv;
              p_dz += wgt * dy.x * Zv;  // <D, Z> (the cost's first term when y is stale)
              av = (T)(x + dy.x + sigma * r);
            } else {
              const double xn = x + sigma * r;
              if (lead) {
                a.Xt_out[off] = xn;
                a.Xt32[slot32(off)] = (float)xn;
              }
              p_cx += wgt * Ce * (xn + dy.x);
              av = (T)(xn + dy.x);
            }
          } else if (MODE == M_XMV) {
            av = (T)((double)xv[s2][v] + dy.x);
          } else {  // HVP (FP64 tiles; the FP32-tile HVP is k_hvp32)
            bv = (T)dy.y;
            av = (T)((double)xv[s2][v] + dy.x + sigma * Ce);
          }
        }
        tAw[rv * LP + li] = av;
        if (HAS_B) tBw[rv * LP + li] = bv;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // row side: out_R[row][pcol] += sum_c A[row][c] U_C[c][pcol] (+ B Y_C)
      // column side: out_C^T[pcol][c] += sum_r U_R[r][pcol] A[r][c] (+ Y_R B)
      for (int j = 0; j < 4; ++j) {
        const T a1 = tAw[li * LP + 4 * j + lk];
        const T a2 = tAw[(4 * j + lk) * LP + li];
        T b1 = 0, b2 = 0;
        if (HAS_B) {
          b1 = tBw[li * LP + 4 * j + lk];
          b2 = tBw[(4 * j + lk) * LP + li];
        }
        const int rc = (sc * 16 + 4 * j + lk) * LPW + li;
        const int rr = (w * 16 + 4 * j + lk) * LPW + li;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          accR[c] = mfma(a1, cU[rc + 16 * c], accR[c]);
          if (!diag) accC[sc][c] = mfma(rU[rr + 16 * c], a2, accC[sc][c]);
          if (HAS_B) {
            accR[c] = mfma(b1, cY[rc + 16 * c], accR[c]);
            if (!diag) accC[sc][c] = mfma(rY[rr + 16 * c], b2, accC[sc][c]);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // row-side partial of this tile: rows w*16 + drow(lk, v), columns c*16 + li
    T* rp = (T*)a.rowpart + ((size_t)t * 64 + w * 16) * pw + col0 + li;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) rp[drow<T>(lk, v) * pw + 16 * c] = accR[c][v];
  }
  // column-side partial of the segment: sum the four waves (row sub-blocks)
  T* cred = tA;  // 3 x 256 values (the transpose buffers are free now)
  T* cp = (T*)a.colpart + (size_t)sidx * 64 * pw;
  for (int sc = 0; sc < 4; ++sc) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // accC[sc][c]: lane (lk, li), v -> pcol c*16 + drow(lk, v), col li
      __syncthreads();
      if (w > 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) cred[(w - 1) * 256 + drow<T>(lk, v) * 16 + li] = accC[sc][c][v];
      }
      __syncthreads();
      if (w == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pc = drow<T>(lk, v);
          T sum = accC[sc][c][v];
          sum += cred[0 * 256 + pc * 16 + li];
          sum += cred[1 * 256 + pc * 16 + li];
          sum += cred[2 * 256 + pc * 16 + li];
          cp[(sc * 16 + li) * pw + col0 + c * 16 + pc] = sum;
        }
      }
    }
  }
  if ((MODE == M_GRAD || MODE == M_MULT) && lead) {
    double vals[NWP] = {p_r2, p_xz, p_dz, p_cx};
    for (int qq = 0; qq < NWP; ++qq) {
      __syncthreads();
      red[tid] = vals[qq];
      __syncthreads();
      for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
      }
      if (tid == 0) a.wgpart[(size_t)sidx * NWP + qq] = red[0];
    }
  }
}

// ---------------------------------------------------------------------------
// FP32-tile HVP product pass (mixed precision).  Per packed entry e of class g
// the Euclidean HVP 2 G U + 2 sigma Q(Y U^T + U Y^T) Y needs the entry-wise
//     A_e = Xt_e + (D_g - sigma y_g) + sigma C_e   (coefficient of U)
//     B_e = -sigma y'_g                            (coefficient of Y)
// while sigma S U = sigma Y (Y^T U) and the rank-2p part sigma (Y U^T + U Y^T) Y
// are added in FP64 by the row finaliser from the Gram matrices, so no S tile
// is formed here.  Class data are one 8-byte gather of the FP32 pair
// {D_g - sigma y_g, -sigma y'_g}, entry data the class word and the FP32
// shadow of Xt: 8 bytes per packed entry and 8 per class.  The factor columns are cut into slices of SW <= 64 columns; the
// slices of one segment go to consecutive workgroups of one XCD so that they
// share the entry and class reads through that XCD's L2.
// ---------------------------------------------------------------------------
struct H32Args {
  const uint32_t* cls32;  // class words in FP32-tile order (slot32)
  const float* Xt32;
  const double* Ct;
  const Seg* segs;
  int nseg, seg_per_xcd, nsl, pw;
  const float* Yp;
  const float* Up;
  const float2* ab32;   // per class {D - sigma y, -sigma y'}
  float sigma;
  float* rowpart;
  float* colpart;
};

template <int SW>
struct H32Lds {
  static constexpr int LPW = SW + 1;
  static constexpr size_t slab = 64 * LPW;
  static constexpr size_t tbuf = 16 * LP;
  static constexpr size_t bytes = (4 * slab + 8 * tbuf) * sizeof(float);
};

template <int SW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SW == 16 ? 4 : 2))) void k_hvp32(H32Args a) {
  typedef H32Lds<SW> L;
  constexpr int NC = SW / 16, LPW = L::LPW;
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int sl = loc % a.nsl, sloc = loc / a.nsl;
  if (sloc >= a.seg_per_xcd) return;
  const int sidx = xcd * a.seg_per_xcd + sloc;
  if (sidx >= a.nseg) return;
  const int col0 = sl * SW, pw = a.pw;
  const Seg sg = a.segs[sidx];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* sYc = (float*)smem_raw;
  float* sUc = sYc + L::slab;
  float* sYr = sUc + L::slab;
  float* sUr = sYr + L::slab;
  float* tA = sUr + L::slab;
  float* tB = tA + 4 * L::tbuf;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int i = tid; i < 64 * SW; i += 256) {
    const int r = i / SW, c = i % SW;
    const size_t o = (size_t)(sg.J * 64 + r) * pw + col0 + c;
    sYc[r * LPW + c] = a.Yp[o];
    sUc[r * LPW + c] = a.Up[o];
  }
  const float sigma = a.sigma;
  v4f accC[4][NC];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) accC[i][c] = v4f{0, 0, 0, 0};
  float* tAw = tA + w * L::tbuf;
  float* tBw = tB + w * L::tbuf;

  // per tile: the entry words and the factor rows are loaded at the top of the
  // tile (loading those of the next tile during the products measured slower)
  constexpr bool PREF_ROWS = (SW == 16);
  constexpr int RPT = PREF_ROWS ? 64 * SW / 256 : 1;  // factor-row values per thread
  uint32_t cwv[4][4];
  float xv[4][4];
  float yrv[RPT], urv[RPT];
  auto load_tile = [&](int I) {
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    // FP32-tile order: this lane's four entries (rows 4 lk .. 4 lk + 3 of
    // column li in each sub-block) are one 16-byte vector
    const size_t tb32 = (size_t)t * TSLOTS + (size_t)(w * 4) * 256 + li * 16 + 4 * lk;
#pragma unroll
    for (int sc = 0; sc < 4; ++sc) {
      const uint4 cw4 = *(const uint4*)(a.cls32 + tb32 + sc * 256);
      const float4 x4 = *(const float4*)(a.Xt32 + tb32 + sc * 256);
      cwv[sc][0] = cw4.x;
      cwv[sc][1] = cw4.y;
      cwv[sc][2] = cw4.z;
      cwv[sc][3] = cw4.w;
      xv[sc][0] = x4.x;
      xv[sc][1] = x4.y;
      xv[sc][2] = x4.z;
      xv[sc][3] = x4.w;
    }
    if (PREF_ROWS) {
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int i = tid + 256 * e, r = i / SW, c = i % SW;
        const size_t o = (size_t)(I * 64 + r) * pw + col0 + c;
        yrv[e] = a.Yp[o];
        urv[e] = a.Up[o];
      }
    }
  };
  for (int I = sg.I0; I <= sg.I1; ++I) {
    load_tile(I);
    __syncthreads();
    if (PREF_ROWS) {
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int i = tid + 256 * e, r = i / SW, c = i % SW;
        sYr[r * LPW + c] = yrv[e];
        sUr[r * LPW + c] = urv[e];
      }
    } else {
      for (int i = tid; i < 64 * SW; i += 256) {
        const int r = i / SW, c = i % SW;
        const size_t o = (size_t)(I * 64 + r) * pw + col0 + c;
        sYr[r * LPW + c] = a.Yp[o];
        sUr[r * LPW + c] = a.Up[o];
      }
    }
    __syncthreads();
    const long long t = (long long)sg.J * (sg.J + 1) / 2 + I;
    const bool diag = (I == sg.J);
    v4f accR[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) accR[c] = v4f{0, 0, 0, 0};
    // entry data of this wave's 16 x 64 slab: lane (li, lk) holds column li,
    // rows 4 lk + v of each 16 x 16 sub-block (the FP32 MFMA result layout)
    const size_t tb = (size_t)t * TSLOTS + (size_t)(w * 4) * 256 + li;
    float av[4][4], bv[4][4];
#pragma unroll
    for (int sc = 0; sc < 4; ++sc)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t cw = cwv[sc][v];
        const bool valid = !(cw & 0x80000000u);
        const uint32_t id = valid ? (cw & CLS_MASK) : 0u;
        const float2 ab = a.ab32[id];
        const float we = (float)coef_of(cw);  // coefficient of the slot in A_gamma
        float A = xv[sc][v] + we * ab.x;
        if (a.Ct) A += sigma * (float)a.Ct[tb + sc * 256 + (4 * lk + v) * 16];
        av[sc][v] = valid ? A : 0.0f;
        bv[sc][v] = valid ? we * ab.y : 0.0f;
      }
#pragma unroll
    for (int sc = 0; sc < 4; ++sc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        tAw[(4 * lk + v) * LP + li] = av[sc][v];
        tBw[(4 * lk + v) * LP + li] = bv[sc][v];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // row side:    out_R[row][pcol] += sum_c A[row][c] U_C[c][pcol] + B[row][c] Y_C[c][pcol]
      // column side: out_C^T[pcol][c] += sum_r U_R[r][pcol] A[r][c] + Y_R[r][pcol] B[r][c]
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float a1 = tAw[li * LP + 4 * j + lk];
        const float a2 = tAw[(4 * j + lk) * LP + li];
        const float b1 = tBw[li * LP + 4 * j + lk];
        const float b2 = tBw[(4 * j + lk) * LP + li];
        const int rc = (sc * 16 + 4 * j + lk) * LPW + li;
        const int rr = (w * 16 + 4 * j + lk) * LPW + li;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          accR[c] = mfma(a1, sUc[rc + 16 * c], accR[c]);
          accR[c] = mfma(b1, sYc[rc + 16 * c], accR[c]);
          if (!diag) {
            accC[sc][c] = mfma(sUr[rr + 16 * c], a2, accC[sc][c]);
            accC[sc][c] = mfma(sYr[rr + 16 * c], b2, accC[sc][c]);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // row-side partial of this tile: rows w*16 + 4 lk + v, columns col0 + c*16 + li
    float* rp = a.rowpart + ((size_t)t * 64 + w * 16) * pw + col0 + li;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) rp[(4 * lk + v) * pw + 16 * c] = accR[c][v];
  }
  // column-side partial of the segment: sum of the four waves (row sub-blocks)
  float* cred = tA;  // 3 x 256 floats (the transpose buffers are free now)
  float* cp = a.colpart + (size_t)sidx * 64 * pw;
  for (int sc = 0; sc < 4; ++sc) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      __syncthreads();
      if (w > 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) cred[(w - 1) * 256 + (4 * lk + v) * 16 + li] = accC[sc][c][v];
      }
      __syncthreads();
      if (w == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pc = 4 * lk + v;
          float sum = accC[sc][c][v];
          sum += cred[0 * 256 + pc * 16 + li];
          sum += cred[1 * 256 + pc * 16 + li];
          sum += cred[2 * 256 + pc * 16 + li];
          cp[(sc * 16 + li) * pw + col0 + c * 16 + pc] = sum;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// row finalisers: thread per (row, pcol); 16 lanes per row
// ---------------------------------------------------------------------------
struct RowArgs {
  int n, p, pw, nb, nseg;
  const int* seg_start;  // nb + 1
  const void* rowpart;
  const void* colpart;
};

// sum of the partials of output (r, k): the row-side partials of tiles (I, J),
// J >= I, and the column-side partials of the segments of column block I;
// with spl > 1 this lane takes every spl-th of them, starting at `part`
template <typename T>
__device__ __forceinline__ double row_sum(const RowArgs& ra, int r, int k, int part = 0, int spl = 1) {
  const int I = r >> 6, rr = r & 63;
  const T* rp = (const T*)ra.rowpart;
  const T* cp = (const T*)ra.colpart;
  const int pw = ra.pw;
  double s = 0.0;
#pragma unroll 8
  for (int J = I + part; J < ra.nb; J += spl) {
    const long long t = ((long long)J * (J + 1) >> 1) + I;
    s += (double)rp[((size_t)t * 64 + rr) * pw + k];
  }
  for (int q = ra.seg_start[I] + part; q < ra.seg_start[I + 1]; q += spl)
    s += (double)cp[((size_t)q * 64 + rr) * pw + k];
  return s;
}

// Thread layout of the split row finalisers: L = min(pw, 64) columns per row,
// each (row, column) shared by SPL = 64 / L lanes (pw <= 32) that split its
// partial sums; lane index = (row * L + column) * SPL + part.  Sums over the
// SPL lanes and over the L columns of a row are xor butterflies, which give
// every lane the same bits (each step adds a commuted pair).
__device__ __forceinline__ int row_split(int pw) { return pw >= 64 ? 1 : 64 / pw; }
__device__ __forceinline__ double sum_parts(double v, int spl) {
  for (int off = 1; off < spl; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double sum_row_split(double v, int L, int spl) {
  for (int off = L >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off * spl, 64);
  return v;
}

// sum over the pw lanes of one row (pw = 16, 32 or 64), fixed butterfly order
__device__ __forceinline__ double sum_row(double v, int pw) {
  for (int off = pw >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, pw);
  return v;
}

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 16);
  return v;
}

// Threads: L = min(pw, 64) lanes per row; lane c0 owns columns c0, c0 + L,
// ... (RM of them, RM = pw / 64 rounded up to a power of two for pw > 64);
// row dots are butterfly sums over the L lanes.
__device__ __forceinline__ int row_lanes(int pw) { return pw < 64 ? pw : 64; }

template <int RM>
__global__ __launch_bounds__(256) void k_row_grad(RowArgs ra, const double* __restrict__ Y,
                                                  double* __restrict__ egrad, double* __restrict__ rgrad,
                                                  double* __restrict__ zvec) {
  const int L = row_lanes(ra.pw), spl = row_split(ra.pw);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int part = idx % spl, rc = idx / spl;
  const int r = rc / L, c0 = rc % L;
  const bool in = r < ra.n;
  double gy[RM], y[RM];
  double zp = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    const bool kin = in && k < ra.p && k < ra.pw;
    gy[j] = sum_parts(kin ? row_sum<double>(ra, r, k, part, spl) : 0.0, spl);
    y[j] = kin ? Y[(size_t)r * ra.p + k] : 0.0;
    zp += gy[j] * y[j];
  }
  const double z = sum_row_split(zp, L, spl);
  if (in && c0 == 0 && part == 0) zvec[r] = z;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    if (in && part == 0 && k < ra.p && k < ra.pw) {
      if (egrad) egrad[(size_t)r * ra.p + k] = 2.0 * gy[j];
      if (rgrad) rgrad[(size_t)r * ra.p + k] = 2.0 * (gy[j] - z * y[j]);
    }
  }
}

// lr (nullable, n x p): precomputed low-rank term (wide factors); otherwise
// it is formed here from the Gram matrices.  dotpart (nullable): the block's
// partial of <U, HU> (fixed-order tree over the block), for the tCG curvature.
template <typename T, int RM>
__global__ __launch_bounds__(256) void k_row_hvp(RowArgs ra, const double* __restrict__ Y,
                                                 const double* __restrict__ U, const double* __restrict__ gram,
                                                 const double* __restrict__ lr_pre, const double* __restrict__ zvec,
                                                 double sigma, int riem, double* __restrict__ HU,
                                                 double* __restrict__ dotpart, double* __restrict__ nonfin) {
  const int pw = ra.pw, L = row_lanes(pw), spl = row_split(pw);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int part = idx % spl, rc = idx / spl;
  const int r = rc / L, c0 = rc % L;
  const bool in = r < ra.n;
  // low-rank terms sigma [Y (Y^T U + U^T Y) + U (Y^T Y)]: sigma S U and the
  // rank-2p part of sigma (Y U^T + U Y^T) Y (the tiles carry neither)
  const double* YtY = gram;
  const double* YtU = gram + GRAM_U;
  double Ht[RM], y[RM], u[RM];
  double dp = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    const bool kin = in && k < ra.p && k < pw;
    double h = kin ? row_sum<T>(ra, r, k, part, spl) : 0.0;
    double lr = 0.0;
    if (kin) {
      if (lr_pre) {
        if (part == 0) lr = lr_pre[(size_t)r * ra.p + k];
      } else {
        for (int i = part; i < ra.p; i += spl) {
          const double yi = Y[(size_t)r * ra.p + i];
          const double ui = U[(size_t)r * ra.p + i];
          lr += yi * (YtU[k * pw + i] + YtU[i * pw + k]) + ui * YtY[i * pw + k];
        }
      }
    }
    Ht[j] = 2.0 * sum_parts(h + sigma * lr, spl);
    y[j] = kin ? Y[(size_t)r * ra.p + k] : 0.0;
    u[j] = kin ? U[(size_t)r * ra.p + k] : 0.0;
    dp += Ht[j] * y[j];
  }
  const double d = riem ? sum_row_split(dp, L, spl) : 0.0;
  const double zr = (riem && in) ? zvec[r] : 0.0;
  double uh = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    if (in && part == 0 && k < ra.p && k < pw) {
      const double v = riem ? Ht[j] - d * y[j] - 2.0 * zr * u[j] : Ht[j];
      if (!isfinite(v)) *nonfin = 1.0;  // sticky non-finite flag
      HU[(size_t)r * ra.p + k] = v;
      uh += u[j] * v;
    }
  }
  if (dotpart) {
    __shared__ double red[256];
    red[threadIdx.x] = uh;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) dotpart[blockIdx.x] = red[0];
  }
}

// out[0] = sum of nblk partials in a fixed order (one block)
__global__ __launch_bounds__(256) void k_sum_partials(int nblk, const double* __restrict__ part,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void k_row_mult(RowArgs ra, const double* __restrict__ Y,
                                                  double* __restrict__ zmult, double* __restrict__ zout,
                                                  double* __restrict__ zpart) {
  __shared__ double red[256];
  const int L = row_lanes(ra.pw);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx / L, c0 = idx % L;
  const bool in = r < ra.n;
  double zp = 0.0;
  for (int k = c0; k < ra.pw; k += L) {
    const bool kin = in && k < ra.p;
    const double o = kin ? row_sum<double>(ra, r, k) : 0.0;
    zp += o * (kin ? Y[(size_t)r * ra.p + k] : 0.0);
  }
  const double z = sum_row(zp, L);
  if (in && c0 == 0) {
    zmult[r] = z;
    if (zout) zout[r] = z;
  }
  red[threadIdx.x] = (in && c0 == 0) ? z : 0.0;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) zpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_row_xmv(RowArgs ra, const double* __restrict__ V,
                                                 const double* __restrict__ zmult, double* __restrict__ XV) {
  const int L = row_lanes(ra.pw);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx / L, c0 = idx % L;
  if (r >= ra.n) return;
  for (int k = c0; k < ra.p && k < ra.pw; k += L) {
    const double o = row_sum<double>(ra, r, k);
    XV[(size_t)r * ra.p + k] = o - zmult[r] * V[(size_t)r * ra.p + k];
  }
}

// scalar reduction (single block, fixed order)
__global__ __launch_bounds__(256) void k_scalars(int mode, const double* __restrict__ wgpart, int nseg,
                                                 const double* __restrict__ zpart, int nz,
                                                 const double* __restrict__ btypart, int nbty, double sigma,
                                                 double* scal, double* f_out, double* kkt_out, int frozen) {
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
  __syncthreads();
  red[threadIdx.x] = threadIdx.x < nbty ? btypart[threadIdx.x] : 0.0;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double bty = red[0];
    const double r2 = tot[0], xz = tot[1], cx = tot[3];
    scal[SC_R2] = r2;
    scal[SC_XZ] = xz;
    scal[SC_BTY] = bty;
    if (mode == M_GRAD) {
      // <D, Z> = b^T y(S) (section 3 opening); with a stale y (direct-DSDP
      // subproblem) it is accumulated entry by entry instead
      const double f = (frozen ? tot[2] : bty) + xz + 0.5 * sigma * r2;
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

// Gram matrices Y^T Y and Y^T U (pw x pw, FP64, row pitch pw) with MFMA over
// 4-row chunks.  The NC x NC grid of 16 x 16 block pairs (NC = pw / 16) is
// spread over the four waves and over groups (blockIdx.y) of at most 16
// pairs, four per wave; for NC = 1 the waves split the rows instead.  Every
// (block, row group) writes its own partial; a fixed-order final sum follows.
// with_yy = 0 skips Y^T Y (kept from an earlier call at the same Y).
struct GramSplit {
  int NC, NPAIR, RS, PPW, NGRP;
  __host__ __device__ explicit GramSplit(int pw) {
    NC = pw / 16;
    NPAIR = NC * NC;
    RS = NPAIR >= 4 ? 1 : 4 / NPAIR;                            // row groups
    PPW = NPAIR >= 16 ? 4 : (NPAIR >= 4 ? NPAIR / 4 : 1);       // pairs per wave
    NGRP = NPAIR >= 16 ? NPAIR / 16 : 1;                         // pair groups
  }
};

__global__ __launch_bounds__(256) void k_gram_part(int n, int p, int pw, int with_yy, const double* __restrict__ Y,
                                                   const double* __restrict__ U, double* __restrict__ part) {
  const GramSplit GS(pw);
  const int NC = GS.NC, RS = GS.RS, PPW = GS.PPW;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int per = (n + gridDim.x - 1) / gridDim.x;
  const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  const int rg = w % RS, pbase = blockIdx.y * 4 * PPW + (w / RS) * PPW;
  v4d ayy[4], ayu[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ayy[q] = v4d{0, 0, 0, 0};
    ayu[q] = v4d{0, 0, 0, 0};
  }
  for (int rb = r0 + 4 * rg; rb < r1; rb += 4 * RS) {
    const int r = rb + lk;
    const bool rok = r < r1;
    // A[i][k] = Y[r_k][i] (lane i + 16 k), B[k][j] = Y[r_k][j] / U[r_k][j]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q >= PPW) break;
      const int pr = pbase + q, bi = pr / NC, bj = pr % NC;
      const int ci = 16 * bi + li, cj = 16 * bj + li;
      const double yi = (rok && ci < p) ? Y[(size_t)r * p + ci] : 0.0;
      const double uj = (rok && cj < p) ? U[(size_t)r * p + cj] : 0.0;
      if (with_yy) {
        const double yj = (rok && cj < p) ? Y[(size_t)r * p + cj] : 0.0;
        ayy[q] = mfma(yi, yj, ayy[q]);
      }
      ayu[q] = mfma(yi, uj, ayu[q]);
    }
  }
  double* out = part + ((size_t)blockIdx.x * RS + rg) * 2 * pw * pw;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q >= PPW) break;
    const int pr = pbase + q, bi = pr / NC, bj = pr % NC;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = drow<double>(lk, v);
      if (with_yy) out[(16 * bi + rr) * pw + 16 * bj + li] = ayy[q][v];
      out[pw * pw + (16 * bi + rr) * pw + 16 * bj + li] = ayu[q][v];
    }
  }
}

__global__ __launch_bounds__(256) void k_gram_final(int nblk, int len, int e0, const double* __restrict__ part,
                                                    double* __restrict__ gram, int pw, int per_thread) {
  // part: nblk x (2 pw^2); gram: Y^T Y at [0, pw^2), Y^T U at [GRAM_U, GRAM_U + pw^2).
  // Elements e0 .. len - 1.  per_thread = 0: one wave per element, lanes take
  // every 64th partial, then a butterfly; 1: one thread per element, partials
  // added in order.
  const int pw2 = pw * pw;
  if (per_thread) {
    const int e = e0 + blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * len + e];
    gram[e < pw2 ? e : GRAM_U + (e - pw2)] = s;
    return;
  }
  const int e = e0 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= len) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += part[(size_t)b * len + e];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) gram[e < pw2 ? e : GRAM_U + (e - pw2)] = s;
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

// y export: the class averages of the last S-pass
__global__ __launch_bounds__(256) void k_y_export(long long m, const double2* __restrict__ cy, double* __restrict__ y) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < m) y[g] = cy[g].y;
}

// dense <-> tile layout for Xt
__global__ __launch_bounds__(256) void k_set_dense(int n, int nb, long long nslots, const double* __restrict__ X,
                                                   double* __restrict__ Xt, float* __restrict__ Xt32,
                                                   double* __restrict__ nonfin) {
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
  if (!isfinite(v)) *nonfin = 1.0;  // sticky non-finite flag
  Xt[s] = v;
  Xt32[slot32(s)] = (float)v;
}

__global__ __launch_bounds__(256) void k_get_dense(int n, int nb, long long nslots, const double* __restrict__ Xt,
                                                   const uint32_t* __restrict__ cls, const double2* __restrict__ cy,
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
  if (add_D) v += coef_of(cls[s]) * cy[cls[s] & CLS_MASK].x;
  X[(size_t)r * n + c] = v;
  X[(size_t)c * n + r] = v;
}

// vector helpers for the solver (deterministic two-stage dot products)
__global__ __launch_bounds__(256) void k_dots(DotPtrs dp, int npairs, long long len, double* __restrict__ part) {
  __shared__ double red[256];
  for (int q = 0; q < npairs; ++q) {
    double s = 0.0;
    const double* x = dp.a[q];
    const double* y = dp.b[q];
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
  __shared__ double red[256];
  const int q = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[(size_t)q * nblk + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = red[0];
}

// h_j = <V_j, w> for j < k: one block per basis vector (fixed order)
__global__ __launch_bounds__(256) void k_vt_w(int n, const double* __restrict__ V, const double* __restrict__ w,
                                              double* __restrict__ h) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += V[(size_t)j * n + i] * w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[j] = red[0];
}

// QT = Q^T for a row-major n x r Q (QT row-major r x n), 16 x 16 tiles via LDS
__global__ __launch_bounds__(256) void k_transpose(int n, int r, const double* __restrict__ Q, double* __restrict__ QT) {
  __shared__ double t[16][17];
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (i0 + ty < n && j0 + tx < r) t[ty][tx] = Q[(size_t)(i0 + ty) * r + j0 + tx];
  __syncthreads();
  if (j0 + ty < r && i0 + tx < n) QT[(size_t)(j0 + ty) * n + i0 + tx] = t[tx][ty];
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

// truncated-CG update (Steihaug-Toint step), from the iterate of step j
// (suffix _c) into that of step j + 1 (suffix _n): L lanes per row (L = the
// smallest power of two >= p, at most 64), lane c0 owns columns c0, c0 + L, ...
// The step length alpha = rr / <d, Hd> is formed here from sc_c = {rr, <d, Hd>}
// of step j, so the host can enqueue the update before it has read them.
// part 1: eta_n = eta_c + alpha d; Heta_n = Heta_c + alpha Hd;
// r_n = P_Y(r_c + alpha Hd); block partials of ||r_n||^2
template <int RM>
__global__ __launch_bounds__(256) void k_tcg_update1(int n, int p, int L, const double* __restrict__ Y,
                                                     const double* __restrict__ sc_c,
                                                     const double* __restrict__ eta_c,
                                                     const double* __restrict__ Heta_c,
                                                     const double* __restrict__ r_c, const double* __restrict__ d_c,
                                                     const double* __restrict__ Hd_c, double* __restrict__ eta_n,
                                                     double* __restrict__ Heta_n, double* __restrict__ r_n,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  const double alpha = sc_c[0] / sc_c[1];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = idx / L, c0 = idx % L;
  const bool in = i < n;
  double rn[RM];
  double dr = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    rn[j] = 0.0;
    if (in && k < p) {
      const size_t o = (size_t)i * p + k;
      eta_n[o] = eta_c[o] + alpha * d_c[o];
      Heta_n[o] = Heta_c[o] + alpha * Hd_c[o];
      rn[j] = r_c[o] + alpha * Hd_c[o];
      dr += rn[j] * Y[o];
    }
  }
  for (int off = L >> 1; off >= 1; off >>= 1) dr += __shfl_xor(dr, off, L);
  double rr = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    if (in && k < p) {
      const size_t o = (size_t)i * p + k;
      rn[j] -= dr * Y[o];
      r_n[o] = rn[j];
      rr += rn[j] * rn[j];
    }
  }
  red[threadIdx.x] = rr;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// part 2: rr_n = ||r_n||^2 from part 1's nblk partials (every block sums them
// in the same fixed order), beta = rr_n / rr_c, d_n = P_Y(-r_n + beta d_c);
// block 0 writes sc_n[0] = rr_n
template <int RM>
__global__ __launch_bounds__(256) void k_tcg_update2(int n, int p, int L, const double* __restrict__ Y, int nblk,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ sc_c, double* __restrict__ sc_n,
                                                     const double* __restrict__ r_n,
                                                     const double* __restrict__ d_c, double* __restrict__ d_n) {
  __shared__ double red[256];
  {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
  }
  const double rr_new = red[0], beta = rr_new / sc_c[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) sc_n[0] = rr_new;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = idx / L, c0 = idx % L;
  const bool in = i < n;
  double dn[RM];
  double dd = 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    dn[j] = 0.0;
    if (in && k < p) {
      const size_t o = (size_t)i * p + k;
      dn[j] = -r_n[o] + beta * d_c[o];
      dd += dn[j] * Y[o];
    }
  }
  for (int off = L >> 1; off >= 1; off >>= 1) dd += __shfl_xor(dd, off, L);
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const int k = c0 + j * L;
    if (in && k < p) {
      const size_t o = (size_t)i * p + k;
      d_n[o] = dn[j] - dd * Y[o];
    }
  }
}

// Yout (n x q) = Yin (n x p) M (p x q, row-major); optional row normalisation
// (one thread per row; the row norm is taken in a first pass)
__global__ __launch_bounds__(256) void k_rightmul(int n, int p, int q, const double* __restrict__ Yin,
                                                  const double* __restrict__ M, int normalize,
                                                  double* __restrict__ Yout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double nrm = 0.0;
  if (normalize) {
    for (int c = 0; c < q; ++c) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += Yin[(size_t)i * p + k] * M[k * q + c];
      nrm += s * s;
    }
  }
  const double inv = (normalize && nrm > 0.0) ? 1.0 / sqrt(nrm) : 1.0;
  for (int c = 0; c < q; ++c) {
    double s = 0.0;
    for (int k = 0; k < p; ++k) s += Yin[(size_t)i * p + k] * M[k * q + c];
    Yout[(size_t)i * q + c] = s * inv;
  }
}

// rank-one compression: out_i = sign((Y v)_i) in {+1, -1} (zero to +1), the
// width-1 point of the oblique manifold nearest the leading direction v of Y
__global__ __launch_bounds__(256) void k_sign_col(int n, int p, const double* __restrict__ Yin,
                                                  const double* __restrict__ v, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < p; ++k) s += Yin[(size_t)i * p + k] * v[k];
  out[i] = (s >= 0.0) ? 1.0 : -1.0;
}

// column `col` of U (n x p) = v; with zero_rest the other columns are cleared
__global__ __launch_bounds__(256) void k_set_col(int n, int p, int col, const double* __restrict__ v,
                                                 double* __restrict__ U, int zero_rest) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (zero_rest)
    for (int k = 0; k < p; ++k) U[(size_t)i * p + k] = (k == col) ? v[i] : 0.0;
  else
    U[(size_t)i * p + col] = v[i];
}

// w -= V h  (V: k column vectors of length n stored one after another)
__global__ __launch_bounds__(256) void k_gemv_sub(int n, int k, const double* __restrict__ V,
                                                  const double* __restrict__ h, double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += V[(size_t)j * n + i] * h[j];
  w[i] -= s;
}

// out = V s (Ritz vector)
__global__ __launch_bounds__(256) void k_gemv(int n, int k, const double* __restrict__ V,
                                              const double* __restrict__ sv, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += V[(size_t)j * n + i] * sv[j];
  out[i] = s;
}

// ---------------------------------------------------------------------------
// generic class-sum finalisation: fixed-point sums -> class averages
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_final_S(long long m, long long* __restrict__ sacc,
                                                 const double* __restrict__ invc, const double* __restrict__ Cavg,
                                                 const double* __restrict__ scal, double2* __restrict__ cy) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  double y = (double)sacc[g] / scal[SC_SCALE_S] * invc[g];
  if (Cavg) y += Cavg[g];
  sacc[g] = 0;
  cy[g].y = y;
}

__global__ __launch_bounds__(256) void k_final_Z(long long m, long long* __restrict__ sacc,
                                                 const double* __restrict__ invc, const double* __restrict__ scal,
                                                 double sigma, double2* __restrict__ ab64) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  ab64[g].y = -sigma * ((double)sacc[g] / scal[SC_SCALE_Z] * invc[g]);
  sacc[g] = 0;
}

// FP64 HVP: class coefficient D - sigma y of U (y of the last S-pass)
__global__ __launch_bounds__(256) void k_make_a64(long long m, const double2* __restrict__ cy, double sigma,
                                                  double2* __restrict__ ab64) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  const double2 dy = cy[g];
  ab64[g].x = dy.x - sigma * dy.y;
}

// FP32-tile HVP: class coefficient -sigma y' of Y
__global__ __launch_bounds__(256) void k_final_Z32(long long m, long long* __restrict__ sacc,
                                                   const double* __restrict__ invc, const double* __restrict__ scal,
                                                   double sigma, float2* __restrict__ ab32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  ab32[g].y = (float)(-sigma * ((double)sacc[g] / scal[SC_SCALE_Z] * invc[g]));
  sacc[g] = 0;
}

// FP32-tile HVP: class coefficient D - sigma y of U (y of the last S-pass)
// direct-DSDP subproblem: its Hessian in S is sigma I (no projection), so the
// class coefficient of Y in the HVP is zero
__global__ __launch_bounds__(256) void k_zero_ycoef(long long m, double2* __restrict__ ab64, float2* __restrict__ ab32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  ab64[g].y = 0.0;
  ab32[g].y = 0.0f;
}
__global__ __launch_bounds__(256) void k_make_a32(long long m, const double2* __restrict__ cy, double sigma,
                                                  float2* __restrict__ ab32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m) return;
  const double2 dy = cy[g];
  ab32[g].x = (float)(dy.x - sigma * dy.y);
}

// b^T y over the classes that may carry b != 0 (deterministic two-stage)
__global__ __launch_bounds__(256) void k_bty_part(long long range, const double* __restrict__ b,
                                                  const double2* __restrict__ cy, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < range; g += (long long)gridDim.x * 256)
    acc += b[g] * cy[g].y;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Structured class averages of the order-2 BQP moment relaxation
// (paragraph on BQPs: basis v(x), classes by symmetric difference), colex
// basis and colex class ids.  For the symmetric bilinear form
//   B(alpha, beta) = Y_alpha . Y_beta                      (S-pass, Z = Y Y^T)
//   B(alpha, beta) = Y_alpha . U_beta + U_alpha . Y_beta   (HVP, Z = Y U^T + U Y^T)
// the ordered class sum of class gamma is twice the sum of B over the
// unordered entry pairs of the class (plus the diagonal for gamma = {}):
//   {a<b<c<d}: (ab|cd) + (ac|bd) + (ad|bc)        |gamma| = 6
//   {a<b<c}  : (a|bc) + (b|ac) + (c|ab)           |gamma| = 6
//   {i<j}    : ({}|ij) + (i|j) + sum_l (il|jl)     |gamma| = 2q
//   {i}      : ({}|i) + sum_j (j|ij)              |gamma| = 2q
//   {}       : sum_alpha B(alpha, alpha)          |gamma| = n
// Degree 4 (96% of the classes), two passes over the pair rows of the basis
// (in colex order the rows {x, c}, x < c, are consecutive, and so are the
// pair rows t = C(b, 2) + a themselves):
// (for factors of at most 32 columns a single-pass kernel, bqp4_block, is
// used instead: see there)
//   pass 1 (k_bqp_pass1): (ab|cd) for fixed d is an MFMA GEMM of the rows
//     {c, d} of a 16-block of c against 64 consecutive pair rows t, masked to
//     t < C(c, 2); kept in p1[C(d, 4) + C(c, 3) + t] (the degree-4 local id);
//   pass 2 (k_bqp_pass2): one workgroup per (c, d) forms the full c x c matrix
//     M[x][y] = (xc|yd) from LDS-staged chunks of the rows {x, c} and {y, d};
//     then (ac|bd) + (ad|bc) = M[a][b] + M[b][a], transposed through LDS, is
//     added to p1 and each class {a<b<c<d} is written once.
// Degrees 0-3 read the table T[r][x] = B(row r, row x) of every basis row r
// against the rows {} and {i} (one small GEMM, the k_bqpT tasks), and the
// contraction star[i][j] = sum_l (il|jl) (the k_bqpStar tasks, partials over
// residues of l), both launched with pass 1, and are finished by k_bqpFin.
// No class map is read, no atomics are used, every sum has a fixed order.
// MFMA operands come straight from the staged rows: lane (i, k) loads the
// W-vector of columns W k .. W k + W - 1 of row i, and the W MFMAs of a
// 4W-column chunk use its W components (a permutation of the contraction
// index shared by both operands).
// ---------------------------------------------------------------------------
// binomials without 64-bit integer division (emulated on the GPU): x <= 362
__device__ __forceinline__ long long c2(long long x) { return (x * (x - 1)) >> 1; }
__device__ __forceinline__ long long c3(long long x) {
  const int xi = (int)x;
  return xi < 3 ? 0 : (long long)((unsigned)(xi * (xi - 1) * (xi - 2)) / 6u);
}
__device__ __forceinline__ long long c4(long long x) {
  const long long t = c3(x);  // C(x,4) = C(x,3) (x - 3) / 4, exact
  return x < 4 ? 0 : (t * (x - 3)) >> 2;
}
// largest c with C(c, 3) <= t, and largest b with C(b, 2) <= t (t < 2^24:
// a single-precision first guess, corrected exactly in integers)
__device__ __forceinline__ int inv_c3(long long t) {
  int c = (int)cbrtf(6.0f * (float)t) + 1;
  while (c3(c) > t) --c;
  while (c3(c + 1) <= t) ++c;
  return c;
}
__device__ __forceinline__ int inv_c2(long long t) {
  int b = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
  while (c2(b) > t) --b;
  while (c2(b + 1) <= t) ++b;
  return b;
}

struct BqpArgs {
  int q;
  int pw;              // row pitch of the staged factors
  int nkc;             // 16-column chunks covering p
  long long off2, off3, off4;
  const void* Yp;
  const void* Up;
  const int4* items4;  // single-pass work items (c, d0, a0, b0)
  const int4* items;   // pass-1 work items (d, c0, t0, 0)
  const int2* items2;  // pass-2 work items (c, d)
  void* p1;            // pass-1 results (T), C(q, 4) of them
  double* T;           // n x (q + 1) table B(row r, row x), x in {}, {0}, ..., {q-1}
  double* star;        // STAR_LG x q x q partials of sum_l (il|jl), as [lg][j][i]
  double* dst;         // output element g at dst[g * stride]
  int stride;          // 2: the .y field of cy (S-pass) or of ab64 (FP64 HVP)
  double* part;        // degree-0 partials
  float2* dst32;       // FP32-tile HVP: class coefficient -sigma y'_g written to dst32[g].y instead
  double scale32;      // -sigma
};

// final class average `val` of class g: the S-pass class average (FP64), or
// the HVP class coefficient -sigma val (FP64 or FP32)
template <typename T, bool ZMODE>
__device__ __forceinline__ void bqp_store(const BqpArgs& a, long long g, double val) {
  if (ZMODE && sizeof(T) == 4)
    a.dst32[g].y = (float)(a.scale32 * val);
  else if (ZMODE)
    a.dst[g * a.stride] = a.scale32 * val;
  else
    a.dst[g * a.stride] = val;
}

// row of the colex basis: {} -> 0, {i} -> 1 + i, {i<j} -> 1 + q + C(j,2) + i
__device__ __forceinline__ int prow(int q, int i, int j) { return 1 + q + (int)c2(j) + i; }
// row of the pair {x, y}; row 0 (a valid row whose products are discarded)
// when x == y or an index is out of range
__device__ __forceinline__ int pair_row(int q, int x, int y) {
  if (x == y || x < 0 || y < 0 || x >= q || y >= q) return 0;
  return x < y ? prow(q, x, y) : prow(q, y, x);
}

template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4(const T* p) {
  return *(const typename V4<T>::type*)p;
}

// acc += B(row ra, row rb) over the 16-column chunks (A rows per lane li,
// B rows per lane li; lane (li, lk) reads columns 16 kc + 4 lk .. + 3)
template <typename T, bool ZMODE>
__device__ __forceinline__ void bform_mfma(const T* Y, const T* U, size_t ra, size_t rb, int nkc, int lk,
                                           typename V4<T>::type& acc) {
  for (int kc = 0; kc < nkc; ++kc) {
    const int k0 = 16 * kc + 4 * lk;
    const auto ya = ld4(Y + ra + k0), yb = ld4(Y + rb + k0);
    if (ZMODE) {
      const auto ua = ld4(U + ra + k0), ub = ld4(U + rb + k0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc = mfma(ya[e], ub[e], acc);
        acc = mfma(ua[e], yb[e], acc);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = mfma(ya[e], yb[e], acc);
    }
  }
}

// Single-pass degree-4 variant for narrow factors (p <= 32, where the two
// passes below are bound by latency rather than by the matrix cores): one
// (c, 16 d's, 16 a's, 16 b's) block per workgroup; (ab|cd) is an MFMA tile in
// (a, d) for each b, (ac|bd) + (ad|bc) an MFMA tile in (a, b) for each d, and
// the first is transposed through LDS onto the second.
template <typename T, bool ZMODE>
__device__ __forceinline__ void bqp4_block(const BqpArgs& a, int item) {
  typedef typename V4<T>::type v4;
  constexpr int DB = 2;            // d values whose operands are loaded together
  __shared__ T t1s[16 * 16 * 17];  // (ab|cd) as [b][a][d]
  const int4 it = a.items4[item];
  const int c = it.x, d0 = it.y, a0 = it.z, b0 = it.w;
  const int q = a.q, pw = a.pw, nkc = a.nkc;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const T* Y = (const T*)a.Yp;
  const T* U = (const T*)a.Up;
  // (ab|cd): for b = b0 + 4 w + bb an MFMA tile with rows a = a0 + i, columns d = d0 + j
  {
    const size_t rcd = (size_t)pair_row(q, c, d0 + li) * pw;
    size_t rab[4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) rab[bb] = (size_t)pair_row(q, a0 + li, b0 + 4 * w + bb) * pw;
    v4 acc[4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) acc[bb] = v4{0, 0, 0, 0};
    for (int kc = 0; kc < nkc; ++kc) {
      const int k0 = 16 * kc + 4 * lk;
      const v4 yb = ld4(Y + rcd + k0);
      const v4 ub = ZMODE ? ld4(U + rcd + k0) : yb;
      v4 ya[4], ua[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        ya[bb] = ld4(Y + rab[bb] + k0);
        ua[bb] = ZMODE ? ld4(U + rab[bb] + k0) : ya[bb];
      }
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (ZMODE) {
            acc[bb] = mfma(ya[bb][e], ub[e], acc[bb]);
            acc[bb] = mfma(ua[bb][e], yb[e], acc[bb]);
          } else {
            acc[bb] = mfma(ya[bb][e], yb[e], acc[bb]);
          }
        }
    }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int v = 0; v < 4; ++v) t1s[((4 * w + bb) * 16 + drow<T>(lk, v)) * 17 + li] = acc[bb][v];
  }
  __syncthreads();
  // (ac|bd) + (ad|bc): for d = d0 + 4 w + dd an MFMA tile with rows a = a0 + i, columns b = b0 + j
  const size_t rac = (size_t)pair_row(q, a0 + li, c) * pw;
  const size_t rbc = (size_t)pair_row(q, b0 + li, c) * pw;
  const long long base_c = a.off4 + c3(c);
  const int bn = b0 + li;
  // FP32 tiles: (ac|bd) and (ad|bc) are two entries of the class and get their
  // own accumulators, so that the class sum itself is formed in FP64
  constexpr bool SPLIT = sizeof(T) == 4;
  v4 accd[4], accd2[4];
  for (int dh = 0; dh < 4; dh += DB) {
    size_t rad[DB], rbd[DB];
#pragma unroll
    for (int u = 0; u < DB; ++u) {
      const int d = d0 + 4 * w + dh + u;
      rad[u] = (size_t)pair_row(q, a0 + li, d) * pw;
      rbd[u] = (size_t)pair_row(q, bn, d) * pw;
    }
    v4 acc[DB], acc2[DB];
#pragma unroll
    for (int u = 0; u < DB; ++u) acc[u] = acc2[u] = v4{0, 0, 0, 0};
    for (int kc = 0; kc < nkc; ++kc) {
      const int k0 = 16 * kc + 4 * lk;
      const v4 yac = ld4(Y + rac + k0), ybc = ld4(Y + rbc + k0);
      const v4 uac = ZMODE ? ld4(U + rac + k0) : yac, ubc = ZMODE ? ld4(U + rbc + k0) : ybc;
      v4 yad[DB], ybd[DB], uad[DB], ubd[DB];
#pragma unroll
      for (int u = 0; u < DB; ++u) {
        yad[u] = ld4(Y + rad[u] + k0);
        ybd[u] = ld4(Y + rbd[u] + k0);
        uad[u] = ZMODE ? ld4(U + rad[u] + k0) : yad[u];
        ubd[u] = ZMODE ? ld4(U + rbd[u] + k0) : ybd[u];
      }
#pragma unroll
      for (int u = 0; u < DB; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (ZMODE) {
            acc[u] = mfma(yac[e], ubd[u][e], acc[u]);
            acc[u] = mfma(uac[e], ybd[u][e], acc[u]);
            if (SPLIT) {
              acc2[u] = mfma(yad[u][e], ubc[e], acc2[u]);
              acc2[u] = mfma(uad[u][e], ybc[e], acc2[u]);
            } else {
              acc[u] = mfma(yad[u][e], ubc[e], acc[u]);
              acc[u] = mfma(uad[u][e], ybc[e], acc[u]);
            }
          } else {
            acc[u] = mfma(yac[e], ybd[u][e], acc[u]);
            if (SPLIT)
              acc2[u] = mfma(yad[u][e], ybc[e], acc2[u]);
            else
              acc[u] = mfma(yad[u][e], ybc[e], acc[u]);
          }
        }
    }
#pragma unroll
    for (int u = 0; u < DB; ++u) {
      accd[dh + u] = acc[u];
      accd2[dh + u] = acc2[u];
    }
  }
  // stores last (vector memory counters retire in order: a store ahead of a
  // load would make the load's wait include it)
#pragma unroll
  for (int dd = 0; dd < 4; ++dd) {
    const int d = d0 + 4 * w + dd;
    if (d < q) {
      const long long base = base_c + c4(d);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int al = drow<T>(lk, v), an = a0 + al;
        if (an < bn && bn < c) {
          const double t1 = (double)t1s[(li * 16 + al) * 17 + 4 * w + dd];
          const double t23 = SPLIT ? (double)accd[dd][v] + (double)accd2[dd][v] : (double)accd[dd][v];
          bqp_store<T, ZMODE>(a, base + c2(bn) + an, (t1 + t23) * (1.0 / 3.0));
        }
      }
    }
  }
}

// pass 1: (ab|cd) for the 16 pairs {c, d}, c = c0 .. c0 + 15 (A operand rows,
// loaded once per chunk), against the pair rows t = t0 .. t0 + 63 (four B
// operand tiles); one wave per item
template <typename T, bool ZMODE>
__device__ __forceinline__ void bqp1_item(const BqpArgs& a, int4 it, int lane) {
  typedef typename V4<T>::type v4;
  const int q = a.q, pw = a.pw, li = lane & 15, lk = lane >> 4;
  const int d = it.x, c0 = it.y;
  const long long t0 = it.z, npair = c2(q);
  const T* Y = (const T*)a.Yp;
  const T* U = (const T*)a.Up;
  const int cl = c0 + li;
  const size_t ra = (size_t)(cl < d ? prow(q, cl, d) : 0) * pw;
  size_t rb[4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const long long tl = t0 + 16 * s4 + li;
    rb[s4] = (size_t)(tl < npair ? 1 + q + tl : 0) * pw;
  }
  v4 acc[4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) acc[s4] = v4{0, 0, 0, 0};
  for (int kc = 0; kc < a.nkc; ++kc) {
    const int k0 = 16 * kc + 4 * lk;
    const v4 ya = ld4(Y + ra + k0);
    const v4 ua = ZMODE ? ld4(U + ra + k0) : ya;
    v4 yb[4], ub[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      yb[s4] = ld4(Y + rb[s4] + k0);
      ub[s4] = ZMODE ? ld4(U + rb[s4] + k0) : yb[s4];
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (ZMODE) {
          acc[s4] = mfma(ya[e], ub[s4][e], acc[s4]);
          acc[s4] = mfma(ua[e], yb[s4][e], acc[s4]);
        } else {
          acc[s4] = mfma(ya[e], yb[s4][e], acc[s4]);
        }
      }
  }
  T* p1 = (T*)a.p1;
  const long long base_d = c4(d);
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const long long tl = t0 + 16 * s4 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cc = c0 + drow<T>(lk, v);
      if (cc >= 2 && cc < d && tl < c2(cc)) p1[base_d + c3(cc) + tl] = acc[s4][v];
    }
  }
}

// pair index pi -> (A, B), A <= B, pi = B (B + 1) / 2 + A
__device__ __forceinline__ void pair_of(int pi, int& A, int& B) {
  B = (int)((sqrtf(8.0f * (float)pi + 1.0f) - 1.0f) * 0.5f);
  while (B * (B + 1) / 2 > pi) --B;
  while ((B + 1) * (B + 2) / 2 <= pi) ++B;
  A = pi - B * (B + 1) / 2;
}

// pass 2: one workgroup per (c, d).  R >= 16 ceil(c / 16) staged rows per
// array, chunks of KC = 4 W columns, NP 16-block pairs (A <= B) per wave and
// pass; tiles (A, B) and (B, A) of M are accumulated together.
template <typename T, bool ZMODE, int R, int W, int NP>
__global__ __launch_bounds__(256) void k_bqp_pass2(BqpArgs a) {
  typedef T vw __attribute__((ext_vector_type(W)));
  typedef typename V4<T>::type v4;
  constexpr int KC = 4 * W;
  constexpr int STR = KC + 16 / (int)sizeof(T);  // padded LDS row (16 bytes of padding)
  constexpr int NA = ZMODE ? 4 : 2;               // staged arrays Yc, Yd (, Uc, Ud)
  constexpr int OPS = NA * R * STR;
  constexpr int SCR = 4 * 2 * 16 * 17;            // per-wave transpose tiles
  constexpr int UPR = KC * (int)sizeof(T) / 16;   // 16-byte units per staged row
  __shared__ __align__(16) T lds[OPS > SCR ? OPS : SCR];
  const int2 it = a.items2[blockIdx.x];
  const int c = it.x, d = it.y, q = a.q, pw = a.pw;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int nT = (c + 15) >> 4, npair = nT * (nT + 1) / 2, nrow = 16 * nT;
  const int nchunk = a.nkc * 16 / KC;
  const T* Y = (const T*)a.Yp;
  const T* U = (const T*)a.Up;
  const size_t rowc = (size_t)prow(q, 0, c), rowd = (size_t)prow(q, 0, d);
  T* Yc = lds;
  T* Yd = lds + R * STR;
  T* Uc = lds + 2 * R * STR;
  T* Ud = lds + 3 * R * STR;
  const T* p1 = (const T*)a.p1;
  const long long base4 = c4(d) + c3(c);  // degree-4 local id of {a, b, c, d} minus C(b, 2) + a
  for (int pass = 0; pass * 4 * NP < npair; ++pass) {
    v4 acc[NP][2];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j][0] = acc[j][1] = v4{0, 0, 0, 0};
    for (int ch = 0; ch < nchunk; ++ch) {
      __syncthreads();
      // staged rows x < c of the four arrays (zeros below 16 nT), 16-byte units
      for (int u = tid; u < NA * nrow * UPR; u += 256) {
        const int arr = u / (nrow * UPR), rem = u - arr * (nrow * UPR), x = rem / UPR, part = rem - x * UPR;
        uint4 val = {0u, 0u, 0u, 0u};
        if (x < c) {
          const T* src = (arr < 2 ? Y : U) + ((arr & 1 ? rowd : rowc) + x) * pw + ch * KC;
          val = ((const uint4*)src)[part];
        }
        ((uint4*)(lds + (size_t)arr * R * STR + x * STR))[part] = val;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int pi = pass * 4 * NP + j * 4 + w;
        if (pi < npair) {
          int A, B;
          pair_of(pi, A, B);
          const int oa = (16 * A + li) * STR + W * lk, ob = (16 * B + li) * STR + W * lk;
          const vw yca = *(const vw*)(Yc + oa), ydb = *(const vw*)(Yd + ob);
          const vw ycb = *(const vw*)(Yc + ob), yda = *(const vw*)(Yd + oa);
          if (ZMODE) {
            const vw uca = *(const vw*)(Uc + oa), udb = *(const vw*)(Ud + ob);
            const vw ucb = *(const vw*)(Uc + ob), uda = *(const vw*)(Ud + oa);
#pragma unroll
            for (int e = 0; e < W; ++e) {
              acc[j][0] = mfma(yca[e], udb[e], acc[j][0]);
              acc[j][0] = mfma(uca[e], ydb[e], acc[j][0]);
            }
            if (A != B) {
#pragma unroll
              for (int e = 0; e < W; ++e) {
                acc[j][1] = mfma(ycb[e], uda[e], acc[j][1]);
                acc[j][1] = mfma(ucb[e], yda[e], acc[j][1]);
              }
            }
          } else {
#pragma unroll
            for (int e = 0; e < W; ++e) acc[j][0] = mfma(yca[e], ydb[e], acc[j][0]);
            if (A != B) {
#pragma unroll
              for (int e = 0; e < W; ++e) acc[j][1] = mfma(ycb[e], yda[e], acc[j][1]);
            }
          }
        }
      }
    }
    // M[a][b] + M[b][a] through the wave's two 16 x 17 transpose tiles
    __syncthreads();
    T* S1 = lds + w * 2 * 16 * 17;
    T* S2 = S1 + 16 * 17;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int pi = pass * 4 * NP + j * 4 + w;
      int A = 0, B = 0;
      if (pi < npair) {
        pair_of(pi, A, B);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          S1[drow<T>(lk, v) * 17 + li] = acc[j][0][v];  // S1[a'][b'] = M[16 A + a'][16 B + b']
          S2[drow<T>(lk, v) * 17 + li] = acc[j][1][v];  // S2[b'][a'] = M[16 B + b'][16 A + a']
        }
      }
      __syncthreads();
      if (pi < npair) {
        const T* St = A != B ? S2 : S1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ao = li, bo = 4 * lk + v;
          const int an = 16 * A + ao, bn = 16 * B + bo;
          if (an < bn && bn < c) {
            // the three entries of class {a, b, c, d}, summed in FP64
            const double m2 = (double)S1[ao * 17 + bo] + (double)St[bo * 17 + ao];
            const long long g4 = base4 + c2(bn) + an;
            bqp_store<T, ZMODE>(a, a.off4 + g4, ((double)p1[g4] + m2) * (1.0 / 3.0));
          }
        }
      }
      __syncthreads();
    }
  }
}

// T[r][x] = B(row r, row x) for every basis row r and x in 0..q (row x is {}
// for x = 0 and {x-1} otherwise); blocks with blockIdx.y = 0 also write the
// partial sum of B(row r, row r) over their 16 rows (class {})
template <typename T, bool ZMODE>
__device__ __forceinline__ void bqpT_tile(const BqpArgs& a, int n, int bx, int by, int lane) {
  typedef typename V4<T>::type v4;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = bx * 16, x0 = by * 16;
  const int q = a.q, pw = a.pw;
  const T* Y = (const T*)a.Yp;
  const T* U = (const T*)a.Up;
  const int r = r0 + li, x = x0 + li;
  const size_t ra = (size_t)(r < n ? r : 0) * pw, rx = (size_t)(x <= q ? x : 0) * pw;
  v4 acc = {0, 0, 0, 0};
  bform_mfma<T, ZMODE>(Y, U, ra, rx, a.nkc, lk, acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = r0 + drow<T>(lk, v);
    if (rr < n && x <= q) a.T[(size_t)rr * (q + 1) + x] = (double)acc[v];
  }
  if (by == 0) {
    double d = 0.0;
    if (lk == 0 && r < n) {
      for (int k = 0; k < 16 * a.nkc; ++k) {
        const double yk = (double)Y[ra + k];
        d += ZMODE ? 2.0 * yk * (double)U[ra + k] : yk * yk;
      }
    }
    d = sum16(d);
    if (lane == 0) a.part[bx] = d;
  }
}

// star partials: sum over l = lg, lg + STAR_LG, ... of (il|jl) for the 16 x 16
// tile (I, J), I <= J, of (i, j); the term l = i or l = j is left out.  Stored
// as star[lg][j][i], so that the finisher's threads (consecutive i at fixed j)
// read consecutive addresses.
template <typename T, bool ZMODE>
__device__ __forceinline__ void bqpStar_tile(const BqpArgs& a, int tile, int lg, int lane) {
  typedef typename V4<T>::type v4;
  const int li = lane & 15, lk = lane >> 4;
  int J = 0;
  while ((J + 1) * (J + 2) / 2 <= tile) ++J;
  const int I = tile - J * (J + 1) / 2;
  const int q = a.q, pw = a.pw;
  const T* Y = (const T*)a.Yp;
  const T* U = (const T*)a.Up;
  const int i = 16 * I + li, j = 16 * J + li;
  // each l gives one entry (il|jl) of class {i, j}: FP32 tiles fold it into
  // an FP64 sum after its dot product
  double accs[4] = {0.0, 0.0, 0.0, 0.0};
  v4 acc = {0, 0, 0, 0};
  for (int l = lg; l < q; l += STAR_LG) {
    if (sizeof(T) == 4) acc = v4{0, 0, 0, 0};
    const bool iok = i < q && i != l, jok = j < q && j != l;
    const size_t ri = (size_t)pair_row(q, i, l) * pw, rj = (size_t)pair_row(q, j, l) * pw;
    for (int kc = 0; kc < a.nkc; ++kc) {
      const int k0 = 16 * kc + 4 * lk;
      const v4 z = {0, 0, 0, 0};
      const v4 yi = iok ? ld4(Y + ri + k0) : z, yj = jok ? ld4(Y + rj + k0) : z;
      if (ZMODE) {
        const v4 ui = iok ? ld4(U + ri + k0) : z, uj = jok ? ld4(U + rj + k0) : z;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc = mfma(yi[e], uj[e], acc);
          acc = mfma(ui[e], yj[e], acc);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = mfma(yi[e], yj[e], acc);
      }
    }
    if (sizeof(T) == 4)
#pragma unroll
      for (int v = 0; v < 4; ++v) accs[v] += (double)acc[v];
  }
  if (sizeof(T) != 4)
#pragma unroll
    for (int v = 0; v < 4; ++v) accs[v] = (double)acc[v];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int ii = 16 * I + drow<T>(lk, v);
    if (ii < q && j < q) a.star[((size_t)lg * q + j) * q + ii] = accs[v];
  }
}

// Pass 1 and the degree 0-3 tables in one launch: blocks [0, nb1) give one
// pass-1 item (of n1) to each wave, the blocks after them one T or star tile.
// With single = 1 the first n1 blocks take single-pass degree-4 items instead.
template <typename T, bool ZMODE>
__global__ __launch_bounds__(256) void k_bqp_pass1(BqpArgs a, int n, int n1, int nTx, int nTy, int nS, int single) {
  const int nb1 = single ? n1 : (n1 + 3) / 4;
  if ((int)blockIdx.x < nb1) {
    if (single) {
      bqp4_block<T, ZMODE>(a, blockIdx.x);
      return;
    }
    const int item = (int)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item < n1) bqp1_item<T, ZMODE>(a, a.items[item], threadIdx.x & 63);
    return;
  }
  const int task = ((int)blockIdx.x - nb1) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nT = nTx * nTy;
  if (task < nT)
    bqpT_tile<T, ZMODE>(a, n, task % nTx, task / nTx, lane);
  else if (task < nT + nS * STAR_LG)
    bqpStar_tile<T, ZMODE>(a, (task - nT) % nS, (task - nT) / nS, lane);
}

// Finisher of the structured class sums, one launch: the first nb01 blocks
// take the classes of degree 0 and 1 (one wave each, lanes split the sum,
// fixed butterfly order): {} = sum of the degree-0 partials / n,
// {i} = (({}|i) + sum_j (j|ij)) / q; the other blocks take the classes of
// degree 2 and 3 (one thread each).
template <typename T, bool ZMODE>
__global__ __launch_bounds__(256) void k_bqpFin(BqpArgs a, int n, int nblkT, int nb01) {
  const int q = a.q, ldT = q + 1;
  const double* Tt = a.T;
  if ((int)blockIdx.x < nb01) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (g > q) return;
    double s = 0.0;
    if (g == 0) {
      for (int i = lane; i < nblkT; i += 64) s += a.part[i];
    } else {
      const int i = g - 1;
      if (lane == 0) s = Tt[(size_t)(1 + i) * ldT];
      for (int j = lane; j < q; j += 64)
        if (j != i) s += Tt[(size_t)pair_row(q, i, j) * ldT + 1 + j];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) bqp_store<T, ZMODE>(a, g, s / (double)(g == 0 ? n : q));
    return;
  }
  const long long g = a.off2 + (long long)(blockIdx.x - nb01) * 256 + threadIdx.x;
  if (g >= a.off4) return;
  double val;
  if (g < a.off3) {
    const long long t = g - a.off2;
    const int j = inv_c2(t), i = (int)(t - c2(j));
    double sp[STAR_LG];
#pragma unroll
    for (int lg = 0; lg < STAR_LG; ++lg) sp[lg] = a.star[((size_t)lg * q + j) * q + i];
    double s = Tt[(size_t)prow(q, i, j) * ldT] + Tt[(size_t)(1 + i) * ldT + 1 + j];
#pragma unroll
    for (int lg = 0; lg < STAR_LG; ++lg) s += sp[lg];
    val = s / (double)q;
  } else {
    const long long t = g - a.off3;
    const int c = inv_c3(t);
    const long long t2 = t - c3(c);
    const int b = inv_c2(t2), aa = (int)(t2 - c2(b));
    val = (Tt[(size_t)prow(q, b, c) * ldT + 1 + aa] + Tt[(size_t)prow(q, aa, c) * ldT + 1 + b] +
           Tt[(size_t)prow(q, aa, b) * ldT + 1 + c]) *
          (1.0 / 3.0);
  }
  bqp_store<T, ZMODE>(a, g, val);
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
  a.pw = P->pw;
  a.nsl = P->pw > 64 ? P->pw / 64 : 1;
  a.Xt_out = P->Xt;
  a.Yp = P->Yp;
  a.Up = P->Up;
  a.cy = P->cy;
  a.ab64 = P->ab64;
  a.sacc = P->sacc;
  a.Cavg = P->Cavg;
  a.bound = P->bound;
  a.scal = P->scal;
  a.kmax = (double)P->kmax;
  a.sigma = P->sigma;
  a.rowpart = P->rowpart;
  a.colpart = P->colpart;
  a.wgpart = P->wgpart;
  a.frozen = P->frozen ? 1 : 0;
  return a;
}

static unsigned seg_grid(mdsdp_problem P) { return (unsigned)(8 * ((P->nseg + 7) / 8)); }

// factor width of the staged tiles: 16, 32, 64, or a multiple of 64 (cut
// into 64-column slices by the product kernels)
int pw_of(int p) { return p <= 16 ? 16 : (p <= 32 ? 32 : (p <= 64 ? 64 : 64 * ((p + 63) / 64))); }

// slice width of the product kernels for staged width pw
#define SW_DISPATCH(pw, ...)      \
  do {                            \
    if ((pw) == 16) {             \
      constexpr int SWV = 16;     \
      __VA_ARGS__;                \
    } else if ((pw) == 32) {      \
      constexpr int SWV = 32;     \
      __VA_ARGS__;                \
    } else {                      \
      constexpr int SWV = 64;     \
      __VA_ARGS__;                \
    }                             \
  } while (0)

void timer_begin(mdsdp_problem P, hipStream_t s, const char* name) {
  if (!P->timer.on) return;
  Timer::Rec r;
  r.name = name;
  if (hipEventCreate(&r.ev0) != hipSuccess) return;
  if (hipEventRecord(r.ev0, s) != hipSuccess) return;
  P->timer.recs.push_back(r);
  P->timer.open.push_back(P->timer.recs.size() - 1);
}
void timer_end(mdsdp_problem P, hipStream_t s) {
  if (!P->timer.on || P->timer.open.empty()) return;
  Timer::Rec& r = P->timer.recs[P->timer.open.back()];
  P->timer.open.pop_back();
  if (hipEventCreate(&r.ev1) != hipSuccess) return;
  (void)hipEventRecord(r.ev1, s);
}

mdsdp_status launch_stage(mdsdp_problem P, int p, const double* Y, const double* U, bool fp32,
                          hipStream_t s) {
  if (!U) P->gram_yy_valid = false;  // an S-pass: Y may have changed
  P->last_p = p;
  P->pw = pw_of(p);
  timer_begin(P, s, "stage");
  unsigned long long* bnd = P->bqp_q > 0 ? nullptr : P->bound;
  if (bnd) MDSDP_HIP(hipMemsetAsync(P->bound, 0, 2 * sizeof(unsigned long long), s));
  const long long cnt = (long long)P->npad * std::min(P->pw, 64);
  if (fp32)
    k_stage<float><<<blocks_for(cnt, 256), 256, 0, s>>>(P->n, p, P->npad, P->pw, Y, U, (float*)P->Yp,
                                                         (float*)P->Up, bnd);
  else
    k_stage<double><<<blocks_for(cnt, 256), 256, 0, s>>>(P->n, p, P->npad, P->pw, Y, U, (double*)P->Yp,
                                                          (double*)P->Up, bnd);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

static mdsdp_status launch_bqp(mdsdp_problem P, bool zmode, bool fp32, hipStream_t s) {
  BqpArgs b{};
  b.q = P->bqp_q;
  b.pw = P->pw;
  b.nkc = (P->last_p + 15) / 16;
  b.off2 = P->bqp_off[2];
  b.off3 = P->bqp_off[3];
  b.off4 = P->bqp_off[4];
  b.Yp = P->Yp;
  b.Up = P->Up;
  b.items4 = P->bqp4_items;
  b.items = P->bqp1_items;
  b.items2 = P->bqp2_items;
  b.p1 = P->bqpP1;
  b.T = P->bqpT;
  b.star = P->bqpStar;
  b.dst = zmode ? (double*)P->ab64 + 1 : (double*)P->cy + 1;
  b.stride = 2;
  b.part = P->gpart + GP_BQP0;
  b.dst32 = P->ab32;
  b.scale32 = -P->sigma;
  const int q = P->bqp_q, n = P->n;
  const unsigned nblkT = (unsigned)((n + 15) / 16), ncolT = (unsigned)((q + 1 + 15) / 16);
  const unsigned nqt = (unsigned)((q + 15) / 16), ntile = nqt * (nqt + 1) / 2;
  const int nS = (int)ntile;
  const long long ntask = (long long)nblkT * ncolT + (long long)nS * STAR_LG;
  // narrow factors (one or two 16-column chunks): the single-pass kernel
  const bool single = b.nkc <= 2;
  const int n1 = single ? P->bqp4_n : P->bqp1_n;
  const unsigned nsum = (unsigned)(single ? n1 : (n1 + 3) / 4) + (unsigned)((ntask + 3) / 4);
  const int rneed = 16 * ((std::max(q - 2, 1) + 15) / 16);  // rows {x, c}, x < c <= q - 2
  const int nb01 = (q + 1 + 3) / 4;
  const unsigned nfin = (unsigned)nb01 + blocks_for(b.off4 - b.off2, 256);
#define PASS2(TT, ZZ, RR, WW, NPP) k_bqp_pass2<TT, ZZ, RR, WW, NPP><<<P->bqp2_n, 256, 0, s>>>(b)
#define PASS2_R(TT, ZZ, NP32, NP64)                                                                         \
  do {                                                                                                      \
    if (P->bqp2_n > 0) {                                                                                    \
      if (rneed <= 64)                                                                                      \
        PASS2(TT, ZZ, 64, 4, (sizeof(TT) == 4 ? NP32 : NP64));                                              \
      else if (rneed <= 128)                                                                                \
        PASS2(TT, ZZ, 128, 4, (sizeof(TT) == 4 ? NP32 : NP64));                                             \
      else if (rneed <= 256)                                                                                \
        PASS2(TT, ZZ, 256, (sizeof(TT) == 4 ? 4 : 2), (sizeof(TT) == 4 ? NP32 : NP64));                     \
      else                                                                                                  \
        PASS2(TT, ZZ, 368, (sizeof(TT) == 4 ? 4 : 2), (sizeof(TT) == 4 ? NP32 : NP64));                     \
    }                                                                                                       \
  } while (0)
#define BQP_LAUNCH(TT, ZZ)                                                                                  \
  do {                                                                                                      \
    timer_begin(P, s, "bqp_sums");                                                                          \
    k_bqp_pass1<TT, ZZ><<<nsum, 256, 0, s>>>(b, n, n1, (int)nblkT, (int)ncolT, nS, single ? 1 : 0);        \
    if (!single) PASS2_R(TT, ZZ, 7, 4);                                                                     \
    timer_end(P, s);                                                                                        \
    timer_begin(P, s, "bqp_fin");                                                                           \
    k_bqpFin<TT, ZZ><<<nfin, 256, 0, s>>>(b, n, (int)nblkT, nb01);                                          \
    timer_end(P, s);                                                                                        \
  } while (0)
  if (!zmode)
    BQP_LAUNCH(double, false);
  else if (fp32)
    BQP_LAUNCH(float, true);
  else
    BQP_LAUNCH(double, true);
#undef BQP_LAUNCH
#undef PASS2_R
#undef PASS2
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_classsum_S(mdsdp_problem P, hipStream_t s) {
  P->a32_valid = false;
  P->a64_valid = false;
  timer_begin(P, s, "classsum_S");
  if (P->bqp_q > 0) {
    mdsdp_status st = launch_bqp(P, false, false, s);
    if (st != MDSDP_OK) return st;
  } else {
    KArgs a = make_args(P);
    k_classsum<double, false><<<seg_grid(P), 256, 0, s>>>(a);
    k_final_S<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->sacc, P->invc, P->Cavg, P->scal, P->cy);
  }
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_classsum_Z(mdsdp_problem P, bool fp32, hipStream_t s) {
  if (P->frozen) {
    // direct-DSDP subproblem: no class sums of Y U^T + U Y^T; zero coefficients once
    if (!P->ycoef_zero) {
      k_zero_ycoef<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->ab64, P->ab32);
      MDSDP_HIP(hipGetLastError());
      P->ycoef_zero = true;
    }
    return MDSDP_OK;
  }
  P->ycoef_zero = false;
  timer_begin(P, s, fp32 ? "classsum_Z32" : "classsum_Z64");
  if (P->bqp_q > 0) {
    mdsdp_status st = launch_bqp(P, true, fp32, s);
    if (st != MDSDP_OK) return st;
  } else {
    KArgs a = make_args(P);
    if (fp32)
      k_classsum<float, true><<<seg_grid(P), 256, 0, s>>>(a);
    else
      k_classsum<double, true><<<seg_grid(P), 256, 0, s>>>(a);
    if (fp32)
      k_final_Z32<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->sacc, P->invc, P->scal, P->sigma, P->ab32);
    else
      k_final_Z<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->sacc, P->invc, P->scal, P->sigma, P->ab64);
  }
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_bty(mdsdp_problem P, hipStream_t s) {
  const int nblk = 64;
  k_bty_part<<<nblk, 256, 0, s>>>(P->bty_range, P->bvec, P->cy, P->gpart + GP_BTY);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

template <typename T, int MODE, int SW>
static mdsdp_status resid_go(mdsdp_problem P, const KArgs& a, unsigned g, hipStream_t s) {
  typedef ResidLds<T, MODE, SW> L;
  static bool attr_set[64] = {};
  const int dev = P->device & 63;
  if (L::bytes > 65536 && !attr_set[dev]) {
    MDSDP_HIP(hipFuncSetAttribute((const void*)k_resid<T, MODE, SW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)L::bytes));
    attr_set[dev] = true;
  }
  k_resid<T, MODE, SW><<<dim3(g, a.nsl), 256, L::bytes, s>>>(a);
  return MDSDP_OK;
}

mdsdp_status launch_resid(mdsdp_problem P, int mode, bool fp32, hipStream_t s) {
  (void)fp32;  // the FP32-tile HVP has its own kernel (launch_hvp32)
  KArgs a = make_args(P);
  const unsigned g = seg_grid(P);
  mdsdp_status st = MDSDP_OK;
  switch (mode) {
    case M_GRAD:
      timer_begin(P, s, "resid_grad");
      SW_DISPATCH(P->pw, st = (resid_go<double, M_GRAD, SWV>(P, a, g, s)));
      break;
    case M_MULT:
      timer_begin(P, s, "resid_mult");
      if (a.nsl > 1) {
        // sliced update: every slice reads the old Xt, slice 0 writes the new one
        if (!P->Xt2) MDSDP_HIP(hipMalloc((void**)&P->Xt2, (size_t)P->nslots * sizeof(double)));
        a.Xt_out = P->Xt2;
      }
      SW_DISPATCH(P->pw, st = (resid_go<double, M_MULT, SWV>(P, a, g, s)));
      if (a.nsl > 1) std::swap(P->Xt, P->Xt2);
      break;
    case M_XMV:
      timer_begin(P, s, "resid_xmv");
      SW_DISPATCH(P->pw, st = (resid_go<double, M_XMV, SWV>(P, a, g, s)));
      break;
    default:
      if (!P->a64_valid) {
        k_make_a64<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->cy, P->sigma, P->ab64);
        P->a64_valid = true;
      }
      timer_begin(P, s, "resid_hvp64");
      SW_DISPATCH(P->pw, st = (resid_go<double, M_HVP, SWV>(P, a, g, s)));
  }
  timer_end(P, s);
  if (st != MDSDP_OK) return st;
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

template <int SW>
static mdsdp_status hvp32_go(mdsdp_problem P, const H32Args& a, unsigned g, hipStream_t s) {
  typedef H32Lds<SW> L;
  static bool attr_set[64] = {};
  const int dev = P->device & 63;
  if (L::bytes > 65536 && !attr_set[dev]) {
    MDSDP_HIP(hipFuncSetAttribute((const void*)k_hvp32<SW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)L::bytes));
    attr_set[dev] = true;
  }
  k_hvp32<SW><<<g, 256, L::bytes, s>>>(a);
  return MDSDP_OK;
}

mdsdp_status launch_hvp32(mdsdp_problem P, hipStream_t s) {
  if (!P->a32_valid) {
    k_make_a32<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->cy, P->sigma, P->ab32);
    P->a32_valid = true;
  }
  H32Args a{};
  a.cls32 = P->cls32;
  a.Xt32 = P->Xt32;
  a.Ct = P->Ct;
  a.segs = P->segs;
  a.nseg = P->nseg;
  a.seg_per_xcd = (P->nseg + 7) / 8;
  a.pw = P->pw;
  const int sw = std::min(P->pw, 64);
  a.nsl = P->pw / sw;
  a.Yp = (const float*)P->Yp;
  a.Up = (const float*)P->Up;
  a.ab32 = P->ab32;
  a.sigma = (float)P->sigma;
  a.rowpart = (float*)P->rowpart;
  a.colpart = (float*)P->colpart;
  const unsigned g = (unsigned)(8 * a.seg_per_xcd * a.nsl);
  mdsdp_status st = MDSDP_OK;
  timer_begin(P, s, "resid_hvp32");
  if (sw == 16)
    st = hvp32_go<16>(P, a, g, s);
  else if (sw == 32)
    st = hvp32_go<32>(P, a, g, s);
  else
    st = hvp32_go<64>(P, a, g, s);
  timer_end(P, s);
  if (st != MDSDP_OK) return st;
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

static RowArgs row_args(mdsdp_problem P, int p) {
  RowArgs ra;
  ra.n = P->n;
  ra.p = p;
  ra.pw = P->pw;
  ra.nb = P->nb;
  ra.nseg = P->nseg;
  ra.seg_start = P->seg_start;
  ra.rowpart = P->rowpart;
  ra.colpart = P->colpart;
  return ra;
}

// Wide factors (p > 64): the Gram matrices and the low-rank HVP term are
// plain FP64 GEMMs, done by the two MFMA kernels below (no vendor library).
//
// k_gemm_tn_part: partial[c] = A^T B over the rows of chunk c (A, B row-major
// n x p); one wave per 64 x 64 output macro-block and chunk, a 4 x 4 grid of
// 16 x 16 MFMA tiles fed by one A and one B fragment of 4 rows per tile row /
// column; partial[c] is row-major with pitch pw inside the Gram partial layout
// (stride 2 pw^2 between chunks), added in a fixed order by k_gram_final.
__global__ __launch_bounds__(256) void k_gemm_tn_part(int n, int p, int pw, int rows, int nmb,
                                                      const double* __restrict__ A, const double* __restrict__ B,
                                                      double* __restrict__ part) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int chunk = blockIdx.y;
  if (wid >= nmb * nmb) return;
  const int I0 = (wid / nmb) * 64, J0 = (wid % nmb) * 64;
  const int r0 = chunk * rows, r1 = min(n, r0 + rows);
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  for (int r = r0; r < r1; r += 4) {
    const int rr = r + lk;
    const bool rin = rr < r1;
    double fa[4], fb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int ci = I0 + 16 * a + li, cj = J0 + 16 * a + li;
      fa[a] = (rin && ci < p) ? A[(size_t)rr * p + ci] : 0.0;
      fb[a] = (rin && cj < p) ? B[(size_t)rr * p + cj] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = mfma(fa[a], fb[b], acc[a][b]);
  }
  double* out = part + (size_t)chunk * 2 * pw * pw;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = I0 + 16 * a + drow<double>(lk, v), j = J0 + 16 * b + li;
        if (i < pw && j < pw) out[(size_t)i * pw + j] = acc[a][b][v];
      }
}

// k_lowrank: LR = Y (Y^T U + U^T Y) + U (Y^T Y) (n x p row-major), with
// Y^T Y at gram and Y^T U at gram + GRAM_U (pitch gp): one wave per 16 rows
// and 64 output columns, contraction over 2p (the Y part, then the U part).
__global__ __launch_bounds__(256) void k_lowrank(int n, int p, int gp, const double* __restrict__ Y,
                                                 const double* __restrict__ U, const double* __restrict__ gram,
                                                 double* __restrict__ LR) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int R0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16, K0 = blockIdx.y * 64;
  if (R0 >= n) return;
  const double* YtY = gram;
  const double* YtU = gram + GRAM_U;
  v4d acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = v4d{0, 0, 0, 0};
  const int row = R0 + li;
  for (int part = 0; part < 2; ++part) {
    const double* F = part == 0 ? Y : U;
    for (int t0 = 0; t0 < p; t0 += 4) {
      const int t = t0 + lk;
      const double fa = (row < n && t < p) ? F[(size_t)row * p + t] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = K0 + 16 * c + li;
        double fb = 0.0;
        if (t < p && k < p)
          fb = part == 0 ? YtU[(size_t)k * gp + t] + YtU[(size_t)t * gp + k] : YtY[(size_t)t * gp + k];
        acc[c] = mfma(fa, fb, acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = R0 + drow<double>(lk, v), k = K0 + 16 * c + li;
      if (r < n && k < p) LR[(size_t)r * p + k] = acc[c][v];
    }
}

// Gram partials of A^T B for wide factors: the rows in nch chunks (one chunk's
// product per partial, offset `half` in the Gram partial layout)
static mdsdp_status gram_wide(mdsdp_problem P, int p, int pw, int& nch, const double* A, const double* B,
                              size_t half, hipStream_t s) {
  const int n = P->n;
  int rows = (n + nch - 1) / nch;
  rows = (rows + 3) & ~3;
  nch = (n + rows - 1) / rows;
  const int nmb = (p + 63) / 64;
  k_gemm_tn_part<<<dim3(blocks_for((long long)nmb * nmb, 4), nch), 256, 0, s>>>(n, p, pw, rows, nmb, A, B,
                                                                                 P->gpart + GP_GRAM + half);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_gram(mdsdp_problem P, int p, const double* Y, const double* U, hipStream_t s,
                         bool with_yy) {
  // the Gram width follows p itself (not the last staged width)
  const int gpw = pw_of(p);
  if (gpw > 64) {
    timer_begin(P, s, "gram");
    P->gram_pw = gpw;
    const size_t pw2 = (size_t)gpw * gpw;
    int nch = (int)std::max<size_t>(1, std::min<size_t>({64, GRAM_PART_MAX / (2 * pw2),
                                                               (size_t)(P->n + 63) / 64}));
    mdsdp_status st = MDSDP_OK;
    if (with_yy) st = gram_wide(P, p, gpw, nch, Y, Y, 0, s);
    if (st == MDSDP_OK) st = gram_wide(P, p, gpw, nch, Y, U, pw2, s);
    if (st != MDSDP_OK) return st;
    const int len = (int)(2 * pw2), e0 = with_yy ? 0 : (int)pw2;
    k_gram_final<<<blocks_for(len - e0, 256), 256, 0, s>>>(nch, len, e0, P->gpart + GP_GRAM, P->gram, gpw, 1);
    timer_end(P, s);
    MDSDP_HIP(hipGetLastError());
    return MDSDP_OK;
  }
  // row blocks: short dependent load/MFMA chains per wave, at most 256
  // partials per Gram element for the final sum, within the partial buffer
  const GramSplit GS(gpw);
  const int nblk = (int)std::max<size_t>(
      1, std::min<size_t>({(size_t)(256 / GS.RS), (size_t)(P->n + 15) / 16,
                           GRAM_PART_MAX / ((size_t)GS.RS * 2 * gpw * gpw)}));
  timer_begin(P, s, "gram");
  P->gram_pw = gpw;
  const int len = 2 * gpw * gpw, e0 = with_yy ? 0 : gpw * gpw;
  const int nparts = nblk * GS.RS;
  k_gram_part<<<dim3(nblk, GS.NGRP), 256, 0, s>>>(P->n, p, gpw, with_yy ? 1 : 0, Y, U, P->gpart + GP_GRAM);
  k_gram_final<<<(len - e0 + 3) / 4, 256, 0, s>>>(nparts, len, e0, P->gpart + GP_GRAM, P->gram, gpw, 0);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_grad(mdsdp_problem P, int p, const double* Y, double* egrad, double* rgrad,
                                  double* f, hipStream_t s) {
  RowArgs ra = row_args(P, p);
  timer_begin(P, s, "row_grad");
  const unsigned nblk = blocks_for((long long)P->n * 64, 256);  // L * SPL = 64 lanes per row
  const int rm = P->pw <= 64 ? 1 : P->pw / 64;
  if (rm <= 1)
    k_row_grad<1><<<nblk, 256, 0, s>>>(ra, Y, egrad, rgrad, P->zvec);
  else if (rm <= 2)
    k_row_grad<2><<<nblk, 256, 0, s>>>(ra, Y, egrad, rgrad, P->zvec);
  else if (rm <= 4)
    k_row_grad<4><<<nblk, 256, 0, s>>>(ra, Y, egrad, rgrad, P->zvec);
  else
    k_row_grad<8><<<nblk, 256, 0, s>>>(ra, Y, egrad, rgrad, P->zvec);
  k_scalars<<<1, 256, 0, s>>>(M_GRAD, P->wgpart, P->nseg, nullptr, 0, P->gpart + GP_BTY, 64, P->sigma, P->scal, f,
                              nullptr, P->frozen ? 1 : 0);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_hvp(mdsdp_problem P, int p, bool fp32, const double* Y, const double* U,
                                 double* HU, int riem, hipStream_t s, double* dotpart, double* dot_out) {
  RowArgs ra = row_args(P, p);
  timer_begin(P, s, "row_hvp");
  const unsigned nblk = blocks_for((long long)P->n * 64, 256);  // L * SPL = 64 lanes per row
  const double* lr = nullptr;
  if (p > 64) {
    // LR = Y (Y^T U + U^T Y) + U (Y^T Y) by an MFMA kernel (k_lowrank)
    const int n = P->n;
    k_lowrank<<<dim3(blocks_for(n, 64), (p + 63) / 64), 256, 0, s>>>(n, p, P->gram_pw, Y, U, P->gram, P->lrbuf);
    MDSDP_HIP(hipGetLastError());
    lr = P->lrbuf;
  }
  const int rm = P->pw <= 64 ? 1 : P->pw / 64;
#define ROW_HVP(TT, RMV) \
  k_row_hvp<TT, RMV><<<nblk, 256, 0, s>>>(ra, Y, U, P->gram, lr, P->zvec, P->sigma, riem, HU, dot_out ? dotpart : nullptr, \
                                             P->scal + SC_NONFIN)
  if (fp32) {
    if (rm <= 1)
      ROW_HVP(float, 1);
    else if (rm <= 2)
      ROW_HVP(float, 2);
    else if (rm <= 4)
      ROW_HVP(float, 4);
    else
      ROW_HVP(float, 8);
  } else {
    if (rm <= 1)
      ROW_HVP(double, 1);
    else if (rm <= 2)
      ROW_HVP(double, 2);
    else if (rm <= 4)
      ROW_HVP(double, 4);
    else
      ROW_HVP(double, 8);
  }
#undef ROW_HVP
  if (dot_out) k_sum_partials<<<1, 256, 0, s>>>((int)nblk, dotpart, dot_out);
  timer_end(P, s);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_mult(mdsdp_problem P, int p, const double* Y, double* z, double* kkt,
                                  hipStream_t s) {
  RowArgs ra = row_args(P, p);
  const unsigned nblk = blocks_for((long long)P->n * std::min(P->pw, 64), 256);
  k_row_mult<<<nblk, 256, 0, s>>>(ra, Y, P->zmult, z, P->zpart);
  k_scalars<<<1, 256, 0, s>>>(M_MULT, P->wgpart, P->nseg, P->zpart, (int)nblk, P->gpart + GP_BTY, 64, P->sigma,
                              P->scal, nullptr, kkt, 0);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rowfinal_xmv(mdsdp_problem P, int k, const double* V, double* XV, hipStream_t s) {
  RowArgs ra = row_args(P, k);
  k_row_xmv<<<blocks_for((long long)P->n * std::min(P->pw, 64), 256), 256, 0, s>>>(ra, V, P->zmult, XV);
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
  k_y_export<<<blocks_for(P->m, 256), 256, 0, s>>>(P->m, P->cy, y);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_set_dense(mdsdp_problem P, const double* X, hipStream_t s) {
  k_set_dense<<<blocks_for(P->nslots, 256), 256, 0, s>>>(P->n, P->nb, P->nslots, X, P->Xt, P->Xt32,
                                                         P->scal + SC_NONFIN);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_get_dense(mdsdp_problem P, double* X, bool add_D, hipStream_t s) {
  k_get_dense<<<blocks_for(P->nslots, 256), 256, 0, s>>>(P->n, P->nb, P->nslots, P->Xt, P->cls, P->cy,
                                                         add_D ? 1 : 0, X);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_dots(const DotPtrs& dp, int npairs, long long len, double* out_dev, double* part, int nblk,
                      hipStream_t s) {
  k_dots<<<nblk, 256, 0, s>>>(dp, npairs, len, part);
  k_dots_final<<<npairs, 256, 0, s>>>(npairs, nblk, part, out_dev);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_lincomb(long long len, double alpha, const double* x, double beta, const double* y, double* out,
                         hipStream_t s) {
  k_lincomb<<<blocks_for(len, 256), 256, 0, s>>>(len, alpha, x, beta, y, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_tcg_update(int n, int p, const double* Y, const double* sc_c, double* sc_n, const TcgIter& c,
                               const TcgIter& nx, double* part, hipStream_t s) {
  int L = 1;
  while (L < p && L < 64) L <<= 1;
  const int rm = (p + L - 1) / L;
  const unsigned nb = blocks_for((long long)n * L, 256);
#define TCG_GO(RMV)                                                                                          \
  do {                                                                                                       \
    k_tcg_update1<RMV><<<nb, 256, 0, s>>>(n, p, L, Y, sc_c, c.eta, c.Heta, c.r, c.d, c.Hd, nx.eta, nx.Heta,  \
                                          nx.r, part);                                                       \
    k_tcg_update2<RMV><<<nb, 256, 0, s>>>(n, p, L, Y, (int)nb, part, sc_c, sc_n, nx.r, c.d, nx.d);           \
  } while (0)
  if (rm <= 1)
    TCG_GO(1);
  else if (rm <= 2)
    TCG_GO(2);
  else if (rm <= 4)
    TCG_GO(4);
  else
    TCG_GO(8);
#undef TCG_GO
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_vt_w(int n, int k, const double* V, const double* w, double* h, hipStream_t s) {
  k_vt_w<<<k, 256, 0, s>>>(n, V, w, h);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_rightmul(int n, int p, int q, const double* Yin, const double* M, bool normalize,
                             double* Yout, hipStream_t s) {
  k_rightmul<<<blocks_for(n, 256), 256, 0, s>>>(n, p, q, Yin, M, normalize ? 1 : 0, Yout);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_sign_col(int n, int p, const double* Yin, const double* v, double* out, hipStream_t s) {
  k_sign_col<<<blocks_for(n, 256), 256, 0, s>>>(n, p, Yin, v, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_set_col(int n, int p, int col, const double* v, double* U, hipStream_t s, bool zero_rest) {
  k_set_col<<<blocks_for(n, 256), 256, 0, s>>>(n, p, col, v, U, zero_rest ? 1 : 0);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_gemv_sub(int n, int k, const double* V, const double* h, double* w, hipStream_t s) {
  k_gemv_sub<<<blocks_for(n, 256), 256, 0, s>>>(n, k, V, h, w);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

// Lanczos step on the device: alpha_j = h[j] + h2[j] (the two reorthogonal-
// isation passes), beta_j^2 = <w, w>; v_{j+1} = w / beta_j (zeros when beta_j
// vanishes: the host stops at that step)
__global__ __launch_bounds__(256) void k_lanczos_step(int n, int j, const double* __restrict__ h,
                                                      const double* __restrict__ h2, const double* __restrict__ nrm2,
                                                      double* __restrict__ alpha, double* __restrict__ beta2,
                                                      const double* __restrict__ w, double* __restrict__ vnext) {
  const double b2 = *nrm2;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    alpha[j] = h[j] + h2[j];
    beta2[j] = b2;
  }
  if (!vnext) return;
  const double inv = b2 > 0.0 ? 1.0 / sqrt(b2) : 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) vnext[i] = w[i] * inv;
}

mdsdp_status launch_lanczos_step(int n, int j, const double* h, const double* h2, const double* nrm2, double* alpha,
                                 double* beta2, const double* w, double* vnext, bool write_next, hipStream_t s) {
  k_lanczos_step<<<blocks_for(n, 256), 256, 0, s>>>(n, j, h, h2, nrm2, alpha, beta2, w, write_next ? vnext : nullptr);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_transpose(int n, int r, const double* Q, double* QT, hipStream_t s) {
  k_transpose<<<dim3(blocks_for(n, 16), blocks_for(r, 16)), 256, 0, s>>>(n, r, Q, QT);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status launch_deflate(int n, int r, const double* QT, double* w, double* c, hipStream_t s) {
  // w <- (I - Q Q^T) w with QT = Q^T (r x n), twice (classical Gram-Schmidt
  // with one refinement)
  for (int pass = 0; pass < 2; ++pass) {
    mdsdp_status st = launch_vt_w(n, r, QT, w, c, s);
    if (st == MDSDP_OK) st = launch_gemv_sub(n, r, QT, c, w, s);
    if (st != MDSDP_OK) return st;
  }
  return MDSDP_OK;
}

mdsdp_status launch_gemv(int n, int k, const double* V, const double* sv, double* out, hipStream_t s) {
  k_gemv<<<blocks_for(n, 256), 256, 0, s>>>(n, k, V, sv, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

mdsdp_status vec_fill(long long len, double v, double* out, hipStream_t s) {
  k_fill<<<blocks_for(len, 256), 256, 0, s>>>(len, v, out);
  MDSDP_HIP(hipGetLastError());
  return MDSDP_OK;
}

// Fixed device scratch of the entry points that allocate nothing: one copy
// per GPU, held until the process ends.  Host code must not pass `scratch`
// itself to a kernel (in host code the name is a host-side stand-in): the
// device address comes from hipGetSymbolAddress, fetched once per device with
// that device current, and is cached here.
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

mdsdp_status scratch_buffer(double** out) {
  static std::mutex mu;
  static double* ptrs[MAX_DEVICES] = {};
  int dev = 0;
  MDSDP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device index out of range for the fixed scratch");
    return MDSDP_EINVAL;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    ptrs[dev] = (double*)ptr;
  }
  *out = ptrs[dev];
  return MDSDP_OK;
}



}  // namespace mdsdp
