// Internal definitions of the ManiDSDP gfx950 library.
//
// Device layout of the n x n symmetric operands (class map, multiplier Xt,
// optional C).  Only the upper triangle is stored, cut into 64 x 64 tiles
// (I, J), I <= J, enumerated column-block by column-block:
//     tile(I, J) = J (J + 1) / 2 + I.
// Each tile holds 4096 slots: 16 sub-blocks of 16 x 16 in row-major sub-block
// order, each sub-block row-major.  Slot of entry (r, c) of tile (I, J):
//     tile * 4096 + ((r % 64) / 16 * 4 + (c % 64) / 16) * 256 + (r % 16) * 16 + c % 16.
// Off-diagonal tiles (I < J) hold entries with r < c (weight 2 in class sums,
// two-sided in products).  Diagonal tiles (I == J) hold the full symmetric
// 64 x 64 block (both triangles, weight 1, one-sided in products).  Slots with
// r >= n or c >= n are padding: class word -1, value 0.
//
// Class word of a slot: bit 31 set = padding; bits 0..29 = class id; bit 30 =
// "owner" flag, set on exactly one slot of every class (the first in slot
// order), used to clear double-buffered accumulators without a separate pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/manidsdp.h"

namespace mdsdp {

constexpr int TS = 64;          // tile side
constexpr int SB = 16;          // MFMA sub-block side
constexpr int PMAX = 512;       // largest factor width (p <= 512)
constexpr int GRAM_U = PMAX * PMAX;  // offset of Y^T U in the Gram buffer
constexpr int HBUF_LEN = 64 + PMAX * PMAX;  // pinned read-back buffer (doubles)
constexpr int TSLOTS = TS * TS;  // slots per tile
constexpr int LP = 17;          // LDS row pitch (elements) for 16-wide rows
constexpr int STAR_LG = 32;     // residue classes of l in the degree-2 BQP contraction
// class word of a slot: bit 31 padding slot (outside the matrix), bit 30
// first slot of its class, bit 29 coefficient -1 in A_gamma, bit 28 no class
// (coefficient 0: A*(y) is zero there), bits 0..27 the class id
// FP32-tile order of a slot: inside each 16 x 16 sub-block the entry
// (r, c) moves from r * 16 + c to c * 16 + r, so that the four entries an
// FP32 MFMA result lane holds (rows 4 lk .. 4 lk + 3 of column li) are
// consecutive and load as one 16-byte vector
__host__ __device__ inline size_t slot32(size_t s) {
  const size_t e = s & 255;
  return (s & ~(size_t)255) | ((e & 15) << 4) | (e >> 4);
}
constexpr uint32_t CLS_MASK = 0x0FFFFFFFu;
constexpr uint32_t OWNER_BIT = 0x40000000u;
constexpr uint32_t NEG_BIT = 0x20000000u;
constexpr uint32_t FREE_BIT = 0x10000000u;

// Gram partials: gram_blocks(pw) row blocks, each 2 pw^2 doubles (at most
// 4 blocks of 2 x 512 x 512, 2 x 32 x 64 x 64 or 32 x 4 x 2 x 16 x 16)
inline int gram_blocks(int pw) { return pw <= 64 ? 32 : (pw <= 128 ? 16 : (pw <= 256 ? 8 : 4)); }
constexpr size_t GRAM_PART_MAX = 4 * 2 * (size_t)PMAX * PMAX;
// carve of the `gpart` scratch (doubles): Gram partials, b^T y partials,
// degree-0 BQP partials, host-built p x p matrix
constexpr size_t GP_GRAM = 0;
constexpr size_t GP_BTY = GRAM_PART_MAX;
constexpr size_t GP_BQP0 = GP_BTY + 64;
constexpr size_t GP_M = GP_BQP0 + 4096;
constexpr size_t GP_SIZE = GP_M + PMAX * PMAX;

struct Seg {
  int J, I0, I1;  // column block J, row blocks I0..I1 inclusive
};

enum Mode { M_GRAD = 0, M_MULT = 1, M_XMV = 2, M_HVP = 3 };

struct Timer {
  struct Rec {
    std::string name;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<size_t> open;  // indices of records whose end is pending
};

}  // namespace mdsdp

struct mdsdp_problem_s {
  int n = 0;
  long long m = 0;
  int nb = 0;          // number of 64-blocks
  int ntiles = 0;
  long long nslots = 0;
  int nseg = 0;
  int npad = 0;        // nb * 64
  long long kmax = 0;  // largest class (ordered entries)
  double sigma = 1.0;
  double normb = 0.0, normC = 0.0;
  bool hasC = false;
  int device = 0;

  // device arrays
  uint32_t* cls = nullptr;      // nslots class words
  double* Xt = nullptr;         // nslots
  double* Xt2 = nullptr;        // nslots, second multiplier buffer of the sliced update (allocated on first use)
  float* Xt32 = nullptr;        // nslots (FP32 shadow, refreshed on every Xt write), FP32-tile order
  uint32_t* cls32 = nullptr;    // nslots: the class words again, in FP32-tile order
  double* Ct = nullptr;         // nslots or null
  mdsdp::Seg* segs = nullptr;   // nseg
  int* seg_start = nullptr;     // nb + 1: segments of column block J are seg_start[J]..seg_start[J+1]-1
  double2* cy = nullptr;        // m: {D_gamma, y_gamma} (y = class average of Z at the last S-pass)
  double2* ab64 = nullptr;      // m: FP64 HVP class coefficients {D - sigma y (of U), -sigma y' (of Y)}
  bool a64_valid = false;       // ab64[].x matches the current y and sigma
  float2* ab32 = nullptr;       // m: FP32-tile HVP class coefficients {D - sigma y (of U), -sigma y' (of Y)}
  bool a32_valid = false;       // ab32[].x matches the current y and sigma
  double* invc = nullptr;       // m: 1 / |gamma|
  double* bvec = nullptr;       // m: b
  double* Cavg = nullptr;       // m or null: A(C)_gamma / |gamma|
  long long* sacc = nullptr;    // m: fixed-point accumulator of the generic class-sum pass
  long long bty_range = 0;      // classes [0, bty_range) may have b != 0
  // structured BQP path (colex basis and class order), q = 0 when generic
  int bqp_q = 0;
  long long bqp_off[6] = {0, 0, 0, 0, 0, 0};
  int4* bqp4_items = nullptr;   // (c, d0, a0, b0) work items of the single-pass degree-4 kernel
  int bqp4_n = 0;
  int4* bqp1_items = nullptr;   // (d, c0, t0, 0) work items of degree-4 pass 1
  int bqp1_n = 0;
  int2* bqp2_items = nullptr;   // (c, d) work items of degree-4 pass 2
  int bqp2_n = 0;
  double* bqpP1 = nullptr;      // C(q, 4) pass-1 results
  double* bqpT = nullptr;       // n x (q + 1) table of the degree 0..3 pass
  double* bqpStar = nullptr;    // STAR_LG x q x q partials of the degree-2 contraction
  // staging / workspace
  void* Yp = nullptr;           // npad x 16 (double or float)
  void* Up = nullptr;
  double* zvec = nullptr;       // n: diag(G S) at the last cost/grad point
  double* zmult = nullptr;      // n: diag((Xt + D) S) at the last multiplier update
  double* rowpart = nullptr;    // ntiles * 64 * 16
  double* colpart = nullptr;    // nseg * 64 * 16
  double* wgpart = nullptr;     // nseg * 4 scalar partials
  double* zpart = nullptr;      // row-block partials of sum z
  double* gram = nullptr;       // 512: Y^T Y, Y^T U
  double* gpart = nullptr;
  double* scal = nullptr;       // device scalars (SC_*), [7] = S-sum scale, [8] = Z-sum scale
  unsigned long long* bound = nullptr;  // max row norms of Y, U (bit patterns)
  int last_p = 0;
  int pw = 16;         // staged factor width for last_p: 16, 32 or 64
  int gram_pw = 16;    // row pitch of the last Gram matrices written to `gram`
  bool gram_yy_valid = false;  // `gram` holds Y^T Y of the current Y (set by the HVP, cleared by S-passes)
  int gram_yy_p = 0;           // factor width of that Y^T Y
  int last_hvp_prec = -1;      // tile precision of the last mdsdp_hvp call
  double* lrbuf = nullptr;     // n x PMAX: low-rank part of the HVP for p > 64
  bool frozen = false;        // direct-DSDP (ADMM) subproblem: stale y, Hessian sigma I in S
  bool ycoef_zero = false;    // HVP class coefficients of Y zeroed (frozen mode)
  // solver / Lanczos workspace
  double* dotpart = nullptr;
  const double** dotptr = nullptr;  // unused (kept for layout stability)
  double* hbuf = nullptr;       // pinned host buffer for scalar read-backs
  int dot_nblk = 0;
  double* work = nullptr;       // n x 16 x 8 doubles of solver scratch
  double* lz_V = nullptr;       // Lanczos basis, n x lz_cap
  int lz_cap = 0;
  double* lz_w = nullptr;
  double* lz_h = nullptr;
  double* lz_hpart = nullptr;
  mdsdp::Timer timer;
};

// device scalar slots
enum {
  SC_F = 0,        // cost
  SC_BTY = 1,      // b^T y
  SC_XZ = 2,       // sum w Xt Z
  SC_R2 = 3,       // sum w r^2
  SC_SUMZ = 4,     // sum z
  SC_CXZ = 5,      // <C, Xt + D> (for eta_g when C != 0)
  SC_NONFIN = 6,   // sticky non-finite flag
  SC_SCALE_S = 7,  // fixed-point scale of the latest S-sums
  SC_SCALE_Z = 8,  // fixed-point scale of the latest Z'-sums
  SC_BTYP = 9,     // b^T y partials (up to 8 slots at 40..47 are not used)
  SC_FOUT = 16,    // solver: cost read-back
  SC_DOTS = 17,    // solver: dot products read-back (8 slots)
  SC_KKT = 25,     // solver: kkt read-back (4 slots)
  SC_COUNT = 32
};

namespace mdsdp {

void set_error(const std::string& msg);
mdsdp_status hip_fail(hipError_t e, const char* what);

#define MDSDP_HIP(call)                                          \
  do {                                                           \
    hipError_t e__ = (call);                                     \
    if (e__ != hipSuccess) return ::mdsdp::hip_fail(e__, #call); \
  } while (0)

// kernel launchers (kernels.hip)
int pw_of(int p);
mdsdp_status launch_stage(mdsdp_problem P, int p, const double* Y, const double* U, bool fp32,
                          hipStream_t s);
mdsdp_status launch_classsum_S(mdsdp_problem P, hipStream_t s);
mdsdp_status launch_classsum_Z(mdsdp_problem P, bool fp32, hipStream_t s);
mdsdp_status launch_bty(mdsdp_problem P, hipStream_t s);
mdsdp_status launch_resid(mdsdp_problem P, int mode, bool fp32, hipStream_t s);
mdsdp_status launch_hvp32(mdsdp_problem P, hipStream_t s);
mdsdp_status launch_gram(mdsdp_problem P, int p, const double* Y, const double* U,
                         hipStream_t s, bool with_yy = true);
mdsdp_status launch_rowfinal_grad(mdsdp_problem P, int p, const double* Y, double* egrad,
                                  double* rgrad, double* f, hipStream_t s);
// dot_out (nullable): <U, HU> written there (block partials in dotpart, at
// least n / 4 + 1 doubles)
mdsdp_status launch_rowfinal_hvp(mdsdp_problem P, int p, bool fp32, const double* Y,
                                 const double* U, double* HU, int riem, hipStream_t s,
                                 double* dotpart = nullptr, double* dot_out = nullptr);
// the HVP of mdsdp_hvp, optionally with <U, HU> left on the device
mdsdp_status hvp_impl(mdsdp_problem P, int p, int prec, const double* Y, const double* U, double* HU,
                      int riem, hipStream_t s, double* dotpart = nullptr, double* dot_out = nullptr);
mdsdp_status launch_rowfinal_mult(mdsdp_problem P, int p, const double* Y, double* z,
                                  double* kkt, hipStream_t s);
mdsdp_status launch_rowfinal_xmv(mdsdp_problem P, int k, const double* V, double* XV,
                                 hipStream_t s);
mdsdp_status launch_retract(int n, int p, const double* Y, const double* V, double t,
                            double* Yout, hipStream_t s);
mdsdp_status launch_project(int n, int p, const double* Y, const double* U, double* out,
                            hipStream_t s);
mdsdp_status launch_y_export(mdsdp_problem P, double* y, hipStream_t s);
mdsdp_status launch_set_dense(mdsdp_problem P, const double* Xdense, hipStream_t s);
mdsdp_status launch_get_dense(mdsdp_problem P, double* Xdense, bool add_D, hipStream_t s);

// vector kernels used by the solver (kernels.hip)
struct DotPtrs {
  const double* a[8];
  const double* b[8];
};
mdsdp_status vec_dots(const DotPtrs& dp, int npairs, long long len, double* out_dev, double* part, int nblk,
                      hipStream_t s);
mdsdp_status vec_lincomb(long long len, double alpha, const double* x, double beta,
                         const double* y, double* out, hipStream_t s);
mdsdp_status vec_fill(long long len, double v, double* out, hipStream_t s);
// one truncated-CG iterate (n x p each)
struct TcgIter {
  double *eta, *Heta, *r, *d, *Hd;
};
// c -> nx with alpha = sc_c[0] / sc_c[1] (rr, <d, Hd> of c); writes
// sc_n[0] = ||r_nx||^2 (part: n / 4 + 1 doubles of scratch)
mdsdp_status launch_tcg_update(int n, int p, const double* Y, const double* sc_c, double* sc_n, const TcgIter& c,
                               const TcgIter& nx, double* part, hipStream_t s);
mdsdp_status launch_vt_w(int n, int k, const double* V, const double* w, double* h, hipStream_t s);
mdsdp_status launch_rightmul(int n, int p, int q, const double* Yin, const double* M, bool normalize,
                             double* Yout, hipStream_t s);
mdsdp_status launch_sign_col(int n, int p, const double* Yin, const double* v, double* out, hipStream_t s);
mdsdp_status launch_set_col(int n, int p, int col, const double* v, double* U, hipStream_t s,
                           bool zero_rest = true);
mdsdp_status launch_gemv_sub(int n, int k, const double* V, const double* h, double* w, hipStream_t s);
mdsdp_status launch_gemv(int n, int k, const double* V, const double* sv, double* out, hipStream_t s);
// device address of this GPU's fixed scratch (SCRATCH_DOUBLES doubles), for
// the entry points that allocate nothing; fetched once per device
constexpr long long SCRATCH_DOUBLES = 4ll << 20;  // 32 MiB
constexpr int MAX_DEVICES = 64;
mdsdp_status scratch_buffer(double** out);
// one Lanczos step's scalars and normalisation on the device (see solver.cpp)
mdsdp_status launch_lanczos_step(int n, int j, const double* h, const double* h2, const double* nrm2, double* alpha,
                                 double* beta2, const double* w, double* vnext, bool write_next, hipStream_t s);
// QT = Q^T (Q row-major n x r, QT row-major r x n)
mdsdp_status launch_transpose(int n, int r, const double* Q, double* QT, hipStream_t s);
// w <- (I - Q Q^T) w for Q with orthonormal columns, given as QT = Q^T (r x n);
// c: r doubles of scratch
mdsdp_status launch_deflate(int n, int r, const double* QT, double* w, double* c, hipStream_t s);

void timer_begin(mdsdp_problem P, hipStream_t s, const char* name);
void timer_end(mdsdp_problem P, hipStream_t s);

}  // namespace mdsdp
