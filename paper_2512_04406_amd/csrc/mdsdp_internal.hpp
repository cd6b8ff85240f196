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
constexpr int PP = 16;          // padded factor width (p <= 16)
constexpr int TSLOTS = TS * TS;  // slots per tile
constexpr int LP = 17;          // LDS row pitch (elements) for 16-wide rows
constexpr uint32_t CLS_MASK = 0x3FFFFFFFu;
constexpr uint32_t OWNER_BIT = 0x40000000u;

struct Seg {
  int J, I0, I1;  // column block J, row blocks I0..I1 inclusive
};

enum Mode { M_GRAD = 0, M_MULT = 1, M_XMV = 2, M_HVP = 3 };

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<std::string> names;
  std::vector<double> ms;
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
  float* Xt32 = nullptr;        // nslots (FP32 shadow, refreshed on every Xt write)
  double* Ct = nullptr;         // nslots or null
  mdsdp::Seg* segs = nullptr;   // nseg
  int* seg_start = nullptr;     // nb + 1: segments of column block J are seg_start[J]..seg_start[J+1]-1
  double2* cinf = nullptr;      // m: {D_gamma, 1/|gamma|}
  double* Cavg = nullptr;       // m or null: A(C)_gamma / |gamma|
  long long* sS[2] = {nullptr, nullptr};  // fixed-point class sums of Y Y^T (double-buffered)
  long long* sZ[2] = {nullptr, nullptr};  // fixed-point class sums of Y U^T + U Y^T
  int spar = 0, zpar = 0;       // buffer holding the latest sums
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
  // solver / Lanczos workspace
  double* dotpart = nullptr;
  const double** dotptr = nullptr;  // device array of pointers for k_dots
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
  SC_COUNT = 16
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
mdsdp_status launch_stage(mdsdp_problem P, int p, const double* Y, const double* U, bool fp32,
                          hipStream_t s);
mdsdp_status launch_classsum_S(mdsdp_problem P, hipStream_t s);
mdsdp_status launch_classsum_Z(mdsdp_problem P, bool fp32, hipStream_t s);
mdsdp_status launch_resid(mdsdp_problem P, int mode, bool fp32, hipStream_t s);
mdsdp_status launch_gram(mdsdp_problem P, int p, const double* Y, const double* U,
                         hipStream_t s);
mdsdp_status launch_rowfinal_grad(mdsdp_problem P, int p, const double* Y, double* egrad,
                                  double* rgrad, double* f, hipStream_t s);
mdsdp_status launch_rowfinal_hvp(mdsdp_problem P, int p, bool fp32, const double* Y,
                                 const double* U, double* HU, int riem, hipStream_t s);
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
mdsdp_status vec_dots(const double* const* a, const double* const* b, int npairs, long long len,
                      double* out_dev, double* part, int nblk, hipStream_t s);
mdsdp_status vec_lincomb(long long len, double alpha, const double* x, double beta,
                         const double* y, double* out, hipStream_t s);
mdsdp_status vec_fill(long long len, double v, double* out, hipStream_t s);

void timer_begin(mdsdp_problem P, hipStream_t s, const char* name);
void timer_end(mdsdp_problem P, hipStream_t s);

}  // namespace mdsdp
