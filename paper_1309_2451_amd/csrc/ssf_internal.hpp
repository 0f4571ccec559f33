// Internal interface between the host runtime and the pencil-pass kernels.
// Not part of the public C ABI (include/ssf.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssf {

// Operation codes applied on the way in (pre), between the two transforms of
// a fused pass (mid), and on the way out (post).
enum : int { PRE_SCALE = 1, PRE_VPHASE = 2, PRE_ADJ = 4 };
// MID_VNORM: two potential half-steps with the field's norm summed between
// them (imaginary time: the end of one step and the start of the next).
enum : int { MID_NONE = 0, MID_KINETIC = 1, MID_VPHASE = 2, MID_VNORM = 3 };
enum : int { POST_VPHASE = 1, POST_OBS = 2, POST_ADJ = 4, POST_KIN = 8 };
// Potential sources.
enum : int { V_NONE = 0, V_TAB64 = 1, V_TAB32 = 2, V_CTAP = 3 };
// Number of FP64 partial sums per workgroup written by the reductions.
constexpr int NRED_OBS = 8;   // norm, sum x n, sum y n, sum z n, P1, P2, P3, sum V n
constexpr int NRED_ADJ = 3;   // one per guide
constexpr int MAX_GUIDES = 3;

// Kinds of pencil pass.
enum PassKind : int {
  CONTIG_FWD = 0,          // x pencils, forward transform
  CONTIG_INV = 1,          // x pencils, inverse transform (unnormalised)
  CONTIG_FUSED = 2,        // x pencils, inverse - mid op - forward
  STRIDED_FWD = 3,         // y or z pencils, forward
  STRIDED_INV = 4,         // y or z pencils, inverse
  STRIDED_FUSED = 5,       // z pencils, forward - mid op - inverse
  NUM_PASS_KINDS = 6
};

// One instance of a batched launch: its field and its potential -- guide
// tables (A | D | B, MAX_GUIDES planes each, as for a single handle) or an
// FP64 (nz, ny, nx) table.
struct InstDesc {
  const void* in;
  void* out;
  const double* ctap;
  const double* vtab;
  int ix_lo, ix_hi;        // guide partition of this instance (observations)
};

struct PassArgs {
  const void* in;          // storage in  (float2 or double2)
  void* out;               // storage out (may equal in)
  const void* aux;         // companion field for the adjoint reduction (same layout)
  int nx, ny, nz;
  long long nstride;       // element stride along the transformed axis (strided passes)
  long long ostride;       // stride of the outer pencil index (strided passes)
  int nouter;              // extent of the outer pencil index (strided passes)
  int axis;                // 0, 1, 2: axis being transformed
  int pre, mid, post;      // op masks
  int imag;                // 1: imaginary-time factors (real exponentials)
  double cpre, cmid, cpost;  // potential phase multipliers: theta = V * c
  const double2* tw;       // W[t] = exp(-2 pi i t / N), t < N, N = transform length
  const double2* kt[3];    // kinetic factors per axis (FFT bin order); 1/N folded into kt[2]
  int vkind;
  const void* vtab;        // (nz, ny, nx) potential table (f64 or f32)
  const double* ctapA;     // (MAX_GUIDES, nz, nx): v0_g exp(-(x - xc_g(z))^2 / (2 s_g^2)), 0 if unused
  const double* ctapD;     // (MAX_GUIDES, nz, nx): ctapA * (x - xc_g(z)) / s_g^2
  const double* ctapB;     // (MAX_GUIDES, ny): exp(-y^2 / (2 s_g^2))
  int nguides;
  const double* scale;     // device scalar multiplier (PRE_SCALE)
  double* partials;        // per-workgroup FP64 partial sums
  double lo[3], d[3];      // grid origin and spacing
  double kfac[3];          // 2 pi / L per axis
  int ix_lo, ix_hi;        // P1: ix < ix_lo, P3: ix > ix_hi, P2 otherwise
  const int* ixz;          // nullptr, or per plane z: (ix_lo, ix_hi) at [2z], [2z+1]
  int tiles_x, tiles_y;    // tile grid (set by the launcher); partial sums are per tile
  int small_phase;         // |V cmid| bound: 2: <= 0.1, 1: <= pi/4 (no argument reduction), 0: any
  const InstDesc* inst;    // batched launch: ninst instances of this grid (nullptr: single field)
  int ninst;
};

// Tile geometry and launcher for one transform length and one storage type.
struct PassShape {
  int px, po;              // strided: px consecutive x by po outer pencils; contig: px rows
  int threads;             // workgroup size
};

// Strided tile variants (chosen per axis by the autotuner): 0 = px columns of
// 128 B of storage; 1 = half as many columns (half the workgroup and LDS);
// 2 = the variant-0 tile with twice the values per thread, no register
// prefetch, FP32 LDS exchanges for complex64 (two workgroups per CU).
constexpr int NUM_STRIDED_VARIANTS = 3;

struct KernelSet {
  int N;
  PassShape contig[2];                             // [dtype]: 0 = complex64 storage, 1 = complex128
  PassShape strided[2][NUM_STRIDED_VARIANTS];      // [dtype][variant]
  // `tiles` = (tiles_x, tiles_y); the launcher picks the persistent grid.
  hipError_t (*launch)(int kind, int dt_index, int variant, const PassArgs& a, dim3 tiles, hipStream_t s);
};

// Every supported transform length.  The kernel TU is compiled once per entry.
#define SSF_LENGTHS(X) \
  X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) \
  X(12) X(24) X(48) X(96) X(192) X(384) X(768) \
  X(20) X(40) X(80) X(160) X(320) X(640)

#define SSF_DECLARE_SET(NN) extern const KernelSet kernels_##NN;
SSF_LENGTHS(SSF_DECLARE_SET)
#undef SSF_DECLARE_SET

}  // namespace ssf
