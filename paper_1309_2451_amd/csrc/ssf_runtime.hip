// Host runtime and C ABI of libssf (declarations and contracts: include/ssf.h).
//
// The runtime owns per-grid tables (FP64 twiddles, kinetic phase tables,
// three-guide potential tables), the FP64 partial-sum workspace, and the
// sequencing of pencil passes for one Strang step of the Fourier
// split-operator method (Morgan et al., arXiv:1309.2451, Sec. IV):
//   x forward (+ exp(-i V dt/2) on load) -> y forward -> z forward, kinetic
//   phase, z inverse (one pass) -> y inverse -> x inverse (+ exp(-i V dt/2),
//   + reductions on store).
// Between two steps with no observation the x inverse / x forward pair is one
// fused pass with exp(-i V dt) in the middle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ssf.h"
#include "ssf_pass.hpp"

using ssf::PassArgs;
using ssf::KernelSet;

static_assert(ssf::NUM_STRIDED_VARIANTS == SSF_TILE_VARIANTS, "tile variant count of the C ABI");

namespace {

thread_local std::string g_last_error;

ssf_status fail(ssf_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      return fail(e_ == hipErrorOutOfMemory ? SSF_E_NOMEM : SSF_E_DEVICE,             \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    }                                                                                 \
  } while (0)

#define SSF_TRY(expr)                \
  do {                               \
    ssf_status s_ = (expr);          \
    if (s_ != SSF_OK) return s_;     \
  } while (0)

const KernelSet* find_kernels(int n) {
#define SSF_CASE(NN) \
  if (n == NN) return &ssf::kernels_##NN;
  SSF_LENGTHS(SSF_CASE)
#undef SSF_CASE
  return nullptr;
}

constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------------------
// Small kernels: tables, finalisation of reductions, pointwise helpers.
// ---------------------------------------------------------------------------

// Kinetic factor table of one axis: t[j] = exp(-i k_j^2 c) (or exp(-k_j^2 c)
// in imaginary time) times `extra`, k_j = kfac * (j if 2j < n else j - n).
// The phase argument is formed in FP64 from the integer m^2 and reduced
// modulo 2 pi with a two-part constant before sincos.
__global__ void ktab_kernel(double2* t, int n, double kfac, double c, int imag, double extra) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int m = 2 * j < n ? j : j - n;
  const double k = kfac * (double)m;
  const double th = k * k * c;
  double2 f;
  if (imag) {
    f = make_double2(exp(-th) * extra, 0.0);
  } else {
    const double q = rint(th * 0.15915494309189533577);
    double r = fma(-q, 6.283185307179586232, th);
    r = fma(-q, 2.4492935982947064e-16, r);
    double s, co;
    sincos(r, &s, &co);
    f = make_double2(co * extra, -s * extra);
  }
  t[j] = f;
}

// Sum NV partial vectors (stride 8) in a fixed order: thread t takes blocks
// t, t+256, ...; then a fixed-shape tree.  Deterministic.
template <int NV>
__device__ void sum_partials(const double* p, long long nblk, double (&out)[NV], double* sh) {
  double acc[NV];
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (long long b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int q = 0; q < NV; ++q) acc[q] += p[b * 8 + q];
  for (int q = 0; q < NV; ++q) sh[q * 256 + threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NV; ++q) sh[q * 256 + threadIdx.x] += sh[q * 256 + threadIdx.x + w];
    __syncthreads();
  }
  for (int q = 0; q < NV; ++q) out[q] = sh[q * 256];
}

// Finalise an observation from the x-pass partials.  mode bit 0: write obs;
// bit 1: imaginary time (energy = -ln(norm)/(2 dtau), scale = 1/sqrt(norm)).
// kin != nullptr: energy = sum kin * dv / npts + epot.
__global__ void __launch_bounds__(256) obs_finalize(const double* partials, long long nblk, double dv,
                                                    ssf_obs* obs, long long step, int mode, double dtau,
                                                    double* scale, const double* kin, long long nkin,
                                                    double npts) {
  __shared__ double sh[8 * 256];
  double s[8];
  sum_partials<8>(partials, nblk, s, sh);
  double ek = 0.0;
  if (kin) {
    __syncthreads();
    double k1[1];
    sum_partials<1>(kin, nkin, k1, sh);
    ek = k1[0];
  }
  if (threadIdx.x != 0) return;
  const double norm = s[0] * dv;
  ssf_obs o;
  o.norm = norm;
  o.mean[0] = s[1] * dv;
  o.mean[1] = s[2] * dv;
  o.mean[2] = s[3] * dv;
  o.pop[0] = s[4] * dv;
  o.pop[1] = s[5] * dv;
  o.pop[2] = s[6] * dv;
  o.epot = s[7] * dv;
  o.energy = 0.0;
  if (mode & 2) o.energy = -log(norm) / (2.0 * dtau);
  if (kin) o.energy = ek * dv / npts + o.epot;
  o.step = step;
  o.flags = isfinite(norm) ? 0 : 1;
  o.reserved = 0;
  if ((mode & 1) && obs) *obs = o;
  if ((mode & 2) && scale) *scale = 1.0 / sqrt(norm);
}

// G[g][z] += w * sum over the y tiles of plane z of the x-pass partials.
__global__ void adj_finalize(const double* partials, int ytiles, int nz, int nguides, double w, double* G) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * nguides) return;
  const int g = t / nz, z = t % nz;
  double s = 0.0;
  for (int yt = 0; yt < ytiles; ++yt) s += partials[((long long)z * ytiles + yt) * 8 + g];
  G[(long long)g * nz + z] += w * s;
}

// out[g][m] = sum_z G[g][z] B[z][m]: chain rule from guide centres to the
// coefficients of x_g(z) = sum_m c_gm B_m(z).  One thread per (g, m), z in order.
__global__ void profile_grad_kernel(const double* G, const double* B, int nz, int M, int ng, double* out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ng * M) return;
  const int g = t / M, m = t % M;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += G[(long long)g * nz + z] * B[(long long)z * M + m];
  out[t] = s;
}

// Norm, moments, populations and potential energy of a stored field, with the
// same partial layout as the x pass: block (y tile of `rows` rows, plane z).
template <typename S>
__global__ void __launch_bounds__(256) obs_reduce_kernel(PassArgs a, int rows) {
  __shared__ double red[4 * 8];
  const int z = blockIdx.y, y0 = blockIdx.x * rows;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const S* in = (const S*)a.in;
  const int ilo = a.ixz ? a.ixz[2 * z] : a.ix_lo, ihi = a.ixz ? a.ixz[2 * z + 1] : a.ix_hi;
  for (int e = threadIdx.x; e < rows * a.nx; e += 256) {
    const int y = y0 + e / a.nx, x = e % a.nx;
    if (y >= a.ny) break;
    const double2 v = ssf::ld2(in + ((long long)z * a.ny + y) * a.nx + x);
    const double rho = v.x * v.x + v.y * v.y;
    acc[0] += rho;
    acc[1] += (a.lo[0] + x * a.d[0]) * rho;
    acc[2] += (a.lo[1] + y * a.d[1]) * rho;
    acc[3] += (a.lo[2] + z * a.d[2]) * rho;
    if (x < ilo) acc[4] += rho;
    else if (x > ihi) acc[6] += rho;
    else acc[5] += rho;
    acc[7] += ssf::potential_at(a, x, y, z) * rho;
  }
  ssf::block_sum<256, 8>(acc, a.partials + (long long)(blockIdx.y * gridDim.x + blockIdx.x) * 8, red);
}

template <typename S>
__global__ void scale_kernel(S* p, long long n, const double* scale) {
  const double s = *scale;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double2 v = ssf::ld2(p + i);
    ssf::st2(p + i, make_double2(v.x * s, v.y * s));
  }
}

// lambda = psi where x > x_hi (ix > ix_hi, per plane if ixz is set), 0 elsewhere.
template <typename S>
__global__ void mask_kernel(const S* psi, S* lam, long long n, int nx, long long nxy, int ix_hi, const int* ixz) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx);
    const int ihi = ixz ? ixz[2 * (i / nxy) + 1] : ix_hi;
    double2 v = ssf::ld2(psi + i);
    if (x <= ihi) v = make_double2(0.0, 0.0);
    ssf::st2(lam + i, v);
  }
}

// Observations of the ninst fields of a batched group: block (y tile of `rows`
// rows, plane z, instance k); partials are instance-major.
template <typename S>
__global__ void __launch_bounds__(256) obs_reduce_batch(PassArgs a, int rows) {
  __shared__ double red[4 * 8];
  const int k = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * rows;
  const ssf::InstDesc d = a.inst[k];
  const S* in = (const S*)d.in;
  const long long pl = (long long)a.nz * a.nx;
  const long long gplane = (long long)ssf::MAX_GUIDES * pl;
  const double* A = d.ctap;
  const double* B = d.ctap ? d.ctap + 2 * gplane : nullptr;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < rows * a.nx; e += 256) {
    const int y = y0 + e / a.nx, x = e % a.nx;
    if (y >= a.ny) break;
    const double2 v = ssf::ld2(in + ((long long)z * a.ny + y) * a.nx + x);
    const double rho = v.x * v.x + v.y * v.y;
    const long long o = (long long)z * a.nx + x;
    const double V = d.vtab ? d.vtab[((long long)z * a.ny + y) * a.nx + x]
                            : -(A[o] * B[y] + A[pl + o] * B[a.ny + y] + A[2 * pl + o] * B[2 * a.ny + y]);
    acc[0] += rho;
    acc[1] += (a.lo[0] + x * a.d[0]) * rho;
    acc[2] += (a.lo[1] + y * a.d[1]) * rho;
    acc[3] += (a.lo[2] + z * a.d[2]) * rho;
    if (x < d.ix_lo) acc[4] += rho;
    else if (x > d.ix_hi) acc[6] += rho;
    else acc[5] += rho;
    acc[7] += V * rho;
  }
  ssf::block_sum<256, 8>(acc, a.partials + (((long long)k * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 8, red);
}

// Block k: fixed-order sum of instance k's nblk partials -> obs[slot[k]].
__global__ void __launch_bounds__(256) obs_finalize_batch(const double* partials, long long nblk, double dv,
                                                          ssf_obs* obs, const int* slot, long long step) {
  __shared__ double sh[8 * 256];
  double s[8];
  sum_partials<8>(partials + (long long)blockIdx.x * nblk * 8, nblk, s, sh);
  if (threadIdx.x != 0) return;
  ssf_obs o;
  o.norm = s[0] * dv;
  o.mean[0] = s[1] * dv;
  o.mean[1] = s[2] * dv;
  o.mean[2] = s[3] * dv;
  o.pop[0] = s[4] * dv;
  o.pop[1] = s[5] * dv;
  o.pop[2] = s[6] * dv;
  o.epot = s[7] * dv;
  o.energy = 0.0;
  o.step = step;
  o.flags = isfinite(o.norm) ? 0 : 1;
  o.reserved = 0;
  obs[slot[blockIdx.x]] = o;
}

// Plain field copy, one value per lane per iteration (grid-stride).
template <typename S>
__global__ void __launch_bounds__(256) copy_kernel(const S* in, S* out, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    if constexpr (sizeof(S) == 8) ssf::st2(out + i, ssf::ld2(in + i));
    else ssf::st2(out + i, ssf::ldraw(in + i));
  }
}

// out[z nx + x] = dy sum_y |psi(x, y, z)|^2, one thread per (x, z), fixed order.
template <typename S>
__global__ void __launch_bounds__(256) density_xz_kernel(const S* in, int nx, int ny, double dy, double* out) {
  const int x = blockIdx.x * 256 + threadIdx.x, z = blockIdx.y;
  if (x >= nx) return;
  const S* p = in + (long long)z * ny * nx + x;
  double s = 0.0;
#pragma unroll 8
  for (int y = 0; y < ny; ++y) {
    const double2 v = ssf::ld2(p + (long long)y * nx);
    s += v.x * v.x + v.y * v.y;
  }
  out[(long long)z * nx + x] = s * dy;
}

// ---------------------------------------------------------------------------
// Atom-chip potential (Sec. III): thin current-carrying wires lying in the
// chip plane y = 0, a homogeneous bias field across them (x) and an offset
// field along them (z), plus a harmonic trap along z.  One thread per grid
// point sums the Biot-Savart field of every straight wire segment; the
// segments are staged through LDS in chunks.
// ---------------------------------------------------------------------------
struct ChipSeg {
  double ax, az;    // segment start (x, z), length units
  double lx, lz;    // segment vector end - start
  double kI;        // mu0 I / (4 pi length_unit): tesla times length units
  double pad;
};
constexpr int CHIP_CHUNK = 1024;   // segments per LDS stage (48 KiB)

// Field of one straight segment at P = (px, py, pz) relative to the segment
// start (a = P - A) and end (b = P - B, B = A + L): the finite-wire law
//   dB = k I (L x a) (L.a/|a| - L.b/|b|) / |L x a|^2,
// which reduces to mu0 I / (2 pi rho) for an infinitely long wire.  With the
// wire in the plane y = 0, L = (lx, 0, lz) and L x a = (-lz py, lz ax - lx az,
// lx py).  A point on the segment's line gets nothing from it.
__device__ __forceinline__ void seg_field(const ChipSeg& s, double px, double py, double pz, double& bx,
                                          double& by, double& bz) {
  const double ax = px - s.ax, az = pz - s.az;
  const double cy = s.lz * ax - s.lx * az;
  const double l2 = s.lx * s.lx + s.lz * s.lz;
  const double c2 = py * py * l2 + cy * cy;
  if (c2 == 0.0) return;
  const double la = s.lx * ax + s.lz * az;       // L.a
  const double lb = la - l2;                       // L.b
  const double bxr = ax - s.lx, bzr = az - s.lz;
  const double ra = sqrt(ax * ax + py * py + az * az);
  const double rb = sqrt(bxr * bxr + py * py + bzr * bzr);
  const double f = s.kI * (la / ra - lb / rb) / c2;
  bx -= f * s.lz * py;
  by += f * cy;
  bz += f * s.lx * py;
}

// V[z][y][x] = mu_e (|B| - b_ip) + omega_z^2 (z - z_c)^2 / 2, B = wires +
// (b_bias, 0, b_ip).  |B| - b_ip is formed as (|B|^2 - b_ip^2) / (|B| + b_ip)
// with |B|^2 - b_ip^2 = Bx^2 + By^2 + Bwz (Bwz + 2 b_ip): at the guide centres
// |B| is close to b_ip, and the direct difference would cancel.
__global__ void __launch_bounds__(256) chip_kernel(double* V, int nx, int ny, int nz, double lox, double loy,
                                                   double loz, double dx, double dy, double dz, const ChipSeg* seg,
                                                   int nseg, double b_bias, double b_ip, double mu_e, double omz,
                                                   double z_c) {
  __shared__ ChipSeg s_seg[CHIP_CHUNK];
  const long long npts = (long long)nx * ny * nz;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int x = (int)(i % nx);
  const int y = (int)((i / nx) % ny);
  const int z = (int)(i / ((long long)nx * ny));
  const double px = lox + x * dx, py = loy + y * dy, pz = loz + z * dz;
  double bx = 0.0, by = 0.0, bz = 0.0;
  for (int c0 = 0; c0 < nseg; c0 += CHIP_CHUNK) {
    const int cn = min(CHIP_CHUNK, nseg - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cn; j += 256) s_seg[j] = seg[c0 + j];
    __syncthreads();
    if (i < npts)
      for (int j = 0; j < cn; ++j) seg_field(s_seg[j], px, py, pz, bx, by, bz);
  }
  if (i >= npts) return;
  const double tx = bx + b_bias, tz = bz + b_ip;
  const double mag = sqrt(tx * tx + by * by + tz * tz);
  const double excess = (tx * tx + by * by + bz * (bz + 2.0 * b_ip)) / (mag + b_ip);
  const double w = pz - z_c;
  V[i] = mu_e * excess + 0.5 * omz * omz * w * w;
}

// ---------------------------------------------------------------------------
// Handle.
// ---------------------------------------------------------------------------
struct KTab {
  double dt = 0.0;
  int imag = -1;
  double2* t = nullptr;  // [nx | ny | nz]
  unsigned long long use = 0;
};

}  // namespace

struct ssf_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, d[3] = {1, 1, 1};
  double dv = 1.0;
  int dtype = SSF_C128;
  int dti = 1;                         // 0 = complex64, 1 = complex128
  int kti = 1;                         // kernels: dti, or 2 = complex64 storage with FP32 arithmetic
  size_t esize = 16;
  long long npts = 1;
  const KernelSet* ks[3] = {nullptr, nullptr, nullptr};
  double2* tw[3] = {nullptr, nullptr, nullptr};
  static constexpr int NKT = 8;
  KTab kt[NKT];
  unsigned long long kt_clock = 0;
  int vkind = ssf::V_NONE;
  const void* vtab = nullptr;
  double* ctap = nullptr;              // A | D | B
  int nguides = 0;
  double vmax = 0.0;                   // bound on |V| for the guide potential
  int ix_lo = -1, ix_hi = 1 << 30;     // default: everything in P2
  int fuse = 1;
  int split = SSF_SPLIT_VTV;           // ordering of ssf_step in real time
  int* ixz = nullptr;                  // per-plane partition bounds (device, 2 nz)
  int zpart = 0;                       // 1: ixz in use
  int var[3] = {0, 0, 0};              // strided tile variant per axis (autotuned)
  double* partials = nullptr;          // workspace: 2 regions of part_cap blocks x 8 doubles
  long long part_cap = 0;
  double* dscal = nullptr;             // device scalars: [0] scale
  void* work = nullptr;                // field-sized workspace (lazy)
  // Allocation-free steps (ssf_step_noalloc): while set, kinetic tables are
  // built here for the call (up to two: dt and dt/2) instead of in the cache.
  double2* ktfix = nullptr;
  int ktfix_used = 0;
  ChipSeg* chipseg = nullptr;          // wire segments of ssf_chip_potential (device, grows)
  size_t chipseg_cap = 0;
  // optional per-pass timing: an event pair around every pass launch
  int timing = 0;
  std::vector<hipEvent_t> ev[ssf::NUM_PASS_KINDS];
  size_t ev_used[ssf::NUM_PASS_KINDS] = {};
};

namespace {

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// Guide tables on the host, FP64: A_g(x, z), D_g(x, z) = A_g (x - xc_g)/s_g^2
// and B_g(y) for MAX_GUIDES guides (unused ones zero), the layout the pass
// kernels read.
// Returns a bound on |V| over the grid: max over (x, z) of sum_g |A_g(x, z)|
// (every B_g(y) <= 1).
double ctap_tables(const ssf_handle* h, const ssf_ctap_desc* d, std::vector<double>& tab) {
  // The kernels always evaluate MAX_GUIDES guides: unused ones get zero tables.
  const int nx = h->n[0], ny = h->n[1], nz = h->n[2], ng = d->nguides;
  const long long plane = (long long)ssf::MAX_GUIDES * nz * nx;
  tab.assign(2 * plane + (long long)ssf::MAX_GUIDES * ny, 0.0);
  for (int g = 0; g < ng; ++g) {
    const double s2 = d->sigma[g] * d->sigma[g];
    for (int z = 0; z < nz; ++z) {
      const double xc = d->xc[(long long)g * nz + z];
      for (int x = 0; x < nx; ++x) {
        const double dx = h->lo[0] + x * h->d[0] - xc;
        const double A = d->v0[g] * std::exp(-dx * dx / (2.0 * s2));
        tab[((long long)g * nz + z) * nx + x] = A;
        tab[plane + ((long long)g * nz + z) * nx + x] = A * dx / s2;
      }
    }
    for (int y = 0; y < ny; ++y) {
      const double yc = h->lo[1] + y * h->d[1];
      tab[2 * plane + (long long)g * ny + y] = std::exp(-yc * yc / (2.0 * s2));
    }
  }
  double vmax = 0.0;
  for (long long o = 0; o < (long long)nz * nx; ++o) {
    double a = 0.0;
    for (int g = 0; g < ng; ++g) a += std::fabs(tab[(long long)g * nz * nx + o]);
    vmax = std::max(vmax, a);
  }
  return vmax;
}

// Which phase series the fused x pass may use for exp(-i V dt): 2 when
// |V dt| <= 0.1, 1 when |V dt| <= 0.78 (inside pi/4), else 0 (reduction).
int phase_tier(int vkind, double vmax, double dt) {
  if (vkind == ssf::V_NONE) return 2;
  if (vkind != ssf::V_CTAP) return 0;
  const double t = vmax * std::fabs(dt);
  return t <= 0.1 ? 2 : (t <= 0.78 ? 1 : 0);
}

// Partition of x into guide regions as integer bounds: P1 for x_i < x_lo,
// P3 for x_i > x_hi, with x_i = lo + i d (the expression the kernels use).
void partition_indices(const ssf_handle* h, double x_lo, double x_hi, int* ilo, int* ihi) {
  int a = 0;
  while (a < h->n[0] && h->lo[0] + a * h->d[0] < x_lo) ++a;
  int b = h->n[0] - 1;
  while (b >= 0 && h->lo[0] + b * h->d[0] > x_hi) --b;
  *ilo = a;
  *ihi = b;
}



// Grid of one pass kind over the handle's field.
dim3 pass_grid(const ssf_handle* h, int axis, int variant = -1) {
  const KernelSet* ks = h->ks[axis];
  if (axis == 0) {
    const int rows = ks->contig[h->dti].px;
    return dim3((unsigned)ceil_div(h->n[1], rows), (unsigned)h->n[2], 1);
  }
  const auto& sh = ks->strided[h->dti][variant < 0 ? h->var[axis] : variant];
  const int nouter = axis == 1 ? h->n[2] : h->n[1];
  return dim3((unsigned)ceil_div(h->n[0], sh.px), (unsigned)ceil_div(nouter, sh.po), 1);
}

PassArgs base_args(const ssf_handle* h, const void* in, void* out, int axis) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.nx = h->n[0];
  a.ny = h->n[1];
  a.nz = h->n[2];
  a.axis = axis;
  if (axis == 1) {
    a.nstride = h->n[0];
    a.ostride = (long long)h->n[0] * h->n[1];
    a.nouter = h->n[2];
  } else if (axis == 2) {
    a.nstride = (long long)h->n[0] * h->n[1];
    a.ostride = h->n[0];
    a.nouter = h->n[1];
  }
  a.tw = h->tw[axis];
  a.vkind = h->vkind;
  a.vtab = h->vtab;
  if (h->ctap) {
    const long long plane = (long long)ssf::MAX_GUIDES * h->n[2] * h->n[0];
    a.ctapA = h->ctap;
    a.ctapD = h->ctap + plane;
    a.ctapB = h->ctap + 2 * plane;
  }
  a.nguides = h->nguides;
  a.scale = h->dscal;
  a.partials = h->partials;
  for (int q = 0; q < 3; ++q) {
    a.lo[q] = h->lo[q];
    a.d[q] = h->d[q];
    a.kfac[q] = TWO_PI / (h->hi[q] - h->lo[q]);
  }
  a.ix_lo = h->ix_lo;
  a.ix_hi = h->ix_hi;
  a.ixz = h->zpart ? h->ixz : nullptr;
  return a;
}

ssf_status launch(ssf_handle* h, int kind, int axis, const PassArgs& a) {
  const dim3 g = pass_grid(h, axis);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    auto& pool = h->ev[kind];
    size_t& used = h->ev_used[kind];
    while (pool.size() < 2 * (used + 1)) {
      hipEvent_t ev;
      HIP_TRY(hipEventCreate(&ev));
      pool.push_back(ev);
    }
    e0 = pool[2 * used];
    e1 = pool[2 * used + 1];
    ++used;
    HIP_TRY(hipEventRecord(e0, h->stream));
  }
  hipError_t e = h->ks[axis]->launch(kind, h->kti, h->var[axis], a, g, h->stream);
  if (e != hipSuccess) return fail(SSF_E_DEVICE, std::string("pass launch: ") + hipGetErrorString(e));
  if (h->timing) HIP_TRY(hipEventRecord(e1, h->stream));
  return SSF_OK;
}

long long blocks_of(const ssf_handle* h, int axis) {
  const dim3 g = pass_grid(h, axis);
  return (long long)g.x * g.y;
}

ssf_status check_handle(ssf_handle* h) {
  if (!h) return fail(SSF_E_INVALID, "null handle");
  HIP_TRY(hipSetDevice(h->device));
  return SSF_OK;
}

ssf_status check_field(const ssf_handle* h, const void* p, const char* what) {
  if (!p) return fail(SSF_E_INVALID, std::string(what) + " is null");
  if (((uintptr_t)p) % (h->esize / 2) != 0)
    return fail(SSF_E_INVALID, std::string(what) + " is not aligned to the element size");
  return SSF_OK;
}

// Kinetic factor tables of the three axes for (dt, imag) into t[nx | ny | nz].
ssf_status build_ktab(ssf_handle* h, double2* t, double dt, int imag) {
  const double inv_n = 1.0 / (double)h->npts;
  for (int a = 0; a < 3; ++a) {
    const int n = h->n[a];
    const double kfac = TWO_PI / (h->hi[a] - h->lo[a]);
    hipLaunchKernelGGL(ktab_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, h->stream, t, n, kfac, 0.5 * dt,
                       imag, a == 2 ? inv_n : 1.0);
    HIP_TRY(hipGetLastError());
    t += n;
  }
  return SSF_OK;
}

// Kinetic tables for (dt, imag): built on the device once, then reused.  In
// an allocation-free call they are built into the call's scratch instead.
ssf_status get_ktab(ssf_handle* h, double dt, int imag, const double2** out) {
  if (h->ktfix) {
    if (h->ktfix_used >= 2) return fail(SSF_E_INVALID, "more than two kinetic tables in one allocation-free call");
    double2* t = h->ktfix + (size_t)h->ktfix_used++ * (size_t)(h->n[0] + h->n[1] + h->n[2]);
    SSF_TRY(build_ktab(h, t, dt, imag));
    *out = t;
    return SSF_OK;
  }
  for (auto& k : h->kt)
    if (k.t && k.dt == dt && k.imag == imag) {
      k.use = ++h->kt_clock;
      *out = k.t;
      return SSF_OK;
    }
  KTab* slot = &h->kt[0];
  for (auto& k : h->kt) {
    if (!k.t) { slot = &k; break; }
    if (k.use < slot->use) slot = &k;
  }
  if (!slot->t) HIP_TRY(hipMalloc(&slot->t, sizeof(double2) * (h->n[0] + h->n[1] + h->n[2])));
  SSF_TRY(build_ktab(h, slot->t, dt, imag));
  slot->dt = dt;
  slot->imag = imag;
  slot->use = ++h->kt_clock;
  *out = slot->t;
  return SSF_OK;
}

ssf_status finalize_obs(ssf_handle* h, ssf_obs* obs, long long step, int mode, double dtau, const double* kin,
                        long long nkin) {
  hipLaunchKernelGGL(obs_finalize, dim3(1), dim3(256), 0, h->stream, h->partials, blocks_of(h, 0), h->dv, obs, step,
                     mode, dtau, h->dscal, kin, nkin, (double)h->npts);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

// Pointwise reduction of a stored field into the x-pass partial layout.
ssf_status reduce_field(ssf_handle* h, const void* psi) {
  PassArgs a = base_args(h, psi, nullptr, 0);
  const int rows = h->ks[0]->contig[h->dti].px;
  const dim3 g = pass_grid(h, 0);
  if (h->dti == 0)
    hipLaunchKernelGGL(obs_reduce_kernel<float2>, g, dim3(256), 0, h->stream, a, rows);
  else
    hipLaunchKernelGGL(obs_reduce_kernel<double2>, g, dim3(256), 0, h->stream, a, rows);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

ssf_status scale_field(ssf_handle* h, void* psi) {
  const unsigned blocks = (unsigned)std::min<long long>(ceil_div(h->npts, 256), 65536);
  if (h->dti == 0)
    hipLaunchKernelGGL(scale_kernel<float2>, dim3(blocks), dim3(256), 0, h->stream, (float2*)psi, h->npts, h->dscal);
  else
    hipLaunchKernelGGL(scale_kernel<double2>, dim3(blocks), dim3(256), 0, h->stream, (double2*)psi, h->npts, h->dscal);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

// Middle of a step: y forward, z forward + kinetic + z inverse, y inverse.
ssf_status step_middle(ssf_handle* h, void* psi, const double2* kt) {
  PassArgs ay = base_args(h, psi, psi, 1);
  SSF_TRY(launch(h, ssf::STRIDED_FWD, 1, ay));
  PassArgs az = base_args(h, psi, psi, 2);
  az.mid = ssf::MID_KINETIC;
  az.kt[0] = kt;
  az.kt[1] = kt + h->n[0];
  az.kt[2] = kt + h->n[0] + h->n[1];
  SSF_TRY(launch(h, ssf::STRIDED_FUSED, 2, az));
  SSF_TRY(launch(h, ssf::STRIDED_INV, 1, ay));
  return SSF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t ssf_supported_length(int32_t n) { return find_kernels(n) != nullptr ? 1 : 0; }

const char* ssf_status_string(ssf_status s) {
  switch (s) {
    case SSF_OK: return "ok";
    case SSF_E_INVALID: return "invalid argument";
    case SSF_E_UNSUPPORTED: return "unsupported transform length";
    case SSF_E_NOMEM: return "out of device memory";
    case SSF_E_NODEVICE: return "no HIP device";
    case SSF_E_DEVICE: return "HIP runtime error";
    case SSF_E_NONFINITE: return "non-finite norm observed";
    default: return "unknown status";
  }
}

const char* ssf_last_error(void) { return g_last_error.c_str(); }

ssf_status ssf_destroy(ssf_handle* h);

ssf_status ssf_create(const ssf_grid_desc* grid, int32_t dtype, void* hip_stream, ssf_handle** out) {
  if (!grid || !out) return fail(SSF_E_INVALID, "null argument");
  *out = nullptr;
  if (dtype != SSF_C64 && dtype != SSF_C128) return fail(SSF_E_INVALID, "dtype must be SSF_C64 or SSF_C128");
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1) return fail(SSF_E_INVALID, "grid sizes must be >= 1");
    if (!(grid->hi[a] > grid->lo[a]) || !std::isfinite(grid->hi[a] - grid->lo[a]))
      return fail(SSF_E_INVALID, "grid needs hi > lo on every axis");
    if (!find_kernels(grid->n[a]))
      return fail(SSF_E_UNSUPPORTED, "transform length " + std::to_string(grid->n[a]) + " is not supported");
  }
  if ((long long)grid->n[0] * grid->n[1] * grid->n[2] >= (1LL << 31))
    return fail(SSF_E_INVALID, "grids must have fewer than 2^31 points");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(SSF_E_NODEVICE, "no HIP device visible");
  ssf_handle* h = new ssf_handle();
  HIP_TRY(hipGetDevice(&h->device));
  h->stream = (hipStream_t)hip_stream;
  h->dtype = dtype;
  h->dti = dtype == SSF_C64 ? 0 : 1;
  h->kti = h->dti;
  h->esize = dtype == SSF_C64 ? 8 : 16;
  h->npts = 1;
  for (int a = 0; a < 3; ++a) {
    h->n[a] = grid->n[a];
    h->lo[a] = grid->lo[a];
    h->hi[a] = grid->hi[a];
    h->d[a] = (grid->hi[a] - grid->lo[a]) / grid->n[a];
    h->npts *= grid->n[a];
    h->ks[a] = find_kernels(grid->n[a]);
  }
  h->dv = h->d[0] * h->d[1] * h->d[2];
  auto cleanup = [&](ssf_status s) { ssf_destroy(h); return s; };
  // twiddles W_N[t] = exp(-2 pi i t / N), each from its own cos/sin in FP64
  for (int a = 0; a < 3; ++a) {
    const int n = h->n[a];
    std::vector<double2> w(n);
    for (int t = 0; t < n; ++t) {
      const double ang = TWO_PI * (double)t / (double)n;
      w[t] = make_double2(std::cos(ang), -std::sin(ang));
    }
    if (hipMalloc(&h->tw[a], sizeof(double2) * n) != hipSuccess) return cleanup(fail(SSF_E_NOMEM, "twiddle table"));
    if (hipMemcpy(h->tw[a], w.data(), sizeof(double2) * n, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(SSF_E_DEVICE, "twiddle upload"));
  }
  long long cap = 0;
  for (int a = 0; a < 3; ++a)
    for (int v = 0; v < ssf::NUM_STRIDED_VARIANTS; ++v) {
      const dim3 g = pass_grid(h, a, v);
      cap = std::max(cap, (long long)g.x * g.y);
    }
  h->part_cap = cap;
  if (hipMalloc(&h->partials, sizeof(double) * 8 * cap * 2) != hipSuccess)
    return cleanup(fail(SSF_E_NOMEM, "partials workspace"));
  if (hipMalloc(&h->dscal, sizeof(double) * 8) != hipSuccess) return cleanup(fail(SSF_E_NOMEM, "device scalars"));
  const double one[8] = {1, 0, 0, 0, 0, 0, 0, 0};
  if (hipMemcpy(h->dscal, one, sizeof(one), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(SSF_E_DEVICE, "device scalars upload"));
  *out = h;
  return SSF_OK;
}

ssf_status ssf_destroy(ssf_handle* h) {
  if (!h) return SSF_OK;
  (void)hipSetDevice(h->device);
  hipError_t e = hipStreamSynchronize(h->stream);
  for (auto& k : h->kt) if (k.t) (void)hipFree(k.t);
  for (int a = 0; a < 3; ++a) if (h->tw[a]) (void)hipFree(h->tw[a]);
  if (h->ctap) (void)hipFree(h->ctap);
  if (h->ixz) (void)hipFree(h->ixz);
  if (h->partials) (void)hipFree(h->partials);
  if (h->dscal) (void)hipFree(h->dscal);
  if (h->work) (void)hipFree(h->work);
  if (h->chipseg) (void)hipFree(h->chipseg);
  for (auto& pool : h->ev)
    for (hipEvent_t ev : pool) (void)hipEventDestroy(ev);
  delete h;
  if (e != hipSuccess) return fail(SSF_E_DEVICE, std::string("stream error at destroy: ") + hipGetErrorString(e));
  return SSF_OK;
}

ssf_status ssf_set_stream(ssf_handle* h, void* hip_stream) {
  SSF_TRY(check_handle(h));
  h->stream = (hipStream_t)hip_stream;
  return SSF_OK;
}

ssf_status ssf_set_timing(ssf_handle* h, int32_t on) {
  SSF_TRY(check_handle(h));
  h->timing = on ? 1 : 0;
  for (auto& u : h->ev_used) u = 0;
  return SSF_OK;
}

ssf_status ssf_timing_read(ssf_handle* h, double* ms_total, int64_t* launches) {
  SSF_TRY(check_handle(h));
  if (!ms_total || !launches) return fail(SSF_E_INVALID, "null output arrays");
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int k = 0; k < ssf::NUM_PASS_KINDS; ++k) {
    double tot = 0.0;
    for (size_t i = 0; i < h->ev_used[k]; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev[k][2 * i], h->ev[k][2 * i + 1]));
      tot += ms;
    }
    ms_total[k] = tot;
    launches[k] = (int64_t)h->ev_used[k];
    h->ev_used[k] = 0;
  }
  return SSF_OK;
}

ssf_status ssf_set_tiles(ssf_handle* h, const int32_t* choice) {
  SSF_TRY(check_handle(h));
  if (!choice) return fail(SSF_E_INVALID, "null tile choice");
  for (int a = 1; a < 3; ++a)
    if (choice[a] < 0 || choice[a] >= ssf::NUM_STRIDED_VARIANTS) return fail(SSF_E_INVALID, "tile variant out of range");
  h->var[1] = choice[1];
  h->var[2] = choice[2];
  return SSF_OK;
}

ssf_status ssf_get_tiles(ssf_handle* h, int32_t* choice) {
  SSF_TRY(check_handle(h));
  if (!choice) return fail(SSF_E_INVALID, "null tile choice");
  for (int a = 0; a < 3; ++a) choice[a] = h->var[a];
  return SSF_OK;
}

ssf_status ssf_tune(ssf_handle* h, int32_t reps, int32_t* choice_out, double* us_out) {
  SSF_TRY(check_handle(h));
  if (reps < 1) return fail(SSF_E_INVALID, "reps must be >= 1");
  if (!h->work) HIP_TRY(hipMalloc(&h->work, h->esize * h->npts));
  HIP_TRY(hipMemsetAsync(h->work, 0, h->esize * h->npts, h->stream));
  const double2* kt = nullptr;
  SSF_TRY(get_ktab(h, 1e-3, 0, &kt));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int saved_timing = h->timing;
  h->timing = 0;
  ssf_status st = SSF_OK;
  for (int a = 1; a < 3 && st == SSF_OK; ++a) {
    double best = 1e300;
    int best_v = 0;
    for (int v = 0; v < ssf::NUM_STRIDED_VARIANTS && st == SSF_OK; ++v) {
      h->var[a] = v;
      PassArgs pa = base_args(h, h->work, h->work, a);
      int kind = ssf::STRIDED_FWD;
      if (a == 2) {
        kind = ssf::STRIDED_FUSED;
        pa.mid = ssf::MID_KINETIC;
        pa.kt[0] = kt;
        pa.kt[1] = kt + h->n[0];
        pa.kt[2] = kt + h->n[0] + h->n[1];
      }
      st = launch(h, kind, a, pa);                       // warm-up
      if (st != SSF_OK) break;
      if (hipEventRecord(e0, h->stream) != hipSuccess) { st = fail(SSF_E_DEVICE, "event record"); break; }
      for (int r = 0; r < reps && st == SSF_OK; ++r) st = launch(h, kind, a, pa);
      if (st != SSF_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(SSF_E_DEVICE, "event timing");
        break;
      }
      const double us = 1e3 * ms / reps;
      if (us_out) us_out[a * ssf::NUM_STRIDED_VARIANTS + v] = us;
      if (us < best) { best = us; best_v = v; }
    }
    h->var[a] = best_v;
  }
  h->timing = saved_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SSF_OK) { h->var[1] = h->var[2] = 0; return st; }
  if (choice_out)
    for (int a = 0; a < 3; ++a) choice_out[a] = h->var[a];
  return SSF_OK;
}

}  // extern "C"

namespace {

// Key of a tile choice in a tuning cache: the device architecture, the grid,
// the storage type and the arithmetic, and the number of tile variants the
// library has (a library with other variants starts over).
ssf_status tune_key(const ssf_handle* h, std::string* key) {
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, h->device));
  std::ostringstream k;
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  k << "ssf-tiles-v1 " << arch << " " << h->n[0] << "x" << h->n[1] << "x" << h->n[2] << " "
    << (h->dti == 0 ? "c64" : "c128") << " " << (h->kti == 2 ? "f32" : "f64") << " variants" << SSF_TILE_VARIANTS;
  *key = k.str();
  return SSF_OK;
}

}  // namespace

extern "C" {

ssf_status ssf_tune_cached(ssf_handle* h, int32_t reps, const char* cache_path, int32_t* choice_out, int32_t* hit) {
  SSF_TRY(check_handle(h));
  if (!cache_path || !*cache_path) return fail(SSF_E_INVALID, "cache path is empty");
  if (reps < 1) return fail(SSF_E_INVALID, "reps must be >= 1");
  std::string key;
  SSF_TRY(tune_key(h, &key));
  // a line is: <key> | <variant y> <variant z>; the last line with the key wins
  int found[2] = {-1, -1};
  {
    std::ifstream in(cache_path);
    std::string line;
    while (in && std::getline(in, line)) {
      const size_t bar = line.find(" | ");
      if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
      std::istringstream rest(line.substr(bar + 3));
      int vy = -1, vz = -1;
      if (rest >> vy >> vz && vy >= 0 && vy < SSF_TILE_VARIANTS && vz >= 0 && vz < SSF_TILE_VARIANTS) {
        found[0] = vy;
        found[1] = vz;
      }
    }
  }
  if (found[0] >= 0) {
    h->var[1] = found[0];
    h->var[2] = found[1];
    if (choice_out)
      for (int a = 0; a < 3; ++a) choice_out[a] = h->var[a];
    if (hit) *hit = 1;
    return SSF_OK;
  }
  int32_t choice[3] = {0, 0, 0};
  SSF_TRY(ssf_tune(h, reps, choice, nullptr));
  std::ofstream out(cache_path, std::ios::app);
  if (!out) return fail(SSF_E_INVALID, std::string("cannot append to the tuning cache ") + cache_path);
  std::ostringstream line;
  line << key << " | " << choice[1] << " " << choice[2] << "\n";
  out << line.str();
  out.flush();
  if (!out) return fail(SSF_E_INVALID, std::string("cannot write the tuning cache ") + cache_path);
  if (choice_out)
    for (int a = 0; a < 3; ++a) choice_out[a] = choice[a];
  if (hit) *hit = 0;
  return SSF_OK;
}

ssf_status ssf_set_fusion(ssf_handle* h, int32_t fuse_steps) {
  SSF_TRY(check_handle(h));
  h->fuse = fuse_steps ? 1 : 0;
  return SSF_OK;
}

ssf_status ssf_set_arithmetic(ssf_handle* h, int32_t arith) {
  SSF_TRY(check_handle(h));
  if (arith != SSF_ARITH_F64 && arith != SSF_ARITH_F32) return fail(SSF_E_INVALID, "unknown arithmetic mode");
  if (arith == SSF_ARITH_F32 && h->dti != 0)
    return fail(SSF_E_INVALID, "FP32 arithmetic needs complex64 storage");
  h->kti = arith == SSF_ARITH_F32 ? 2 : h->dti;
  return SSF_OK;
}

ssf_status ssf_set_splitting(ssf_handle* h, int32_t order) {
  SSF_TRY(check_handle(h));
  if (order != SSF_SPLIT_VTV && order != SSF_SPLIT_TVT) return fail(SSF_E_INVALID, "unknown splitting order");
  h->split = order;
  return SSF_OK;
}

ssf_status ssf_set_potential_table(ssf_handle* h, const void* v_dev, int32_t v_is_f64) {
  SSF_TRY(check_handle(h));
  if (!v_dev) return fail(SSF_E_INVALID, "potential table is null");
  h->vkind = v_is_f64 ? ssf::V_TAB64 : ssf::V_TAB32;
  h->vtab = v_dev;
  return SSF_OK;
}

ssf_status ssf_clear_potential(ssf_handle* h) {
  SSF_TRY(check_handle(h));
  h->vkind = ssf::V_NONE;
  h->vtab = nullptr;
  return SSF_OK;
}

ssf_status ssf_set_potential_ctap(ssf_handle* h, const ssf_ctap_desc* d) {
  SSF_TRY(check_handle(h));
  if (!d || !d->xc) return fail(SSF_E_INVALID, "null guide description");
  if (d->nguides < 1 || d->nguides > ssf::MAX_GUIDES) return fail(SSF_E_INVALID, "nguides must be 1..3");
  for (int g = 0; g < d->nguides; ++g)
    if (!(d->sigma[g] > 0.0) || !std::isfinite(d->v0[g])) return fail(SSF_E_INVALID, "sigma must be > 0, v0 finite");
  std::vector<double> tab;
  const double vmax = ctap_tables(h, d, tab);
  if (h->ctap) { HIP_TRY(hipStreamSynchronize(h->stream)); (void)hipFree(h->ctap); h->ctap = nullptr; }
  HIP_TRY(hipMalloc(&h->ctap, sizeof(double) * tab.size()));
  HIP_TRY(hipMemcpy(h->ctap, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
  h->nguides = d->nguides;
  h->vmax = vmax;
  h->vkind = ssf::V_CTAP;
  h->vtab = nullptr;
  return SSF_OK;
}

ssf_status ssf_chip_potential(ssf_handle* h, const ssf_chip_desc* d, double* V_dev) {
  SSF_TRY(check_handle(h));
  if (!d || !V_dev) return fail(SSF_E_INVALID, "null chip description or output");
  if (((uintptr_t)V_dev) % sizeof(double) != 0) return fail(SSF_E_INVALID, "V_dev is not aligned to 8 bytes");
  if (d->nwires < 1 || d->nwires > SSF_CHIP_MAX_WIRES || !d->npts || !d->path || !d->current)
    return fail(SSF_E_INVALID, "chip needs 1..16 wires with point counts, paths and currents");
  if (!(d->length_unit > 0.0) || !std::isfinite(d->length_unit))
    return fail(SSF_E_INVALID, "length_unit must be positive");
  if (!std::isfinite(d->b_bias) || !std::isfinite(d->b_ip) || !(d->b_ip >= 0.0) || !std::isfinite(d->mu_over_e0) ||
      !std::isfinite(d->omega_z) || !std::isfinite(d->z_c))
    return fail(SSF_E_INVALID, "chip fields, moment and trap must be finite (b_ip >= 0)");
  // straight segments between consecutive points of every wire
  std::vector<ChipSeg> seg;
  const double k0 = 1.25663706212e-6 / (4.0 * 3.14159265358979323846) / d->length_unit;
  long long off = 0;
  for (int w = 0; w < d->nwires; ++w) {
    const int np = d->npts[w];
    if (np < 2) return fail(SSF_E_INVALID, "every wire needs at least 2 points");
    if (!std::isfinite(d->current[w])) return fail(SSF_E_INVALID, "currents must be finite");
    for (int q = 0; q + 1 < np; ++q) {
      const double* A = d->path + 2 * (off + q);
      ChipSeg c;
      c.ax = A[0];
      c.az = A[1];
      c.lx = A[2] - A[0];
      c.lz = A[3] - A[1];
      c.kI = k0 * d->current[w];
      c.pad = 0.0;
      if (!std::isfinite(c.ax) || !std::isfinite(c.az) || !std::isfinite(c.lx) || !std::isfinite(c.lz))
        return fail(SSF_E_INVALID, "wire points must be finite");
      seg.push_back(c);
    }
    off += np;
  }
  if (seg.size() > h->chipseg_cap) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->chipseg) (void)hipFree(h->chipseg);
    h->chipseg = nullptr;
    h->chipseg_cap = 0;
    HIP_TRY(hipMalloc(&h->chipseg, sizeof(ChipSeg) * seg.size()));
    h->chipseg_cap = seg.size();
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(h->chipseg, seg.data(), sizeof(ChipSeg) * seg.size(), hipMemcpyHostToDevice));
  const long long blocks = ceil_div(h->npts, 256);
  hipLaunchKernelGGL(chip_kernel, dim3((unsigned)blocks), dim3(256), 0, h->stream, V_dev, h->n[0], h->n[1], h->n[2],
                     h->lo[0], h->lo[1], h->lo[2], h->d[0], h->d[1], h->d[2], h->chipseg, (int)seg.size(), d->b_bias,
                     d->b_ip, d->mu_over_e0, d->omega_z, d->z_c);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

ssf_status ssf_set_partition(ssf_handle* h, double x_lo, double x_hi) {
  SSF_TRY(check_handle(h));
  if (!(x_lo <= x_hi)) return fail(SSF_E_INVALID, "partition needs x_lo <= x_hi");
  int ilo = 0, ihi = 0;
  partition_indices(h, x_lo, x_hi, &ilo, &ihi);
  h->ix_lo = ilo;
  h->ix_hi = ihi;
  h->zpart = 0;
  return SSF_OK;
}

ssf_status ssf_set_partition_z(ssf_handle* h, const double* x_lo, const double* x_hi) {
  SSF_TRY(check_handle(h));
  if (!x_lo || !x_hi) return fail(SSF_E_INVALID, "null boundary arrays");
  const int nz = h->n[2];
  std::vector<int> ix(2 * (size_t)nz);
  for (int z = 0; z < nz; ++z) {
    if (!(x_lo[z] <= x_hi[z])) return fail(SSF_E_INVALID, "partition needs x_lo[z] <= x_hi[z]");
    partition_indices(h, x_lo[z], x_hi[z], &ix[2 * z], &ix[2 * z + 1]);
  }
  if (!h->ixz) HIP_TRY(hipMalloc(&h->ixz, sizeof(int) * ix.size()));
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(h->ixz, ix.data(), sizeof(int) * ix.size(), hipMemcpyHostToDevice));
  h->zpart = 1;
  return SSF_OK;
}

ssf_status ssf_fft(ssf_handle* h, void* psi, int32_t axis_mask, int32_t inverse) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, psi, "psi"));
  for (int a = 0; a < 3; ++a) {
    if (!(axis_mask & (1 << a))) continue;
    PassArgs pa = base_args(h, psi, psi, a);
    const int kind = a == 0 ? (inverse ? ssf::CONTIG_INV : ssf::CONTIG_FWD)
                            : (inverse ? ssf::STRIDED_INV : ssf::STRIDED_FWD);
    SSF_TRY(launch(h, kind, a, pa));
  }
  return SSF_OK;
}

static ssf_status run_steps(ssf_handle* h, const void* src, void* psi, int64_t nsteps, double dt, int imag,
                            int64_t obs_every, ssf_obs* obs_dev, bool allow_fuse) {
  const double2* kt = nullptr;
  SSF_TRY(get_ktab(h, dt, imag, &kt));
  if (imag) {
    // scale the input to norm 1 first
    SSF_TRY(reduce_field(h, src));
    SSF_TRY(finalize_obs(h, nullptr, 0, 2, dt, nullptr, 0));
  }
  // Imaginary time renormalises after every step.  Unfused, each step ends
  // with the x inverse pass summing the norm and the next x forward pass
  // applies 1/norm^(1/2) on load.  Fused, the x pass between two steps sums
  // the norm between its two potential half-steps (MID_VNORM) and the scale
  // goes onto the input of the next x pass (every operation in between is
  // linear), so a step costs the same four passes as in real time.
  const bool fuse = allow_fuse && h->fuse;
  int64_t s = 0;
  const void* cur_in = src;
  while (s < nsteps) {
    // chain start: x forward with exp(-i V dt/2) on load
    PassArgs ax = base_args(h, cur_in, psi, 0);
    ax.pre = ssf::PRE_VPHASE | (imag ? ssf::PRE_SCALE : 0);
    ax.cpre = 0.5 * dt;
    ax.imag = imag;
    SSF_TRY(launch(h, ssf::CONTIG_FWD, 0, ax));
    cur_in = psi;
    bool scaled = true;            // imaginary time: the field in flight carries the latest scale
    for (;;) {
      SSF_TRY(step_middle(h, psi, kt));
      ++s;
      const bool obs_due = obs_every > 0 && obs_dev && (s % obs_every) == 0;
      const bool end = !fuse || s == nsteps || obs_due;
      if (end) {
        PassArgs ai = base_args(h, psi, psi, 0);
        ai.pre = (imag && !scaled) ? ssf::PRE_SCALE : 0;
        ai.post = ssf::POST_VPHASE | ((obs_due || imag) ? ssf::POST_OBS : 0);
        ai.cpost = 0.5 * dt;
        ai.imag = imag;
        SSF_TRY(launch(h, ssf::CONTIG_INV, 0, ai));
        if (obs_due || imag) {
          ssf_obs* slot = obs_due ? obs_dev + (s / obs_every - 1) : nullptr;
          SSF_TRY(finalize_obs(h, slot, s, (obs_due ? 1 : 0) | (imag ? 2 : 0), dt, nullptr, 0));
        }
        break;
      }
      PassArgs am = base_args(h, psi, psi, 0);
      am.imag = imag;
      if (imag) {
        am.mid = ssf::MID_VNORM;
        am.cmid = 0.5 * dt;
        am.pre = scaled ? 0 : ssf::PRE_SCALE;
        SSF_TRY(launch(h, ssf::CONTIG_FUSED, 0, am));
        SSF_TRY(finalize_obs(h, nullptr, s, 2, dt, nullptr, 0));
        scaled = false;
      } else {
        am.mid = ssf::MID_VPHASE;
        am.cmid = dt;
        // |V dt| <= pi/4 lets the phase skip its argument reduction
        am.small_phase = phase_tier(h->vkind, h->vmax, dt);
        SSF_TRY(launch(h, ssf::CONTIG_FUSED, 0, am));
      }
    }
  }
  if (imag && nsteps > 0) SSF_TRY(scale_field(h, psi));
  return SSF_OK;
}

// Real-time steps in the T/2 - V - T/2 ordering.  A chain is x forward, a
// half kinetic step (y, z-fused, y), then per step the fused x pass with
// exp(-i V dt) followed by a full kinetic step, except that the last step of
// the chain ends with a half kinetic step and the x inverse (with the
// observation reduction when one is due).  The 1/N of the unnormalised
// transforms is in every z kinetic table, full or half, one per x round trip.
static ssf_status run_steps_tvt(ssf_handle* h, void* psi, int64_t nsteps, double dt, int64_t obs_every,
                                ssf_obs* obs_dev) {
  const double2 *kt = nullptr, *kh = nullptr;
  SSF_TRY(get_ktab(h, dt, 0, &kt));
  SSF_TRY(get_ktab(h, 0.5 * dt, 0, &kh));
  int64_t s = 0;
  while (s < nsteps) {
    PassArgs ax = base_args(h, psi, psi, 0);
    SSF_TRY(launch(h, ssf::CONTIG_FWD, 0, ax));
    SSF_TRY(step_middle(h, psi, kh));
    for (;;) {
      PassArgs am = base_args(h, psi, psi, 0);
      am.mid = ssf::MID_VPHASE;
      am.cmid = dt;
      am.small_phase = phase_tier(h->vkind, h->vmax, dt);
      SSF_TRY(launch(h, ssf::CONTIG_FUSED, 0, am));
      ++s;
      const bool obs_due = obs_every > 0 && obs_dev && (s % obs_every) == 0;
      if (!h->fuse || s == nsteps || obs_due) {
        SSF_TRY(step_middle(h, psi, kh));
        PassArgs ai = base_args(h, psi, psi, 0);
        ai.post = obs_due ? ssf::POST_OBS : 0;
        SSF_TRY(launch(h, ssf::CONTIG_INV, 0, ai));
        if (obs_due) SSF_TRY(finalize_obs(h, obs_dev + (s / obs_every - 1), s, 1, dt, nullptr, 0));
        break;
      }
      SSF_TRY(step_middle(h, psi, kt));
    }
  }
  return SSF_OK;
}

static ssf_status check_step_args(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time,
                                  int64_t obs_every) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, psi, "psi"));
  if (nsteps < 0) return fail(SSF_E_INVALID, "nsteps must be >= 0");
  if (time != SSF_REAL && time != SSF_IMAG) return fail(SSF_E_INVALID, "time must be SSF_REAL or SSF_IMAG");
  if (!std::isfinite(dt) || dt == 0.0) return fail(SSF_E_INVALID, "dt must be finite and nonzero");
  if (time == SSF_IMAG && dt < 0.0) return fail(SSF_E_INVALID, "imaginary time needs dt > 0");
  if (obs_every < 0) return fail(SSF_E_INVALID, "obs_every must be >= 0");
  if (time == SSF_IMAG && h->split == SSF_SPLIT_TVT)
    return fail(SSF_E_UNSUPPORTED, "imaginary time uses the V/2-T-V/2 ordering");
  return SSF_OK;
}

static ssf_status dispatch_steps(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time, int64_t obs_every,
                                 ssf_obs* obs_dev) {
  if (h->split == SSF_SPLIT_TVT) return run_steps_tvt(h, psi, nsteps, dt, obs_every, obs_dev);
  return run_steps(h, psi, psi, nsteps, dt, time == SSF_IMAG ? 1 : 0, obs_every, obs_dev, true);
}

ssf_status ssf_step(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time, int64_t obs_every,
                    ssf_obs* obs_dev) {
  SSF_TRY(check_step_args(h, psi, nsteps, dt, time, obs_every));
  if (nsteps == 0) return SSF_OK;
  return dispatch_steps(h, psi, nsteps, dt, time, obs_every, obs_dev);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free steps.  Everything a step sequence writes besides the field
// and the observation records -- the kinetic tables of its dt (two for the
// T/2-V-T/2 ordering), the FP64 partial sums of the reducing passes and the
// device scale of imaginary time -- lives in one static device array per
// device instead of in handle memory allocated on demand.  Host code never
// uses the array's name as an address: its device address is looked up once
// per device and kept in scratch_dev[].
// ---------------------------------------------------------------------------
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of this device's scratch array (the device must be current).
ssf_status scratch_address(int device, char** out) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return fail(SSF_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SSF_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    scratch_dev[device] = (char*)p;
  }
  *out = scratch_dev[device];
  return SSF_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch layout of one call: [device scalars | 2 kinetic tables | partials].
size_t scratch_need(const ssf_handle* h, size_t* kt_off, size_t* part_off) {
  *kt_off = 256;
  *part_off = *kt_off + round256(2 * sizeof(double2) * (size_t)(h->n[0] + h->n[1] + h->n[2]));
  return *part_off + sizeof(double) * ssf::NRED_OBS * (size_t)h->part_cap;
}

}  // namespace

extern "C" {

int64_t ssf_noalloc_scratch_bytes(void) { return (int64_t)SCRATCH_BYTES; }

int64_t ssf_noalloc_scratch_need(ssf_handle* h) {
  if (!h) return -1;
  size_t a, b;
  return (int64_t)scratch_need(h, &a, &b);
}

ssf_status ssf_step_noalloc(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time, int64_t obs_every,
                            ssf_obs* obs_dev) {
  SSF_TRY(check_step_args(h, psi, nsteps, dt, time, obs_every));
  size_t kt_off, part_off;
  const size_t need = scratch_need(h, &kt_off, &part_off);
  if (need > SCRATCH_BYTES)
    return fail(SSF_E_INVALID, "grid too large for the allocation-free step: it needs " + std::to_string(need) +
                                   " bytes of scratch, the maximum is " + std::to_string(SCRATCH_BYTES));
  char* base = nullptr;
  SSF_TRY(scratch_address(h->device, &base));
  if (nsteps == 0) return SSF_OK;
  // point the handle's per-call buffers into the scratch for this call only;
  // per-pass timing would create events, so it is off for the call
  double* const saved_partials = h->partials;
  double* const saved_dscal = h->dscal;
  const int saved_timing = h->timing;
  h->dscal = (double*)base;
  h->ktfix = (double2*)(base + kt_off);
  h->ktfix_used = 0;
  h->partials = (double*)(base + part_off);
  h->timing = 0;
  const ssf_status st = dispatch_steps(h, psi, nsteps, dt, time, obs_every, obs_dev);
  h->partials = saved_partials;
  h->dscal = saved_dscal;
  h->ktfix = nullptr;
  h->ktfix_used = 0;
  h->timing = saved_timing;
  return st;
}

ssf_status ssf_observables(ssf_handle* h, const void* psi, ssf_obs* obs_dev) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, psi, "psi"));
  if (!obs_dev) return fail(SSF_E_INVALID, "obs_dev is null");
  if (!h->work) HIP_TRY(hipMalloc(&h->work, h->esize * h->npts));
  HIP_TRY(hipMemcpyAsync(h->work, psi, h->esize * h->npts, hipMemcpyDeviceToDevice, h->stream));
  // kinetic part into the second partial region
  double* kin = h->partials + 8 * h->part_cap;
  PassArgs ax = base_args(h, h->work, h->work, 0);
  SSF_TRY(launch(h, ssf::CONTIG_FWD, 0, ax));
  PassArgs ay = base_args(h, h->work, h->work, 1);
  SSF_TRY(launch(h, ssf::STRIDED_FWD, 1, ay));
  PassArgs az = base_args(h, h->work, h->work, 2);
  az.post = ssf::POST_KIN;
  az.partials = kin;
  SSF_TRY(launch(h, ssf::STRIDED_FWD, 2, az));
  SSF_TRY(reduce_field(h, psi));
  return finalize_obs(h, obs_dev, 0, 1, 0.0, kin, blocks_of(h, 2));
}

ssf_status ssf_obs_read(ssf_handle* h, const ssf_obs* obs_dev, ssf_obs* host, int64_t count) {
  SSF_TRY(check_handle(h));
  if (count < 0 || (count > 0 && (!obs_dev || !host))) return fail(SSF_E_INVALID, "bad observation buffers");
  if (count == 0) return SSF_OK;
  HIP_TRY(hipMemcpyAsync(host, obs_dev, sizeof(ssf_obs) * count, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int64_t i = 0; i < count; ++i)
    if (host[i].flags & 1) return fail(SSF_E_NONFINITE, "observation " + std::to_string(i) + " has a non-finite norm");
  return SSF_OK;
}

ssf_status ssf_density_xz(ssf_handle* h, const void* psi, double* out_dev) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, psi, "psi"));
  if (!out_dev) return fail(SSF_E_INVALID, "out_dev is null");
  const dim3 grid((unsigned)ceil_div(h->n[0], 256), (unsigned)h->n[2]);
  if (h->dti == 0)
    hipLaunchKernelGGL(density_xz_kernel<float2>, grid, dim3(256), 0, h->stream, (const float2*)psi, h->n[0], h->n[1],
                       h->d[1], out_dev);
  else
    hipLaunchKernelGGL(density_xz_kernel<double2>, grid, dim3(256), 0, h->stream, (const double2*)psi, h->n[0],
                       h->n[1], h->d[1], out_dev);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

ssf_status ssf_sync(ssf_handle* h) {
  SSF_TRY(check_handle(h));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return SSF_OK;
}

ssf_status ssf_copy(ssf_handle* h, const void* src, void* dst) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, src, "src"));
  SSF_TRY(check_field(h, dst, "dst"));
  const size_t fb = h->esize * h->npts;
  const char* a = (const char*)src;
  const char* b = (const char*)dst;
  if (a < b + fb && b < a + fb) return fail(SSF_E_INVALID, "src and dst overlap");
  const long long n = h->npts;
  const unsigned grid = (unsigned)std::min<long long>(ceil_div(n, 256), 1LL << 20);
  if (h->dtype == SSF_C64)
    hipLaunchKernelGGL(copy_kernel<float2>, dim3(grid), dim3(256), 0, h->stream, (const float2*)src, (float2*)dst, n);
  else
    hipLaunchKernelGGL(copy_kernel<double2>, dim3(grid), dim3(256), 0, h->stream, (const double2*)src, (double2*)dst, n);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

ssf_status ssf_step_ckpt(ssf_handle* h, void* psi, int64_t nsteps, double dt, int64_t every, void* ckpt_dev) {
  SSF_TRY(check_handle(h));
  if (h->split != SSF_SPLIT_VTV) return fail(SSF_E_UNSUPPORTED, "checkpoints and the adjoint use the V/2-T-V/2 ordering");
  SSF_TRY(check_field(h, psi, "psi"));
  SSF_TRY(check_field(h, ckpt_dev, "ckpt_dev"));
  if (nsteps < 0 || every < 1) return fail(SSF_E_INVALID, "need nsteps >= 0 and every >= 1");
  if (!std::isfinite(dt) || dt == 0.0) return fail(SSF_E_INVALID, "dt must be finite and nonzero");
  const size_t fb = h->esize * h->npts;
  for (int64_t s = 0, slot = 0; s < nsteps; s += every, ++slot) {
    HIP_TRY(hipMemcpyAsync((char*)ckpt_dev + slot * fb, psi, fb, hipMemcpyDeviceToDevice, h->stream));
    SSF_TRY(run_steps(h, psi, psi, std::min<int64_t>(every, nsteps - s), dt, 0, 0, nullptr, false));
  }
  return SSF_OK;
}

ssf_status ssf_step_seq(ssf_handle* h, const void* psi0, int64_t nsteps, double dt, void* seq_dev) {
  SSF_TRY(check_handle(h));
  if (h->split != SSF_SPLIT_VTV) return fail(SSF_E_UNSUPPORTED, "checkpoints and the adjoint use the V/2-T-V/2 ordering");
  SSF_TRY(check_field(h, psi0, "psi0"));
  SSF_TRY(check_field(h, seq_dev, "seq_dev"));
  if (nsteps < 0) return fail(SSF_E_INVALID, "nsteps must be >= 0");
  if (!std::isfinite(dt) || dt == 0.0) return fail(SSF_E_INVALID, "dt must be finite and nonzero");
  const size_t fb = h->esize * h->npts;
  char* seq = (char*)seq_dev;
  HIP_TRY(hipMemcpyAsync(seq, psi0, fb, hipMemcpyDeviceToDevice, h->stream));
  for (int64_t s = 0; s < nsteps; ++s)
    SSF_TRY(run_steps(h, seq + s * fb, seq + (s + 1) * fb, 1, dt, 0, 0, nullptr, false));
  return SSF_OK;
}

ssf_status ssf_adjoint_init(ssf_handle* h, const void* psi, void* lambda) {
  SSF_TRY(check_handle(h));
  SSF_TRY(check_field(h, psi, "psi"));
  SSF_TRY(check_field(h, lambda, "lambda"));
  const unsigned blocks = (unsigned)std::min<long long>(ceil_div(h->npts, 256), 65536);
  if (h->dti == 0)
    hipLaunchKernelGGL(mask_kernel<float2>, dim3(blocks), dim3(256), 0, h->stream, (const float2*)psi, (float2*)lambda,
                       h->npts, h->n[0], (long long)h->n[0] * h->n[1], h->ix_hi, h->zpart ? h->ixz : nullptr);
  else
    hipLaunchKernelGGL(mask_kernel<double2>, dim3(blocks), dim3(256), 0, h->stream, (const double2*)psi,
                       (double2*)lambda, h->npts, h->n[0], (long long)h->n[0] * h->n[1], h->ix_hi,
                       h->zpart ? h->ixz : nullptr);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

ssf_status ssf_adjoint_segment(ssf_handle* h, void* lambda, const void* seq_dev, int64_t nsteps, double dt,
                               double* G_dev) {
  SSF_TRY(check_handle(h));
  if (h->split != SSF_SPLIT_VTV) return fail(SSF_E_UNSUPPORTED, "checkpoints and the adjoint use the V/2-T-V/2 ordering");
  SSF_TRY(check_field(h, lambda, "lambda"));
  SSF_TRY(check_field(h, seq_dev, "seq_dev"));
  if (!G_dev) return fail(SSF_E_INVALID, "G_dev is null");
  if (h->vkind != ssf::V_CTAP) return fail(SSF_E_INVALID, "the adjoint needs the guide potential (ssf_set_potential_ctap)");
  if (nsteps < 0) return fail(SSF_E_INVALID, "nsteps must be >= 0");
  if (!std::isfinite(dt) || dt == 0.0) return fail(SSF_E_INVALID, "dt must be finite and nonzero");
  const double2* kt = nullptr;
  SSF_TRY(get_ktab(h, -dt, 0, &kt));
  const size_t fb = h->esize * h->npts;
  const char* seq = (const char*)seq_dev;
  const dim3 gx = pass_grid(h, 0);
  const double w = dt * h->dv;
  const int nzg = h->n[2] * h->nguides;
  for (int64_t s = nsteps - 1; s >= 0; --s) {
    // second potential half-step of step s: Im(conj(lambda_{s+1}) psi_{s+1}) on load, then A^dagger
    PassArgs ax = base_args(h, lambda, lambda, 0);
    ax.pre = ssf::PRE_ADJ | ssf::PRE_VPHASE;
    ax.cpre = -0.5 * dt;
    ax.aux = seq + (s + 1) * fb;
    SSF_TRY(launch(h, ssf::CONTIG_FWD, 0, ax));
    hipLaunchKernelGGL(adj_finalize, dim3((unsigned)ceil_div(nzg, 256)), dim3(256), 0, h->stream, h->partials,
                       (int)gx.x, h->n[2], h->nguides, w, G_dev);
    HIP_TRY(hipGetLastError());
    SSF_TRY(step_middle(h, lambda, kt));
    // first potential half-step of step s: A^dagger, then Im(conj(lambda_s) psi_s) on store
    PassArgs ai = base_args(h, lambda, lambda, 0);
    ai.post = ssf::POST_VPHASE | ssf::POST_ADJ;
    ai.cpost = -0.5 * dt;
    ai.aux = seq + s * fb;
    SSF_TRY(launch(h, ssf::CONTIG_INV, 0, ai));
    hipLaunchKernelGGL(adj_finalize, dim3((unsigned)ceil_div(nzg, 256)), dim3(256), 0, h->stream, h->partials,
                       (int)gx.x, h->n[2], h->nguides, w, G_dev);
    HIP_TRY(hipGetLastError());
  }
  return SSF_OK;
}

ssf_status ssf_profile_grad(ssf_handle* h, const double* G_dev, int32_t nguides, const double* B_dev, int32_t M,
                            double* out_dev) {
  SSF_TRY(check_handle(h));
  if (!G_dev || !B_dev || !out_dev || M < 1 || nguides < 1 || nguides > ssf::MAX_GUIDES)
    return fail(SSF_E_INVALID, "bad profile gradient arguments");
  const int n = nguides * M;
  hipLaunchKernelGGL(profile_grad_kernel, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, h->stream, G_dev, B_dev, h->n[2],
                     M, nguides, out_dev);
  HIP_TRY(hipGetLastError());
  return SSF_OK;
}

}  // extern "C"

namespace {

// Clamped uniform cubic knots over [a, b] with M basis functions.
std::vector<double> bspline_knots(int M, double a, double b) {
  const int nk = M + 4, nseg = M - 3;
  std::vector<double> t(nk);
  for (int i = 0; i < 4; ++i) { t[i] = a; t[nk - 1 - i] = b; }
  for (int i = 1; i < nseg; ++i) t[3 + i] = a + (b - a) * (double)i / (double)nseg;
  return t;
}

// The M basis functions at u (row[0..M-1]): the knot span, then the de Boor
// triangle of its 4 nonzero functions.
void bspline_row(const std::vector<double>& t, int M, double b, double u, double* row) {
  for (int m = 0; m < M; ++m) row[m] = 0.0;
  if (u >= b) {
    row[M - 1] = 1.0;
    return;
  }
  int span = 3;
  while (span < M - 1 && u >= t[span + 1]) ++span;
  double Nl[4] = {1.0, 0.0, 0.0, 0.0};
  double left[4], right[4];
  for (int d = 1; d <= 3; ++d) {
    left[d] = u - t[span + 1 - d];
    right[d] = t[span + d] - u;
    double saved = 0.0;
    for (int r = 0; r < d; ++r) {
      const double den = right[r + 1] + left[d - r];
      const double tmp = den > 0.0 ? Nl[r] / den : 0.0;
      Nl[r] = saved + right[r + 1] * tmp;
      saved = left[d - r] * tmp;
    }
    Nl[d] = saved;
  }
  for (int r = 0; r < 4; ++r) {
    const int m = span - 3 + r;
    if (m >= 0 && m < M) row[m] = Nl[r];
  }
}

}  // namespace

extern "C" {

ssf_status ssf_bspline_basis(int32_t M, double a, double b, const double* z, int32_t nz, double* B_out) {
  if (M < 4 || !(b > a) || nz < 0 || (nz > 0 && (!z || !B_out))) return fail(SSF_E_INVALID, "bad B-spline arguments");
  const std::vector<double> t = bspline_knots(M, a, b);
  for (int iz = 0; iz < nz; ++iz) bspline_row(t, M, b, z[iz], B_out + (long long)iz * M);
  return SSF_OK;
}

ssf_status ssf_bspline_eval(int32_t M, double a, double b, const double* coeffs, int32_t nsets, const double* z,
                            int32_t nz, double* out) {
  if (M < 4 || !(b > a) || nz < 0 || nsets < 0 || (nz > 0 && nsets > 0 && (!z || !out || !coeffs)))
    return fail(SSF_E_INVALID, "bad B-spline arguments");
  const std::vector<double> t = bspline_knots(M, a, b);
  std::vector<double> row(M);
  for (int iz = 0; iz < nz; ++iz) {
    bspline_row(t, M, b, z[iz], row.data());
    for (int k = 0; k < nsets; ++k) {
      double v = 0.0;
      for (int m = 0; m < M; ++m) v += coeffs[(long long)k * M + m] * row[m];
      out[(long long)k * nz + iz] = v;
    }
  }
  return SSF_OK;
}

// ---------------------------------------------------------------------------
// Batched instances (parameter sweeps).  Instances with the same grid form a
// group: one handle (twiddles, kinetic tables, tile choice), per-instance
// guide tables and a device descriptor array.  Every pass of a step is one
// persistent launch over all tiles of all instances of the group; groups run
// concurrently on their own streams, and a chunk of steps is captured in a
// HIP graph (fork/join over the group streams) that is replayed.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct BatchGroup {
  ssf_handle* h = nullptr;
  std::vector<int> members;            // global instance indices
  ssf::InstDesc* d_inst = nullptr;     // device descriptors
  std::vector<ssf::InstDesc> inst;     // host copy
  int* d_slot = nullptr;               // device: members
  std::vector<double*> ctap;           // per-instance guide tables (device)
  double vmax = 0.0;
  double* obs_part = nullptr;          // observation partials, instance-major
  long long obs_blocks = 0;            // per instance
  hipStream_t stream = nullptr;
  hipEvent_t join = nullptr;
};

}  // namespace

struct ssf_batch {
  int count = 0, dtype = 0, device = 0;
  int vkind = ssf::V_CTAP;             // guide tables, or borrowed FP64 potential tables (V_TAB64)
  hipStream_t user = nullptr, cap = nullptr;
  hipEvent_t ev_start = nullptr, ev_fork = nullptr, ev_done = nullptr;
  std::vector<BatchGroup> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_dt = 0.0;
  int64_t graph_k = 0;
  std::vector<const double2*> graph_kt;   // kinetic tables the graph reads
};

namespace {

PassArgs batch_args(BatchGroup& G, int axis, int vkind) {
  PassArgs a = base_args(G.h, nullptr, nullptr, axis);
  a.inst = G.d_inst;
  a.ninst = (int)G.members.size();
  a.vkind = vkind;
  a.vtab = nullptr;
  a.nguides = ssf::MAX_GUIDES;
  return a;
}

// k real-time Strang steps of every instance of the group (fused chain:
// x forward with the half potential phase, k x (y, z, y) with the fused x
// pass between steps, x inverse with the half phase).
ssf_status batch_chunk(BatchGroup& G, int vkind, int64_t k, double dt, const double2* kt) {
  ssf_handle* h = G.h;
  PassArgs ax = batch_args(G, 0, vkind);
  ax.pre = ssf::PRE_VPHASE;
  ax.cpre = 0.5 * dt;
  SSF_TRY(launch(h, ssf::CONTIG_FWD, 0, ax));
  for (int64_t s = 1; s <= k; ++s) {
    PassArgs ay = batch_args(G, 1, vkind);
    SSF_TRY(launch(h, ssf::STRIDED_FWD, 1, ay));
    PassArgs az = batch_args(G, 2, vkind);
    az.mid = ssf::MID_KINETIC;
    az.kt[0] = kt;
    az.kt[1] = kt + h->n[0];
    az.kt[2] = kt + h->n[0] + h->n[1];
    SSF_TRY(launch(h, ssf::STRIDED_FUSED, 2, az));
    SSF_TRY(launch(h, ssf::STRIDED_INV, 1, ay));
    PassArgs am = batch_args(G, 0, vkind);
    if (s < k) {
      am.mid = ssf::MID_VPHASE;
      am.cmid = dt;
      am.small_phase = phase_tier(vkind, G.vmax, dt);
      SSF_TRY(launch(h, ssf::CONTIG_FUSED, 0, am));
    } else {
      am.post = ssf::POST_VPHASE;
      am.cpost = 0.5 * dt;
      SSF_TRY(launch(h, ssf::CONTIG_INV, 0, am));
    }
  }
  return SSF_OK;
}

ssf_status batch_fork(ssf_batch* b) {
  HIP_TRY(hipEventRecord(b->ev_fork, b->cap));
  for (auto& G : b->groups) HIP_TRY(hipStreamWaitEvent(G.stream, b->ev_fork, 0));
  return SSF_OK;
}

ssf_status batch_join(ssf_batch* b) {
  for (auto& G : b->groups) {
    HIP_TRY(hipEventRecord(G.join, G.stream));
    HIP_TRY(hipStreamWaitEvent(b->cap, G.join, 0));
  }
  return SSF_OK;
}

ssf_status batch_chunks_all(ssf_batch* b, int64_t k, double dt, const std::vector<const double2*>& kts) {
  SSF_TRY(batch_fork(b));
  for (size_t i = 0; i < b->groups.size(); ++i) SSF_TRY(batch_chunk(b->groups[i], b->vkind, k, dt, kts[i]));
  return batch_join(b);
}

void batch_free(ssf_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& G : b->groups) {
    if (G.stream) (void)hipStreamSynchronize(G.stream);
    for (double* c : G.ctap) if (c) (void)hipFree(c);
    if (G.d_inst) (void)hipFree(G.d_inst);
    if (G.d_slot) (void)hipFree(G.d_slot);
    if (G.obs_part) (void)hipFree(G.obs_part);
    if (G.join) (void)hipEventDestroy(G.join);
    if (G.h) { G.h->stream = G.stream; (void)ssf_destroy(G.h); }
    if (G.stream) (void)hipStreamDestroy(G.stream);
  }
  if (b->ev_start) (void)hipEventDestroy(b->ev_start);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_done) (void)hipEventDestroy(b->ev_done);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

bool same_grid(const ssf_grid_desc& a, const ssf_grid_desc& c) {
  for (int q = 0; q < 3; ++q)
    if (a.n[q] != c.n[q] || a.lo[q] != c.lo[q] || a.hi[q] != c.hi[q]) return false;
  return true;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Batch of instances with guide potentials (guides != nullptr) or borrowed
// FP64 potential tables (vtabs != nullptr).
ssf_status batch_create(int32_t count, const ssf_grid_desc* grids, const ssf_ctap_desc* guides,
                        const double* const* vtabs, const double* x_lo, const double* x_hi, int32_t dtype,
                        void* hip_stream, ssf_batch** out) {
  if (!out || count < 1 || !grids || (!guides == !vtabs) || !x_lo || !x_hi)
    return fail(SSF_E_INVALID, "bad batch arguments");
  *out = nullptr;
  if (dtype != SSF_C64 && dtype != SSF_C128) return fail(SSF_E_INVALID, "dtype must be SSF_C64 or SSF_C128");
  ssf_batch* b = new ssf_batch();
  b->count = count;
  b->dtype = dtype;
  b->vkind = vtabs ? ssf::V_TAB64 : ssf::V_CTAP;
  b->user = (hipStream_t)hip_stream;
  if (hipGetDevice(&b->device) != hipSuccess) { delete b; return fail(SSF_E_NODEVICE, "no HIP device"); }
  auto bail = [&](ssf_status st) { batch_free(b); return st; };
  std::vector<ssf_grid_desc> keys;
  std::vector<int> gid(count);
  for (int i = 0; i < count; ++i) {
    int g = -1;
    for (size_t j = 0; j < keys.size(); ++j)
      if (same_grid(keys[j], grids[i])) { g = (int)j; break; }
    if (g < 0) { keys.push_back(grids[i]); g = (int)keys.size() - 1; }
    gid[i] = g;
  }
  b->groups.resize(keys.size());
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming) != hipSuccess)
    return bail(fail(SSF_E_DEVICE, "batch streams/events"));
  for (size_t j = 0; j < keys.size(); ++j) {
    BatchGroup& G = b->groups[j];
    if (hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&G.join, hipEventDisableTiming) != hipSuccess)
      return bail(fail(SSF_E_DEVICE, "group stream/event"));
    ssf_status st = ssf_create(&keys[j], dtype, G.stream, &G.h);
    if (st != SSF_OK) return bail(st);
  }
  for (int i = 0; i < count; ++i) {
    BatchGroup& G = b->groups[gid[i]];
    if (!(x_lo[i] <= x_hi[i])) return bail(fail(SSF_E_INVALID, "partition needs x_lo <= x_hi"));
    ssf::InstDesc id;
    std::memset(&id, 0, sizeof(id));
    partition_indices(G.h, x_lo[i], x_hi[i], &id.ix_lo, &id.ix_hi);
    if (vtabs) {
      if (!vtabs[i] || ((uintptr_t)vtabs[i]) % sizeof(double) != 0)
        return bail(fail(SSF_E_INVALID, "potential table null or misaligned"));
      id.vtab = vtabs[i];
      G.inst.push_back(id);
      G.members.push_back(i);
      continue;
    }
    const ssf_ctap_desc* d = &guides[i];
    if (!d->xc || d->nguides < 1 || d->nguides > ssf::MAX_GUIDES) return bail(fail(SSF_E_INVALID, "bad guide description"));
    for (int q = 0; q < d->nguides; ++q)
      if (!(d->sigma[q] > 0.0) || !std::isfinite(d->v0[q])) return bail(fail(SSF_E_INVALID, "sigma must be > 0"));
    std::vector<double> tab;
    const double vm = ctap_tables(G.h, d, tab);
    double* dev = nullptr;
    if (hipMalloc(&dev, sizeof(double) * tab.size()) != hipSuccess) return bail(fail(SSF_E_NOMEM, "guide tables"));
    G.ctap.push_back(dev);
    if (hipMemcpy(dev, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(SSF_E_DEVICE, "guide table upload"));
    G.vmax = std::max(G.vmax, vm);
    id.ctap = dev;
    G.inst.push_back(id);
    G.members.push_back(i);
  }
  for (auto& G : b->groups) {
    const size_t n = G.members.size();
    // the kernels index tiles of all instances of a launch with 32-bit integers
    for (int ax = 0; ax < 3; ++ax)
      for (int v = 0; v < (ax == 0 ? 1 : ssf::NUM_STRIDED_VARIANTS); ++v) {
        const dim3 t = pass_grid(G.h, ax, ax == 0 ? -1 : v);
        if ((long long)t.x * t.y * (long long)n >= (1LL << 31))
          return bail(fail(SSF_E_UNSUPPORTED, "too many tiles in one batch group"));
      }
    const dim3 gx = pass_grid(G.h, 0);
    G.obs_blocks = (long long)gx.x * gx.y;
    if (hipMalloc(&G.d_inst, sizeof(ssf::InstDesc) * n) != hipSuccess ||
        hipMalloc(&G.d_slot, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&G.obs_part, sizeof(double) * 8 * G.obs_blocks * n) != hipSuccess)
      return bail(fail(SSF_E_NOMEM, "batch descriptors"));
    if (hipMemcpy(G.d_slot, G.members.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(SSF_E_DEVICE, "batch slot upload"));
  }
  *out = b;
  return SSF_OK;
}

}  // namespace

extern "C" {

ssf_status ssf_batch_create(int32_t count, const ssf_grid_desc* grids, const ssf_ctap_desc* guides,
                            const double* x_lo, const double* x_hi, int32_t dtype, void* hip_stream,
                            ssf_batch** out) {
  if (!guides) return fail(SSF_E_INVALID, "bad batch arguments");
  return batch_create(count, grids, guides, nullptr, x_lo, x_hi, dtype, hip_stream, out);
}

ssf_status ssf_batch_create_tables(int32_t count, const ssf_grid_desc* grids, const double* const* vtabs,
                                   const double* x_lo, const double* x_hi, int32_t dtype, void* hip_stream,
                                   ssf_batch** out) {
  if (!vtabs) return fail(SSF_E_INVALID, "bad batch arguments");
  return batch_create(count, grids, nullptr, vtabs, x_lo, x_hi, dtype, hip_stream, out);
}

ssf_status ssf_batch_set_stream(ssf_batch* b, void* hip_stream) {
  if (!b) return fail(SSF_E_INVALID, "null batch");
  b->user = (hipStream_t)hip_stream;
  return SSF_OK;
}

ssf_status ssf_batch_destroy(ssf_batch* b) {
  batch_free(b);
  return SSF_OK;
}

ssf_status ssf_batch_info(ssf_batch* b, int32_t* ngroups, int32_t* group_of) {
  if (!b || !ngroups) return fail(SSF_E_INVALID, "null batch");
  *ngroups = (int32_t)b->groups.size();
  if (group_of)
    for (size_t j = 0; j < b->groups.size(); ++j)
      for (int i : b->groups[j].members) group_of[i] = (int32_t)j;
  return SSF_OK;
}

ssf_status ssf_batch_tune(ssf_batch* b, int32_t reps) {
  if (!b) return fail(SSF_E_INVALID, "null batch");
  HIP_TRY(hipSetDevice(b->device));
  for (auto& G : b->groups) {
    G.h->stream = G.stream;
    SSF_TRY(ssf_tune(G.h, reps, nullptr, nullptr));
  }
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return SSF_OK;
}

ssf_status ssf_batch_run(ssf_batch* b, void* const* psi, int64_t nsteps, double dt, int64_t chunk,
                         ssf_obs* obs_dev) {
  if (!b || !psi) return fail(SSF_E_INVALID, "null batch or field array");
  if (nsteps < 0 || chunk < 1) return fail(SSF_E_INVALID, "need nsteps >= 0 and chunk >= 1");
  if (!std::isfinite(dt) || dt == 0.0) return fail(SSF_E_INVALID, "dt must be finite and nonzero");
  HIP_TRY(hipSetDevice(b->device));
  const size_t esize = b->dtype == SSF_C64 ? 8 : 16;
  // descriptors: field pointers of this call (uploaded only when they change).
  // Every pass of the previous call, its graph replays and its observation
  // kernels included, reads the old descriptors; all of that work ends on the
  // capture stream, so the upload waits for it (and for the group streams).
  for (auto& G : b->groups)
    for (size_t k = 0; k < G.members.size(); ++k) {
      void* p = psi[G.members[k]];
      if (!p || ((uintptr_t)p) % (esize / 2) != 0) return fail(SSF_E_INVALID, "field pointer null or misaligned");
    }
  bool waited = false;
  for (auto& G : b->groups) {
    bool changed = false;
    for (size_t k = 0; k < G.members.size(); ++k) {
      void* p = psi[G.members[k]];
      if (G.inst[k].in != p) { G.inst[k].in = p; G.inst[k].out = p; changed = true; }
    }
    if (changed) {
      if (!waited) {
        HIP_TRY(hipStreamSynchronize(b->cap));
        for (auto& H : b->groups) HIP_TRY(hipStreamSynchronize(H.stream));
        waited = true;
      }
      HIP_TRY(hipMemcpy(G.d_inst, G.inst.data(), sizeof(ssf::InstDesc) * G.inst.size(), hipMemcpyHostToDevice));
    }
  }
  HIP_TRY(hipEventRecord(b->ev_start, b->user));
  HIP_TRY(hipStreamWaitEvent(b->cap, b->ev_start, 0));
  // kinetic tables (built on the group streams, ordered after the fork)
  std::vector<const double2*> kts(b->groups.size());
  SSF_TRY(batch_fork(b));
  for (size_t i = 0; i < b->groups.size(); ++i) {
    b->groups[i].h->stream = b->groups[i].stream;
    SSF_TRY(get_ktab(b->groups[i].h, dt, 0, &kts[i]));
  }
  SSF_TRY(batch_join(b));
  // eager part: the remainder (or a first chunk), then graph replays of `chunk` steps
  const int64_t q = nsteps / chunk, r = nsteps % chunk;
  int64_t replays = q;
  if (r > 0) SSF_TRY(batch_chunks_all(b, r, dt, kts));
  else if (q > 0) { SSF_TRY(batch_chunks_all(b, chunk, dt, kts)); replays = q - 1; }
  if (replays > 0) {
    if (!b->exec || b->graph_dt != dt || b->graph_k != chunk || b->graph_kt != kts) {
      if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
      if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
      HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
      ssf_status st = batch_chunks_all(b, chunk, dt, kts);
      hipGraph_t gr = nullptr;
      hipError_t ee = hipStreamEndCapture(b->cap, &gr);
      if (st != SSF_OK) { if (gr) (void)hipGraphDestroy(gr); return st; }
      if (ee != hipSuccess) return fail(SSF_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
      b->graph = gr;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_dt = dt;
      b->graph_k = chunk;
      b->graph_kt = kts;
    }
    for (int64_t i = 0; i < replays; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->cap));
  }
  if (obs_dev) {
    for (auto& G : b->groups) {
      PassArgs a = batch_args(G, 0, b->vkind);
      a.partials = G.obs_part;
      const int rows = G.h->ks[0]->contig[G.h->dti].px;
      const dim3 gx = pass_grid(G.h, 0);
      const dim3 grid(gx.x, gx.y, (unsigned)G.members.size());
      if (b->dtype == SSF_C64)
        hipLaunchKernelGGL(obs_reduce_batch<float2>, grid, dim3(256), 0, b->cap, a, rows);
      else
        hipLaunchKernelGGL(obs_reduce_batch<double2>, grid, dim3(256), 0, b->cap, a, rows);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(obs_finalize_batch, dim3((unsigned)G.members.size()), dim3(256), 0, b->cap, G.obs_part,
                         G.obs_blocks, G.h->dv, obs_dev, G.d_slot, (long long)nsteps);
      HIP_TRY(hipGetLastError());
    }
  }
  HIP_TRY(hipEventRecord(b->ev_done, b->cap));
  HIP_TRY(hipStreamWaitEvent(b->user, b->ev_done, 0));
  return SSF_OK;
}

}  // extern "C"
