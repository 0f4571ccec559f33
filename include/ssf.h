/*
 * ssf.h -- C ABI of libssf, the MI355X (gfx950) split-step Fourier library.
 *
 * libssf propagates a complex wavefunction psi on a periodic 3-D grid with
 * the Fourier split-operator method used for the three-dimensional waveguide
 * simulations of Morgan et al., "Coherent transport by adiabatic passage on
 * atom chips" (arXiv:1309.2451), Sec. IV (time step = 3-D Fourier transforms
 * plus pointwise multiplications by the exponentiated potential and kinetic
 * operators; momentum grid bounded by p_max = pi N / L) and Sec. V
 * (imaginary-time ground state, populations of the three guides).
 * Units: hbar = m = 1, so H = -1/2 laplacian + V.
 *
 * One Strang step (real time, dt):
 *     psi <- exp(-i V dt/2) IFFT[ exp(-i k^2 dt/2) FFT[ exp(-i V dt/2) psi ] ]
 * Imaginary time replaces exp(-i x) by exp(-x) and renormalises every step.
 *
 * Conventions
 *   - Grids: n = {Nx, Ny, Nz}; axis a samples lo[a] + j (hi[a]-lo[a])/n[a],
 *     j = 0..n[a]-1 (periodic, hi excluded).  Each n[a] must be one of the
 *     supported transform lengths (ssf_supported_length).
 *   - Fields live in device memory (HBM), shape (Nz, Ny, Nx), x fastest,
 *     interleaved complex: SSF_C64 = 2 x float (8 B), SSF_C128 = 2 x double
 *     (16 B), contiguous, aligned to the element size.  In complex64 mode all
 *     arithmetic is FP64 in registers and values are rounded once per pass.
 *   - FFT: forward sum_j x_j exp(-2 pi i j k / n), inverse with +i, both
 *     unnormalised in ssf_fft; the step applies 1/(Nx Ny Nz) itself.
 *   - Wavenumbers: k_j = (2 pi / L)(j if 2j < n else j - n).
 *
 * Ownership: the caller owns every device buffer passed in (psi, lambda,
 * potential tables, observation and gradient buffers, checkpoints); the
 * library never frees them.  The handle owns its tables and workspace.
 * Potential tables set with ssf_set_potential_table are borrowed and must
 * stay alive while steps run.
 *
 * Streams: every call enqueues on the handle's HIP stream and returns without
 * waiting, except where noted (ssf_obs_read, ssf_sync, ssf_destroy, and the
 * first use of a new (dt, time) pair, which builds kinetic tables on the
 * device asynchronously but may allocate).  Calls on one handle must come from
 * one thread at a time.
 *
 * Errors: every function returns SSF_OK (0) or a negative ssf_status and
 * never aborts.  ssf_last_error() gives a thread-local message.  Asynchronous
 * device faults surface at the next synchronising call.
 */
#ifndef SSF_H
#define SSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ssf_status;
#define SSF_OK 0
#define SSF_E_INVALID (-1)     /* bad argument: null, shape, alignment, dtype, dt, count */
#define SSF_E_UNSUPPORTED (-2) /* transform length not built into the library */
#define SSF_E_NOMEM (-3)       /* device allocation failed */
#define SSF_E_NODEVICE (-4)    /* no HIP device visible */
#define SSF_E_DEVICE (-5)      /* HIP runtime error (message in ssf_last_error) */
#define SSF_E_NONFINITE (-6)   /* an observation recorded a non-finite norm */

#define SSF_C64 1
#define SSF_C128 2
#define SSF_REAL 0
#define SSF_IMAG 1
#define SSF_SPLIT_VTV 0
#define SSF_SPLIT_TVT 1

typedef struct ssf_handle ssf_handle;

typedef struct ssf_grid_desc {
  int32_t n[3];    /* Nx, Ny, Nz */
  double lo[3];    /* box start per axis */
  double hi[3];    /* box end per axis (excluded) */
} ssf_grid_desc;

/* Three-guide potential (Gaussian stand-in for the chip's guides, Sec. III):
 * V(x,y,z) = - sum_g v0[g] exp(-((x - xc[g][z])^2 + y^2) / (2 sigma[g]^2)). */
typedef struct ssf_ctap_desc {
  int32_t nguides;     /* 1..3 */
  double v0[3];        /* well depths */
  double sigma[3];     /* widths (> 0) */
  const double* xc;    /* host, (nguides, Nz) guide centres, copied by the call */
} ssf_ctap_desc;

/* One observation (Sec. V, Figs. 4 and 6: guide populations). */
typedef struct ssf_obs {
  double norm;       /* sum |psi|^2 dV */
  double mean[3];    /* sum r_a |psi|^2 dV (first moments, not divided by norm) */
  double pop[3];     /* P1: x < x_lo, P2: x_lo <= x <= x_hi, P3: x > x_hi */
  double epot;       /* sum V |psi|^2 dV */
  double energy;     /* ssf_observables: <H>; imaginary-time step: -ln(norm ratio)/dt; else 0 */
  int64_t step;      /* steps completed within the call when recorded */
  int32_t flags;     /* bit 0: non-finite norm */
  int32_t reserved;
} ssf_obs;

/* Nonzero if n is a transform length built into the library. */
int32_t ssf_supported_length(int32_t n);

/* Create a handle for one grid and storage type (SSF_C64 / SSF_C128) on the
 * current HIP device, enqueueing on `hip_stream` (NULL = default stream).
 * Allocates tables and workspace (tens of bytes per grid point of x-z plane,
 * plus FP64 partial sums).  Errors: INVALID (null, n < 1, hi <= lo, dtype),
 * UNSUPPORTED (length), NODEVICE, NOMEM, DEVICE. */
ssf_status ssf_create(const ssf_grid_desc* grid, int32_t dtype, void* hip_stream, ssf_handle** out);
/* Synchronises the handle's stream, then frees what the handle owns. */
ssf_status ssf_destroy(ssf_handle* h);
ssf_status ssf_set_stream(ssf_handle* h, void* hip_stream);

/* Borrow a device potential table (Nz, Ny, Nx): FP64 if v_is_f64, else FP32. */
ssf_status ssf_set_potential_table(ssf_handle* h, const void* v_dev, int32_t v_is_f64);
/* Build the three-guide potential tables on the device (synchronous upload).
 * Errors: INVALID (nguides outside 1..3, sigma <= 0, null xc). */
ssf_status ssf_set_potential_ctap(ssf_handle* h, const ssf_ctap_desc* d);
/* Atom-chip potential (Sec. III): thin wires on the chip surface y = 0, each a
 * polyline in the (x, z) plane carrying a constant current; a homogeneous bias
 * field b_bias along +x (across the wires) and an offset field b_ip along +z
 * (along them); a harmonic trap of frequency omega_z along z centred at z_c.
 * The field B is the Biot-Savart sum over the wires' straight segments (each
 * by the closed-form finite-wire law) plus (b_bias, 0, b_ip), and
 *     V = mu_over_e0 (|B| - b_ip) + omega_z^2 (z - z_c)^2 / 2
 * (a low-field-seeking atom's magnetic energy measured from its value at the
 * offset field).  Grid coordinates are in length units of length_unit
 * metres; fields in tesla, currents in ampere; mu_over_e0 is the magnetic
 * moment over the energy unit (per tesla), omega_z in inverse time units.
 * Points on a segment's line get no contribution from it (keep the grid off
 * the plane y = 0). */
#define SSF_CHIP_MAX_WIRES 16
typedef struct ssf_chip_desc {
  int32_t nwires;          /* 1..16 */
  const int32_t* npts;     /* host, points of each wire's polyline (>= 2) */
  const double* path;      /* host, the (x, z) points of every wire, concatenated, length units */
  const double* current;   /* host, current of each wire (A), from its first point to its last */
  double b_bias;           /* T, along +x */
  double b_ip;             /* T, along +z, >= 0 */
  double length_unit;      /* metres per length unit */
  double mu_over_e0;       /* magnetic moment / energy unit, per tesla */
  double omega_z;          /* longitudinal trap frequency */
  double z_c;              /* trap centre (length units) */
} ssf_chip_desc;
/* Evaluate the atom-chip potential on the handle's grid into V_dev, a
 * caller-owned FP64 device table (Nz, Ny, Nx), in FP64 on the device; use it
 * with ssf_set_potential_table(h, V_dev, 1) or a table batch.  Copies the
 * segment list to a device buffer the handle keeps (synchronises the stream
 * first; allocates when the list grows); the evaluation itself is enqueued.
 * Errors: INVALID (null, misaligned, counts, non-finite values). */
ssf_status ssf_chip_potential(ssf_handle* h, const ssf_chip_desc* d, double* V_dev);
/* Remove the potential (free particle). */
ssf_status ssf_clear_potential(ssf_handle* h);
/* Guide regions for the populations: P1 counts grid points with x < x_lo,
 * P3 those with x > x_hi (strict), P2 the rest. */
ssf_status ssf_set_partition(ssf_handle* h, double x_lo, double x_hi);
/* Plane-dependent guide regions (Sec. V, Fig. 4: the population of each guide
 * while the guides move): x_lo[z], x_hi[z] for z = 0 .. Nz-1 (host arrays,
 * copied; e.g. the midlines between neighbouring guide centres).  Used by
 * every population until the next ssf_set_partition, including the target
 * mask of ssf_adjoint_init.  Synchronises the handle's stream. */
ssf_status ssf_set_partition_z(ssf_handle* h, const double* x_lo, const double* x_hi);
/* 0: one Strang step = 5 passes; 1 (default): consecutive steps without an
 * observation between them share one x pass (exp(-i V dt) between the inverse
 * and the next forward x transform), 4 passes per step.  In imaginary time
 * that shared x pass also sums the norm of the field between its two
 * potential half-steps, and the renormalisation rides on the next pass's
 * input.  Same result up to rounding. */
ssf_status ssf_set_fusion(ssf_handle* h, int32_t fuse_steps);
/* Ordering of the symmetric split step taken by ssf_step in real time:
 * SSF_SPLIT_VTV (default) = exp(-iV dt/2) exp(-iT dt) exp(-iV dt/2);
 * SSF_SPLIT_TVT = exp(-iT dt/2) exp(-iV dt) exp(-iT dt/2), the ordering whose
 * per-step count is four Fourier transforms and three multiplications
 * (Sec. IV).  Both are second order.  With TVT consecutive steps share the
 * kinetic passes (steady state: 4 passes per step, like VTV); each chain
 * start and each observation add a half-kinetic y/z round trip.  Imaginary
 * time, ssf_step_ckpt, ssf_step_seq and the adjoint use VTV only and return
 * SSF_E_UNSUPPORTED while TVT is selected. */
ssf_status ssf_set_splitting(ssf_handle* h, int32_t order);
/* Arithmetic of a complex64 handle's passes.  SSF_ARITH_F64 (default): every
 * butterfly, twiddle and factor multiplication in FP64 registers, values
 * rounded to complex64 once per pass.  SSF_ARITH_F32: complex64 bulk
 * arithmetic -- butterflies, twiddle products and LDS exchanges in FP32, every
 * twiddle power an exactly rounded FP32 value of an FP64 table -- while the
 * phase arguments (V dt, k^2 dt) are formed and reduced modulo 2 pi in FP64,
 * each phase or kinetic factor is computed in FP64 and rounded once, and all
 * reductions accumulate in FP64.  Faster in registers, less accurate (the
 * per-step rounding of FP32 transforms accumulates; see the design notes for
 * measured errors).  Single handles only (batches use FP64).  Errors: INVALID
 * (unknown mode, FP32 on a complex128 handle). */
#define SSF_ARITH_F64 0
#define SSF_ARITH_F32 1
ssf_status ssf_set_arithmetic(ssf_handle* h, int32_t arith);

/* Tile autotuner.  The y and z passes come in SSF_TILE_VARIANTS variants of
 * tile shape (0: 128 B of storage per row segment, the next tile prefetched
 * into registers; 1: half-width tile, half the workgroup and LDS, so twice
 * as many workgroups fit a compute unit; 2: the variant-0 tile with twice the
 * values per thread and half the workgroup, no prefetch, complex64 values
 * crossing LDS as FP32, so two workgroups share a compute unit).  ssf_tune
 * times every variant of the y pass (forward) and of the z pass (forward-
 * kinetic-inverse) `reps` times on a field-sized workspace (allocated on
 * first use), keeps the fastest per axis, writes the choice to choice_out[3]
 * (x is always 0) and, if us_out != NULL, the average microseconds per launch
 * to us_out[axis * SSF_TILE_VARIANTS + variant] (3 x SSF_TILE_VARIANTS
 * entries).  Synchronises the stream.  ssf_set_tiles / ssf_get_tiles set and
 * read the choice (e.g. from a cache). */
#define SSF_TILE_VARIANTS 3
/* The tuner with a cache file: if cache_path (a text file, created if
 * missing) holds a choice for this device architecture, grid, storage type
 * and arithmetic, apply it without timing anything (*hit = 1); otherwise run
 * ssf_tune(h, reps, ...), apply its choice and append a line
 * "ssf-tiles-v1 <arch> <Nx>x<Ny>x<Nz> <c64|c128> <f64|f32> variants<V> | <y> <z>"
 * (*hit = 0).  choice_out[3] and hit may be NULL.  Lines that do not parse
 * are ignored; the last matching line wins.  Errors: INVALID (empty path,
 * reps < 1, unwritable file), and those of ssf_tune. */
ssf_status ssf_tune_cached(ssf_handle* h, int32_t reps, const char* cache_path, int32_t* choice_out, int32_t* hit);
ssf_status ssf_tune(ssf_handle* h, int32_t reps, int32_t* choice_out, double* us_out);
ssf_status ssf_set_tiles(ssf_handle* h, const int32_t* choice);
ssf_status ssf_get_tiles(ssf_handle* h, int32_t* choice);

/* Pass timing for measurement: while on, every pass launch is bracketed by
 * a pair of HIP events on the handle's stream.  ssf_timing_read synchronises
 * the stream and returns, per pass kind, the summed kernel time in ms and the
 * number of launches since timing was switched on or last read, then resets.
 * Kinds (6 entries): 0 x forward, 1 x inverse, 2 x inverse-phase-forward,
 * 3 y/z forward, 4 y/z inverse, 5 z forward-kinetic-inverse. */
ssf_status ssf_set_timing(ssf_handle* h, int32_t on);
ssf_status ssf_timing_read(ssf_handle* h, double* ms_total, int64_t* launches);

/* nsteps Strang steps of psi (in place) with time step dt (nonzero, finite;
 * dt < 0 runs backwards; imaginary time needs dt > 0).  time = SSF_REAL or
 * SSF_IMAG.  If obs_every > 0 and obs_dev != NULL, after every obs_every-th
 * step an ssf_obs is written to obs_dev[step/obs_every - 1] (caller provides
 * nsteps/obs_every slots).  Imaginary time renormalises to norm 1 after every
 * step; the input is first scaled to norm 1.  No allocation after the first
 * call with a given (dt, time); no synchronisation. */
ssf_status ssf_step(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time,
                    int64_t obs_every, ssf_obs* obs_dev);

/* Allocation-free steps, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and results (bitwise) as ssf_step, on
 * the same handle and kernels; it never calls hipMalloc, hipFree or any
 * allocating routine.  What a step sequence writes besides psi and obs_dev --
 * the kinetic tables of dt (and dt/2 in the T/2-V-T/2 ordering), the FP64
 * partial sums of the reducing passes and the device scale of imaginary
 * time -- lives in one static device array per GPU of
 * ssf_noalloc_scratch_bytes() bytes (16 MiB, held until the process ends).
 * Every word of it is written before it is read within a call, so nothing is
 * cleared between calls.  The array is shared by every handle on that GPU:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and give wrong results.  Per-pass timing (ssf_set_timing) is ignored
 * during the call.  Errors as ssf_step, and INVALID when the grid needs more
 * scratch than the maximum (ssf_noalloc_scratch_need(h) bytes: about 64 B per
 * x-pass tile, e.g. 4 MiB for 512^3), checked before anything is enqueued. */
ssf_status ssf_step_noalloc(ssf_handle* h, void* psi, int64_t nsteps, double dt, int32_t time,
                            int64_t obs_every, ssf_obs* obs_dev);
int64_t ssf_noalloc_scratch_bytes(void);
int64_t ssf_noalloc_scratch_need(ssf_handle* h);

/* Unnormalised 1-D transforms of psi (in place) along the axes in axis_mask
 * (bit 0 = x, 1 = y, 2 = z); inverse != 0 uses exp(+...). */
ssf_status ssf_fft(ssf_handle* h, void* psi, int32_t axis_mask, int32_t inverse);

/* Observables of psi into obs_dev[0], including <H> = sum (k^2/2)|FFT psi|^2 dV/N
 * + sum V |psi|^2 dV.  Allocates a field-sized workspace on first use. */
ssf_status ssf_observables(ssf_handle* h, const void* psi, ssf_obs* obs_dev);
/* Copy count observations to the host (synchronises the stream).  Returns
 * SSF_E_NONFINITE if any copied record has flags bit 0 set. */
ssf_status ssf_obs_read(ssf_handle* h, const ssf_obs* obs_dev, ssf_obs* host, int64_t count);
/* Density in the x-z plane integrated over y (Sec. V, Fig. 5):
 * out_dev[z * Nx + x] = sum_y |psi(x, y, z)|^2 dy, FP64, (Nz, Nx) device array,
 * summed in a fixed order. */
ssf_status ssf_density_xz(ssf_handle* h, const void* psi, double* out_dev);
/* Wait for the handle's stream; reports pending asynchronous errors. */
ssf_status ssf_sync(ssf_handle* h);
/* dst = src for one field of the handle (storage type, layout as above), by a
 * plain kernel that reads and writes every value once with the same per-lane
 * access width as the pass kernels: its HBM traffic is exactly 2 x field
 * bytes, which calibrates profiler byte counters.  src and dst must not
 * overlap. */
ssf_status ssf_copy(ssf_handle* h, const void* src, void* dst);

/* Real-time propagation with checkpoints: before the steps s*every
 * (s = 0 .. ceil(nsteps/every)-1) psi is copied to slot s of ckpt_dev
 * (field-sized slots, contiguous).  Steps are never merged, so
 * ssf_step_seq from a checkpoint reproduces the same states bitwise. */
ssf_status ssf_step_ckpt(ssf_handle* h, void* psi, int64_t nsteps, double dt, int64_t every,
                         void* ckpt_dev);
/* seq_dev slot 0 = psi0, slot s = state after s real-time steps, s <= nsteps
 * (nsteps + 1 field-sized slots). */
ssf_status ssf_step_seq(ssf_handle* h, const void* psi0, int64_t nsteps, double dt, void* seq_dev);

/* Adjoint of the final target population F = sum_{x > x_hi} |psi_N|^2 dV
 * (Sec. V, Fig. 6: transfer fidelity) with respect to the guide centres
 * xc[g][z] of the potential set by ssf_set_potential_ctap.
 * ssf_adjoint_init: lambda = psi where x > x_hi, 0 elsewhere.
 * ssf_adjoint_segment: with seq_dev the nsteps+1 states of one segment
 * (ssf_step_seq), walks the segment backwards: lambda <- U(-dt) lambda, and
 * for every potential half-step adds dt sum dV/dxc_g Im(conj(lambda) psi) dV
 * to G_dev[g][z] (FP64, (nguides, Nz), accumulated, caller zeroes it). */
ssf_status ssf_adjoint_init(ssf_handle* h, const void* psi, void* lambda);
ssf_status ssf_adjoint_segment(ssf_handle* h, void* lambda, const void* seq_dev, int64_t nsteps,
                               double dt, double* G_dev);

/* Chain rule to profile coefficients: out_dev[g][m] = sum_z G_dev[g][z] B_dev[z][m]
 * for g < nguides, m < M (device FP64 buffers; B_dev is (Nz, M) row-major). */
ssf_status ssf_profile_grad(ssf_handle* h, const double* G_dev, int32_t nguides, const double* B_dev, int32_t M,
                            double* out_dev);

/* Batched parameter sweeps (Sec. V, Fig. 6: final target population over a
 * range of chip parameters; Sec. IV: concurrent runs).  `count` instances,
 * each with its own grid, guides and partition; instances with identical
 * grids form a group that shares tables and whose passes run as one
 * persistent launch over all of the group's fields.  Groups run concurrently
 * on library-owned streams, ordered after everything already enqueued on
 * `hip_stream` and before anything enqueued there later.
 * ssf_batch_run: nsteps real-time steps of every field psi[i] (host array of
 * device pointers, complex64/complex128 per dtype, in place), the steps in
 * chunks of `chunk` captured once in a HIP graph and replayed; then, if
 * obs_dev != NULL, obs_dev[i] = observation of field i (populations give
 * the transfer fidelity).  ssf_batch_tune runs ssf_tune on every group.
 * Creation copies the guide descriptions (allocates); runs allocate nothing
 * after the first with a given (dt, chunk). */
typedef struct ssf_batch ssf_batch;
ssf_status ssf_batch_create(int32_t count, const ssf_grid_desc* grids, const ssf_ctap_desc* guides,
                            const double* x_lo, const double* x_hi, int32_t dtype, void* hip_stream,
                            ssf_batch** out);
/* The same with borrowed potential tables instead of guides: vtabs[i] is a
 * device FP64 table (Nz_i, Ny_i, Nx_i) of instance i (e.g. from
 * ssf_chip_potential), kept alive by the caller while the batch runs. */
ssf_status ssf_batch_create_tables(int32_t count, const ssf_grid_desc* grids, const double* const* vtabs,
                                   const double* x_lo, const double* x_hi, int32_t dtype, void* hip_stream,
                                   ssf_batch** out);
ssf_status ssf_batch_run(ssf_batch* b, void* const* psi, int64_t nsteps, double dt, int64_t chunk,
                         ssf_obs* obs_dev);
ssf_status ssf_batch_tune(ssf_batch* b, int32_t reps);
/* Order later runs after the work enqueued on `hip_stream` (and work enqueued
 * there afterwards after them), in place of the stream given at creation. */
ssf_status ssf_batch_set_stream(ssf_batch* b, void* hip_stream);
/* Number of groups and the group of each instance (group_of[count], may be NULL). */
ssf_status ssf_batch_info(ssf_batch* b, int32_t* ngroups, int32_t* group_of);
ssf_status ssf_batch_destroy(ssf_batch* b);

/* Host helper: clamped uniform cubic B-spline basis on [a, b] with M >= 4
 * functions evaluated at z[0..nz-1]; B_out is (nz, M) row-major, FP64. */
ssf_status ssf_bspline_basis(int32_t M, double a, double b, const double* z, int32_t nz, double* B_out);
/* Host helper: profiles x_k(z) = sum_m coeffs[k][m] B_m(z) of the same basis
 * for nsets coefficient sets: out is (nsets, nz) row-major, FP64.  With
 * ssf_profile_grad (the transpose of this map) it is the parameterisation of
 * the guide centres whose gradient the adjoint gives. */
ssf_status ssf_bspline_eval(int32_t M, double a, double b, const double* coeffs, int32_t nsets, const double* z,
                            int32_t nz, double* out);

const char* ssf_status_string(ssf_status s);
const char* ssf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SSF_H */
