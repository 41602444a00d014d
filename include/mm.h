/*
 * mm.h -- C ABI of the MI355X micromagnetic effective-field / torque library.
 *
 * The library evaluates, on one AMD MI355X (gfx950), the hot path of the
 * finite-difference micromagnetic method of Vansteenkiste et al., "The design
 * and verification of MuMax3" (arXiv:1406.7635):
 *   - the magnetostatic field as a zero-padded FFT convolution of M = Msat m
 *     with the cell-averaged demagnetising kernel (section "Magnetostatic
 *     field"),
 *   - the 6-neighbour exchange field over region-indexed materials with the
 *     harmonic-mean inter-region coupling (section "Heisenberg exchange
 *     interaction", Eqs. eqBexch1 and eqBexch),
 *   - uniaxial anisotropy (section "Magneto-crystalline anisotropy") and the
 *     applied (Zeeman) field,
 *   - the Landau-Lifshitz torque (Eq. eqLLG) and the Runge-Kutta solvers of
 *     section "Dynamics" with the adaptive step of section "Adaptive time
 *     step", and relax() of section "Energy minimization".
 *
 * Units are SI throughout: m is a unit vector, B in tesla, t in seconds,
 * Msat in A/m, Aex in J/m, Ku in J/m^3, gamma in rad/(T s).
 *
 * Memory and layout.  Every pointer whose name ends in _dev is device memory
 * owned by the caller (e.g. a torch tensor).  Vector fields are FP32
 * structure-of-arrays [3][nz][ny][nx] with x fastest (all x components, then
 * all y, then all z).  The region map is uint8 [nz][ny][nx].  The library never
 * frees caller memory; the context owns every scratch buffer, allocated in
 * mm_create and freed in mm_destroy.
 *
 * Streams and synchronisation.  All work is enqueued on the HIP stream given
 * to mm_create (NULL = the legacy default stream).  Calls that return host
 * scalars (mm_rk45_step, mm_rk23_step, mm_run, mm_relax, mm_energy,
 * mm_max_torque) synchronise that stream before returning; the others return
 * as soon as the work is enqueued.  A context is not thread-safe.
 *
 * Errors.  Every int-returning call returns an mm_status; no exception or
 * abort crosses the ABI.  mm_strerror() gives a static description.  After
 * MM_EDEVICE the context should be destroyed.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MM_OK = 0,
    MM_EINVAL = -1,          /* bad argument (null pointer, non-positive size, NaN parameter) */
    MM_ENOMEM = -2,          /* device allocation failed */
    MM_EDEVICE = -3,         /* a HIP runtime call failed */
    MM_EUNSUPPORTED = -4,    /* valid but not supported: padded length > 4096, PBC */
    MM_ENONFINITE = -5,      /* a step produced a non-finite error estimate */
    MM_ESTEP = -6,           /* the adaptive step fell below dt_min */
    MM_ENOTCONVERGED = -7,   /* relax hit max_steps before MaxErr reached its floor */
    MM_ESTATE = -8,          /* call order: e.g. demag enabled but kernel not initialised */
    MM_ESCRATCH = -9         /* mm_beff_noalloc: the spectrum exceeds the static scratch */
} mm_status;

/* Size of the static spectrum scratch of mm_beff_noalloc, in MiB per GPU. */
#define MM_STATIC_SCRATCH_MIB 32

#define MM_NREGIONS 256
#define MM_NPAIRS (MM_NREGIONS * (MM_NREGIONS + 1) / 2)

typedef struct mm_ctx mm_ctx;

/* Finite-difference grid (section "Material Regions"): nx*ny*nz orthorhombic
 * cells of dx*dy*dz metres.  Each axis is zero-padded for the aperiodic
 * convolution to the power of two >= 2n-1 (no padding when n = 1); padded
 * lengths above 4096 return MM_EUNSUPPORTED.
 * pbc[a] >= 0: periodic boundary conditions along axis a (x, y, z) by macro
 * geometry (section "Magnetostatic field", paragraph "Periodic boundary
 * conditions"): P = pbc[a] > 0 counts the images of the box along that axis
 * such that a cell feels every source, image or not, whose displacement lies
 * within +-(n P - 1) cells (the field of a box 2 n P cells long around it),
 * and the exchange stencil wraps around.  0: open boundary.  The images enter
 * the kernel only: the field passes are the same (the periodic axis keeps its
 * zero padding).  Ensembles take pbc = {0,0,0} only. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t pbc[3];
} mm_grid;

/* Region look-up tables (section "Material Regions": a 256-entry table per
 * parameter indexed by the cell's region; interfacial parameters in a lower
 * triangular matrix indexed by the two regions).  Msat = 0 marks a
 * non-magnetic cell: its B_eff and torque are zero and it does not couple by
 * exchange.  exch_scale[i*(i+1)/2 + j], i >= j, is the inter-region scale S of
 * Eq. eqBexch; S(i,i) is taken as 1 whatever is stored.  anis_u need not be
 * normalised by the caller: it is used as given.  gamma_ll = 0 selects the
 * default 1.7595e11 rad/(T s). */
typedef struct {
    double msat[MM_NREGIONS];
    double aex[MM_NREGIONS];
    double alpha[MM_NREGIONS];
    double ku1[MM_NREGIONS];
    double ku2[MM_NREGIONS];
    double anis_u[MM_NREGIONS][3];
    double bext[MM_NREGIONS][3];
    double exch_scale[MM_NPAIRS];
    double gamma_ll;
} mm_params;

/* Adaptive-step options (section "Adaptive time step").  max_err is the
 * paper's MaxErr (default 1e-5 when <= 0), headroom its 0.8 (default when
 * <= 0); dt is clamped to [dt_min, dt_max] (dt_max <= 0 means unbounded).
 * precess = 0 drops the m x B term (relax). */
typedef struct {
    double max_err;
    double headroom;
    double dt_min;
    double dt_max;
    int32_t precess;
    int32_t reserved;
} mm_solver_opts;

/* Counters of a multi-step run. */
typedef struct {
    int64_t steps;       /* accepted steps */
    int64_t rejects;     /* rejected attempts */
    int64_t evals;       /* torque evaluations (B_eff + torque passes) */
    double t;            /* time reached */
    double dt;           /* next step size */
    double err;          /* error estimate of the last attempt */
} mm_run_stats;

/* Sizes chosen by the context, for callers and tests. */
typedef struct {
    int32_t px, py, pz;          /* padded FFT lengths */
    int32_t kx;                  /* px/2 + 1 spectral columns */
    int32_t ncomp;               /* demag kernel components stored: 4 (nz == 1) or 6 */
    int32_t reserved;
    int64_t ncell;
    int64_t khat_elems;          /* floats in the FP32 kernel spectrum */
    int64_t device_bytes;        /* device memory owned by the context */
} mm_info;

/* Create a context for grid g with parameters p on the given HIP stream
 * (hipStream_t passed as void*, NULL for the default stream).  region_dev is a
 * caller-owned uint8 [nz][ny][nx] device array, copied into the context.
 * Allocates every buffer; derives the FP32 region tables and the exchange
 * pair table on the device.  Demag is enabled but needs mm_demag_kernel_init
 * before the first field evaluation.  Returns MM_EINVAL for null pointers,
 * non-positive sizes, non-finite cell sizes or negative pbc, MM_EUNSUPPORTED
 * for padded lengths above 4096, more than 2^28 cells, or an image window
 * (the product over the axes of n P, or n without images) above 2^26
 * displacements, MM_ENOMEM if allocation fails. */
int mm_create(mm_ctx **out, const mm_grid *g, const mm_params *p, const uint8_t *region_dev,
              void *hip_stream);

/* Build the demagnetising kernel (section "Magnetostatic field", paragraph
 * "Magnetostatic kernel"): the cell-averaged tensor N(d) for every cell
 * displacement in FP64 on the GPU -- Newell's closed form near the origin,
 * Gauss-Legendre quadrature of the dipole tensor far away -- mirrored into the
 * padded grid using its symmetries, Fourier transformed in FP64, scaled by
 * -mu0 / (px py pz) and truncated to FP32.  Only the non-redundant octant of
 * the real spectrum is kept (4 components in 2D, 6 in 3D).  With periodic
 * axes the tensor is evaluated over the whole image window (0 .. n P - 1 cells
 * along such an axis) and each box displacement takes the sum over its
 * images (its negative-displacement images by the tensor's parity) before
 * the mirror fill.  Temporary FP64 buffers are allocated and freed inside the
 * call.  Synchronous. */
int mm_demag_kernel_init(mm_ctx *c);

/* Replace the material tables (same validation as mm_create).  Invalidates
 * the solver's cached first-stage torque. */
int mm_set_params(mm_ctx *c, const mm_params *p);

/* enable = 0 drops the magnetostatic term (the paper's EnableDemag = false). */
int mm_set_demag(mm_ctx *c, int32_t enable);

/* B_eff = B_demag + B_exch + B_anis + B_ext at m (section "Landau-Lifshitz
 * torque", list of contributions).  beff_dev: [3][nz][ny][nx] output.
 * bdemag_dev may be NULL; otherwise it receives the magnetostatic field
 * alone, in every cell (including Msat = 0 cells, where B_eff is 0). */
int mm_beff(mm_ctx *c, const float *m_dev, float *beff_dev, float *bdemag_dev);

/* mm_beff for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results as mm_beff; the call itself allocates
 * nothing (no hipMalloc / hipFree, no event or host-container growth).  The
 * FFT spectrum, which mm_beff keeps in the context, lives instead in one
 * static device array of MM_STATIC_SCRATCH_MIB MiB per GPU, loaded with the
 * library and held until the process ends; its address on each device is
 * resolved by the first mm_create on that device.  Every spectrum element is
 * written before it is read within a call, so nothing needs clearing between
 * calls.  All calls on one GPU share the array: calls that overlap on one GPU
 * (two contexts, two streams or two threads) race and give wrong fields.
 * Returns MM_ESCRATCH, before any work is enqueued, when the grid's spectrum
 * (3 (px/2 + 1) ny nz complex64 in 2D and thin 3D grids, 3 (px/2 + 1) py nz
 * in other 3D grids) exceeds the array; MM_ESTATE as mm_beff.  Launch timing
 * (mm_timing_enable) does not cover this call. */
int mm_beff_noalloc(mm_ctx *c, const float *m_dev, float *beff_dev, float *bdemag_dev);

/* Landau-Lifshitz torque (Eq. eqLLG, damping sign):
 * tau = -gamma/(1+alpha^2) [m x B + alpha m x (m x B)], m x B dropped when
 * precess = 0.  Elementwise from a given field; tau_dev in 1/s. */
int mm_llg_torque(mm_ctx *c, const float *m_dev, const float *beff_dev, float *tau_dev,
                  int32_t precess);

/* Fused evaluation of B_eff and the torque at m (one "torque evaluation" in
 * the sense of the paper's throughput, section "Performance"). */
int mm_torque(mm_ctx *c, const float *m_dev, float *tau_dev, int32_t precess);

/* One classical RK4 step of fixed size dt (not among the paper's solvers;
 * provided for fixed-step trajectories), then m is renormalised. */
int mm_rk4_step(mm_ctx *c, float *m_dev, double dt, int32_t precess);

/* One attempt of the Dormand-Prince 5(4) pair (section "Dynamics", RK45)
 * from (m, *t) with step *dt.  eps = dt max_cells |sum_j (b_j - b*_j) k_j|
 * (section "Adaptive time step"); accepted when eps <= max_err, in which case
 * m <- normalise(5th-order solution) and *t += dt.  *dt is replaced by the
 * next step: dt headroom (max_err/eps)^(1/5) clamped to [0.1, 2] times dt
 * (2 when eps = 0) and to [dt_min, dt_max].  The torque of the last stage is
 * cached and reused as the next step's first (first-same-as-last); it is
 * recomputed after mm_solver_reset, mm_set_params, mm_set_demag, a change of
 * m pointer or of precess.  Synchronous. */
int mm_rk45_step(mm_ctx *c, float *m_dev, double *t, double *dt, const mm_solver_opts *o,
                 int32_t *accepted, double *err);

/* Same for the Bogacki-Shampine 3(2) pair (RK32 of the paper; exponent 1/3).
 * Both return MM_EUNSUPPORTED while a temperature is set. */
int mm_rk23_step(mm_ctx *c, float *m_dev, double *t, double *dt, const mm_solver_opts *o,
                 int32_t *accepted, double *err);

/* Advance with solver 45 (Dormand-Prince), 23 (Bogacki-Shampine) or 12 (Heun,
 * RK12 of section "Dynamics": k1 at m, k2 at m + dt k1, new state
 * m + dt (k1 + k2)/2, Euler error estimate, exponent 1/2; two torque
 * evaluations per attempt, no first-same-as-last) until t_end (the last step
 * is clipped to land on it) or until max_attempts attempts, with the step
 * controller running on the device (no host round trip per step).  While a
 * temperature is set (mm_set_temperature) only solver 12 runs, at the fixed
 * step *dt (section "Thermal fluctuations": every step accepted; max_err and
 * the step limits are ignored) with the thermal field of each step added to
 * B_eff in both stages; the other solvers return MM_EUNSUPPORTED.  *t and *dt
 * are read and updated.  stats may be NULL.  Returns MM_ESTEP / MM_ENONFINITE
 * if the run stopped on those conditions, MM_EDEVICE if a chunk of attempts
 * left the device-side solver state unchanged (no step, reject or end). */
int mm_run(mm_ctx *c, float *m_dev, int32_t solver, double t_end, int64_t max_attempts,
           double *t, double *dt, const mm_solver_opts *o, mm_run_stats *stats);

/* relax() of section "Energy minimization": precession off, RK23 steps in
 * blocks of 3; an energy phase until the total energy stops decreasing, then
 * torque phases until max|tau| stops decreasing, halving MaxErr (starting
 * from o->max_err) after each, until MaxErr < min_max_err (1e-9 if <= 0).
 * Energies are FP64 reductions on the device.  Outputs may be NULL.
 * MM_ENOTCONVERGED if max_steps attempts were used first. */
int mm_relax(mm_ctx *c, float *m_dev, const mm_solver_opts *o, double min_max_err,
             int64_t max_steps, double *energy_out, double *max_torque_out, int64_t *steps_out);

/* Energies in joules (FP64 reduction on the device), in the order demag,
 * exchange, anisotropy, Zeeman, total: V sum[-1/2 M.B_demag - 1/2 M.B_exch
 * - 1/2 M.B_anis(Ku1) - 1/4 M.B_anis(Ku2) - M.B_ext]. e_terms5: host double[5]. */
int mm_energy(mm_ctx *c, const float *m_dev, double *e_terms5);

/* max over cells of |tau| (1/s) at m. */
int mm_max_torque(mm_ctx *c, const float *m_dev, int32_t precess, double *out);

/* Forget the cached first-stage torque (call after changing m in place). */
int mm_solver_reset(mm_ctx *c);

int mm_get_info(mm_ctx *c, mm_info *info);

/* Time-dependent excitation (section "Material Regions", paragraph
 * "Time-dependent parameters"): term `slot` (0..3) adds f(t) g(r) to B_eff,
 * f(t) = a + b sin(omega t + phi), g_dev a caller-owned device profile
 * [3][nz][ny][nx] (FP32, tesla) that must outlive its use; g_dev = NULL clears
 * the slot.  Every field evaluation inside mm_run and the single-step calls
 * takes f at its stage time t + c_s dt (c_s the stage's node of the
 * tableau); mm_beff, mm_torque, mm_energy and mm_max_torque take it at the
 * context's current time (the end of the last run, 0 before); the field is
 * part of B_eff but not of the energies; relax ignores it and mm_rk4_step
 * (which has no time argument) returns MM_EUNSUPPORTED while a term is set.
 * The surrogate stages are not used while a term is set.  Allocates the
 * field buffer the first time. */
int mm_set_excitation(mm_ctx *c, int32_t slot, const float *g_dev, double a, double b, double omega,
                      double phi);

/* enable = 1: mm_run with at least 16 attempts captures one attempt as a HIP
 * graph on a stream of the context's own (default priority, ordered after the
 * work on the context stream by events) and replays it, one host launch per
 * attempt; results are identical to direct launches.  Off by default: on the
 * measured ROCm stack the replays run slower than the direct launches (1024^2
 * film 0.44 ms against 0.42 ms per attempt, 16^2 0.154 against 0.136 ms).
 * Never used while kernel timing or the surrogate is active; if a capture
 * fails the run launches directly. */
int mm_set_run_graphs(mm_ctx *c, int32_t enable);

/* Temperature (section "Thermal fluctuations"): temp_k[256] in kelvin per
 * region (host array; NULL = 0 K everywhere), and the seed of the generator.
 * Each cell then carries the thermal field
 *   B_therm = eta sqrt(2 alpha kB T / (Msat gamma_LL dV dt))
 * (the paper's form with B_sat = mu0 Msat), eta three standard normal numbers
 * per cell and step, held over the stages of a step and drawn anew for each
 * accepted step, from Philox4x32-10 (Salmon et al., SC 2011): counter (cell
 * index, step mod 2^32, step div 2^32, 0), key (seed mod 2^32, seed div 2^32),
 * 32-bit outputs x -> u = (floor(x / 2^8) + 1/2) / 2^24, Box-Muller
 * eta_x, eta_y = sqrt(-2 ln u0) (cos, sin)(2 pi u1),
 * eta_z = sqrt(-2 ln u2) cos(2 pi u3).  step counts the steps accepted since
 * this call (which resets it).  The field enters mm_run with solver 12 only
 * (relax and the single-step calls run at 0 K or refuse).  Allocates the
 * field buffer the first time.  Synchronises.  MM_EINVAL for a negative or
 * non-finite temperature. */
int mm_set_temperature(mm_ctx *c, const double *temp_k, uint64_t seed);

/* Cubic magneto-crystalline anisotropy (section "Magneto-crystalline
 * anisotropy"), per region: kc[256][3] = (Kc1, Kc2, Kc3) in J/m^3 and the axes
 * c1[256][3], c2[256][3] (host arrays, normalised here; c3 = c1 x c2, so c1
 * and c2 should be perpendicular).  Adds to B_eff, with a_i = c_i . m,
 *   -2 Kc1/Msat sum_i a_i (a_j^2 + a_k^2) c_i - 2 Kc2/Msat sum_i a_i a_j^2 a_k^2 c_i
 *   -4 Kc3/Msat sum_i a_i^3 (a_j^4 + a_k^4) c_i
 * and to the anisotropy energy -1/4 M.B(Kc1) - 1/6 M.B(Kc2) - 1/8 M.B(Kc3).
 * kc = NULL removes it.  Tables are rebuilt by mm_set_params (Msat).  Ensembles
 * have no cubic term.  Synchronises. */
int mm_set_cubic_anisotropy(mm_ctx *c, const double *kc, const double *c1, const double *c2);

/* Induced (interfacial) Dzyaloshinskii-Moriya interaction (section
 * "Dzyaloshinskii-Moriya interaction"): dind[256] = D per region in J/m^2
 * (host array; NULL removes it).  Adds to the exchange field
 *   B_DM = 2D/Msat (dm_z/dx, dm_z/dy, -dm_x/dx - dm_y/dy)
 * with central differences (m_{i+1} - m_{i-1})/(2 Delta_i) and the boundary
 * rule of the paper: an in-plane neighbour missing at the boundary of the
 * magnet -- outside an open edge of the grid, or a non-magnetic cell
 * (Msat = 0) -- is replaced by m + n Delta dm/di|_b (n = -1 on the low side,
 * +1 on the high side), dm/dx|_b = D/(2A) (-m_z, 0, m_x), dm/dy|_b = D/(2A)
 * (0, -m_z, m_y)
 * (D, A, Msat of the cell's region), and that ghost also enters the exchange
 * field as 2A/Msat (ghost - m)/Delta^2.  Its energy is counted with the
 * exchange energy (-1/2 M.B).  Tables are rebuilt by mm_set_params.
 * Ensembles have no DMI.  Synchronises. */
int mm_set_dmi(mm_ctx *c, const double *dind);

/* The thermal field of generator step `step` with time step dt into out_dev
 * ([3][nz][ny][nx] floats, T), as the Heun steps take it.  MM_ESTATE before
 * mm_set_temperature. */
int mm_thermal_field(mm_ctx *c, double dt, uint64_t step, float *out_dev);

/* Diagnostics.  mm_demag_tensor_dump writes the FP64 real-space tensor N(d)
 * for d = (i dx, j dy, k dz), 0 <= i < nx etc., as [6][nz][ny][nx] doubles
 * (component order xx, yy, zz, xy, xz, yz) into out_dev (recomputed on the
 * device; on a periodic grid, the sum over the images of each displacement,
 * as the kernel takes it; synchronises then).  mm_demag_kernel_dump copies the FP32 kernel spectrum, layout
 * [kx][ky_h][kz_h][ncomp] (h = folded index 0..p/2; ncomp = 6 in 3D with
 * order xx, yy, zz, xy, xz, yz, or 4 when nz == 1: xx, yy, zz, xy),
 * khat_elems floats.  mm_exchange_dump writes the per-face exchange
 * coefficient c(r, r_n)/D^2 actually gathered by the field kernels, as
 * [6][nz][ny][nx] floats in face order -x, +x, -y, +y, -z, +z (0 where the
 * neighbour is missing; across a periodic boundary the neighbour is the
 * cell at the other end of an axis longer than one cell). */
int mm_demag_tensor_dump(mm_ctx *c, double *out_dev);
int mm_demag_kernel_dump(mm_ctx *c, float *out_dev);
int mm_exchange_dump(mm_ctx *c, float *out_dev);

/* Kernel timing with HIP events on the context stream.  mm_timing_enable(c,
 * which, 1) has every later launch of kernel class `which` (0 = x-forward FFT
 * pass, 1 = column (y/z) convolution pass, 2 = x-inverse FFT + field/torque
 * pass, 3 = fused x-inverse of one Runge-Kutta stage and x-forward of the
 * next) record an event pair at the start and end of the kernel itself (3D:
 * from the start of the y-forward to the end of the y-inverse launch); the
 * event pairs are created by this call.  mm_timing_read returns the number of
 * launches and the summed milliseconds since enabling (synchronises).
 * Enabling again restarts the count; enable = 0 frees the events. */
int mm_timing_enable(mm_ctx *c, int32_t which, int32_t enable);
int mm_timing_read(mm_ctx *c, int32_t which, int64_t *launches, double *total_ms);

/* Checkpoint and resume.  A run continues bit for bit from a saved state
 * given the same m (the caller's array, saved by the caller) and the (t, dt)
 * that mm_run returned.  The saved state holds the device-side solver record
 * (the map of stage-derivative buffers, the controller's scalars and
 * counters, the thermal generator's step counter), the FSAL flags with the
 * first-stage derivative of the next step (3 ncell floats, when valid), and
 * the thermal seed.  mm_state_size gives the largest size; mm_state_save
 * writes it to a host buffer (synchronous); mm_state_load restores it into a
 * context created with the same grid and parameters (temperature, DMI,
 * cubic anisotropy and excitations set again by the caller before the
 * load: setting a temperature resets the generator step that the load
 * restores), binding the
 * FSAL derivative to m_dev.  MM_EINVAL for a short buffer, another grid or a
 * buffer that is not a saved state. */
int mm_state_size(mm_ctx *c, int64_t *bytes);
int mm_state_save(mm_ctx *c, void *host_buf, int64_t bytes);
int mm_state_load(mm_ctx *c, const void *host_buf, int64_t bytes, const float *m_dev);

/* Arithmetic of the DFT stages of the y convolution.  MM_PREC_FP32 (the
 * default) runs them in FP32 on the vector units.  MM_PREC_BF16 and
 * MM_PREC_FP16 run them as matrix-core GEMMs (16 x 16 x 32) on operands split
 * into two low-precision parts, x = x_hi + x_lo, keeping hi.hi + hi.lo + lo.hi
 * in FP32 accumulators (FP16 inputs scaled per column, or per workgroup of
 * columns in 3D, by powers of two); the K^ product, the twiddles and
 * everything outside the column passes stay FP32.  The matrix-core form
 * exists for 2D grids whose padded y length is 2048 (the y convolution) and
 * for 3D grids of more than four layers whose padded y and z lengths lie in
 * 64 ... 1024 (y forward, z convolution and y inverse); other grids return
 * MM_EUNSUPPORTED and keep FP32.  Takes effect for later field evaluations;
 * the FSAL derivative is recomputed. */
typedef enum { MM_PREC_FP32 = 0, MM_PREC_BF16 = 1, MM_PREC_FP16 = 2 } mm_precision;
int mm_set_conv_precision(mm_ctx *c, int32_t prec);

/* ---- Ensembles ------------------------------------------------------------
 * An ensemble advances many independent grids together (each with its own
 * size, cell size, region map, region tables, time step and solver state):
 * every pass of a Runge-Kutta stage is one launch over the tiles of all
 * members, the attempt is replayed as a HIP graph, and the number of
 * persistent workgroups of each pass can be tuned on the device.  Per member
 * the arithmetic is that of a single context (section "Magnetostatic field"
 * for the convolution, section "Dynamics" and "Adaptive time step" for the
 * solver); only the scheduling differs.
 *
 * Layout: the members' arrays are stored back to back in member order.  With
 * ncell_i = nx_i ny_i nz_i and off_i = ncell_0 + ... + ncell_{i-1}, member i's
 * region map is bytes [off_i, off_i + ncell_i) of the ensemble's uint8 region
 * array and its vector fields (m, B_eff) are floats [3 off_i, 3 off_i +
 * 3 ncell_i) of an FP32 array, [3][nz][ny][nx] within that range.
 *
 * Supported members: padded lengths 64 <= px, py <= 1024 (17 <= nx, ny <=
 * 512) and nz <= 8; at most 65535 members.  Others give MM_EUNSUPPORTED.
 * The ensemble works on a stream of its own; every call first waits for the
 * work already enqueued on the stream given at creation, and that stream
 * waits for the ensemble's work before anything enqueued on it later.
 * mm_batch_run and mm_batch_stats synchronise. */
typedef struct mm_batch mm_batch;

/* grids[n], params[n] (host arrays); region_dev: the concatenated region maps
 * (device, caller-owned, copied).  Allocates every buffer (the ensemble owns
 * them until mm_batch_destroy) and builds each member's region tables.  The
 * demagnetising kernels need mm_batch_demag_kernel_init. */
int mm_batch_create(mm_batch **out, int32_t n, const mm_grid *grids, const mm_params *params,
                    const uint8_t *region_dev, void *hip_stream);
/* FP64 Newell tensors and FP32 kernel spectra of every member, as
 * mm_demag_kernel_init does for one grid (synchronises). */
int mm_batch_demag_kernel_init(mm_batch *b);
/* Cell offset (off_i above) and cell count of member i. */
int mm_batch_member(mm_batch *b, int32_t i, int64_t *cell_offset, int64_t *ncell);
/* B_eff of every member at m_dev into beff_dev (both concatenated FP32). */
int mm_batch_beff(mm_batch *b, const float *m_dev, float *beff_dev);
/* (Re)start every member at time t0 with step dt0 towards t_end with the
 * adaptive solver `solver` (45: Dormand-Prince, 23: Bogacki-Shampine):
 * counters cleared, the first derivative recomputed by the next run. */
int mm_batch_start(mm_batch *b, int32_t solver, double t0, double dt0, double t_end, const mm_solver_opts *o);
/* Attempt steps of every running member (a member stops when it reaches
 * t_end, or with an error status) until none runs or max_attempts attempts
 * have been made.  m_dev: the concatenated states, updated in place.
 * *attempts_out: attempts made; *active_out: members still running.
 * Synchronises.  The stepping is device-controlled; every attempt is one
 * replay of a captured graph when graphs are enabled (the default). */
int mm_batch_run(mm_batch *b, float *m_dev, int64_t max_attempts, int64_t *attempts_out, int32_t *active_out);
/* Counters, time and step of member i after the last run; its status in
 * *status (MM_OK, MM_ENONFINITE or MM_ESTEP).  Synchronises. */
int mm_batch_stats(mm_batch *b, int32_t i, mm_run_stats *out, int32_t *status);
/* The same for every member at once: out[n], status[n] (status may be NULL). */
int mm_batch_stats_all(mm_batch *b, mm_run_stats *out, int32_t *status);
/* enable = 0: launch every kernel of an attempt directly instead of
 * replaying a graph (same kernels, same results). */
int mm_batch_set_graph(mm_batch *b, int32_t enable);
/* Persistent workgroups of batched pass `pass` (0 x passes, 1 2D y
 * convolution, 2 3D y transforms, 3/4/5 3D z convolution for padded z length
 * 4/8/16, 6/7 thin-grid 3D convolution (y FFT, z DFT, inverse y FFT in one
 * pass) for padded z length 4/8, 8 finalisation): grid > 0 (rounded up to a
 * multiple of 8), or 0 for one workgroup per tile.  mm_batch_get_grid reads
 * the current value. */
int mm_batch_set_grid(mm_batch *b, int32_t pass, int32_t grid);
int mm_batch_get_grid(mm_batch *b, int32_t pass, int32_t *grid);
/* Tile shape of pass 0 (x passes) or 1 (2D y convolution): 0 wide (768 /
 * 256 threads per workgroup, the row pairs or columns of the single-grid
 * wide workgroup per work item) or 1 narrow (192 / 64 threads, a quarter of
 * them).  The narrow shape serves padded lengths up to 512: MM_EUNSUPPORTED
 * when a member's px (pass 0) or py (pass 1) is larger, or for another pass.
 * Changing the shape resets the pass's grid to one workgroup per tile.
 * Results do not depend on the shape.  mm_batch_get_tile reads it. */
int mm_batch_set_tile(mm_batch *b, int32_t pass, int32_t tile);
int mm_batch_get_tile(mm_batch *b, int32_t pass, int32_t *tile);
/* Time every pass of one attempt at m_dev for each tile shape that serves
 * every member and a few persistent grid sizes per shape (whole-chip
 * multiples of the pass's resident workgroups, and one workgroup per tile),
 * and keep the fastest (shape, grid) per pass.  Overwrites the stage buffers
 * (the next run recomputes the first derivative); m_dev is only read.
 * Synchronises. */
int mm_batch_autotune(mm_batch *b, const float *m_dev);
void mm_batch_destroy(mm_batch *b);

/* ---- Surrogate of the magnetostatic field ---------------------------------
 * A spectral neural operator (not part of the paper's method: a learned
 * stand-in for the convolution of section "Magnetostatic field") maps m on an
 * nx x ny x 1 grid to a prediction of B_demag:
 *   lift      h_c = sum_j P[c][j] m_j + p[c]                         (32 channels)
 *   4 layers  hhat_c(k) = sum_{x,y} h_c exp(-2 pi i (kx x/nx + ky y/ny)) for the kept
 *             modes kx = 0..15, ky = -8..7; ghat_o(k) = sum_c R[ky+8][kx][o][c] hhat_c(k);
 *             g_o = Re sum_k w_kx ghat_o(k) exp(+2 pi i (...)) / (nx ny) (w_0 = 1, else 2);
 *             h_o <- GELU(g_o + sum_c W[o][c] h_c + b[o]) with GELU(z) = z (1 + erf(z/sqrt 2))/2
 *   project   B_j = out_scale (sum_c Q[j][c] h_c + q[j])
 * weights: host FP32 array of MM_SNO_NWEIGHTS values in the order P[32][3],
 * p[32], then per layer R[16][16][32][32][re,im], W[32][32], b[32], then
 * Q[3][32], q[3]; stored on the device rounded to BF16 (nearest even), all
 * arithmetic FP32.  32 <= nx <= 512, 16 <= ny <= 512, else MM_EUNSUPPORTED;
 * a wrong count gives MM_EINVAL.  Work is enqueued on hip_stream. */
#define MM_SNO_NWEIGHTS 2101603
typedef struct mm_sno mm_sno;
int mm_sno_create(mm_sno **out, int32_t nx, int32_t ny, const float *weights, int64_t nweights,
                  double out_scale, void *hip_stream);
/* Replace the weights (synchronises the stream first). */
int mm_sno_set_weights(mm_sno *s, const float *weights, int64_t nweights);
/* Predicted B_demag [3][ny][nx] of m [3][ny][nx] (device pointers). */
int mm_sno_eval(mm_sno *s, const float *m_dev, float *b_dev);
void mm_sno_destroy(mm_sno *s);
/* Let mm_run with solver 45 (magnetostatic term on, nz = 1, the surrogate's
 * grid equal to the context's) take B_demag from the surrogate at the inner
 * stages 2..6 of every Dormand-Prince attempt.  The last stage, at the new
 * state, is always exact; there the surrogate's prediction is compared with
 * the exact field, err = max_cells |B_sur - B_exact| / max_cells |B_exact|,
 * and if err > tol (or is not finite) the attempt is rejected with dt kept and
 * the rest of that mm_run call uses the exact path (fallback).  The surrogate
 * must outlive its use; s = NULL detaches it.  Allocates two field buffers
 * the first time.  A periodic grid returns MM_EUNSUPPORTED (the network
 * models open boundaries).  Synchronises. */
int mm_set_surrogate(mm_ctx *c, const mm_sno *s, double tol);
/* Accepted steps taken with surrogate stages since mm_set_surrogate,
 * fallbacks since the last solver restart, err of the last checked attempt. */
int mm_surrogate_stats(mm_ctx *c, int64_t *sur_steps, int64_t *fallbacks, double *last_err);

/* Training of the surrogate on the GPU (hand-written forward pass that keeps
 * its activations, backward pass and Adam; FP32 weights and arithmetic).  A
 * trainer holds the FP32 master weights (initialised from `weights`, host,
 * MM_SNO_NWEIGHTS values in the order above), Adam's two moments and the
 * activations of one batch of `batch` samples on an nx x ny grid
 * (32 <= nx <= 512, 16 <= ny <= 512, 1 <= batch <= 256).  m_dev and
 * target_dev are device arrays [batch][3][ny][nx] (target: B_demag /
 * out_scale, the network's output units).  The loss is the mean over the
 * batch of ||y_b - t_b||_2 / ||t_b||_2, y_b the network's output (the
 * gradient of a norm at 0 is taken as 0).
 *   mm_sno_train_grad: loss and its gradient with respect to the weights
 *     (grad_dev: MM_SNO_NWEIGHTS floats on the device, or NULL to keep it
 *     inside the trainer); no update.
 *   mm_sno_train_step: the same, then one Adam step (beta1 0.9, beta2 0.999,
 *     eps 1e-8, bias-corrected) with learning rate lr.
 * loss_out may be NULL: the call then returns without synchronising.  Work
 * is enqueued on hip_stream.  mm_sno_train_get_weights copies the current
 * FP32 weights to the host (synchronises). */
typedef struct mm_sno_trainer mm_sno_trainer;
int mm_sno_train_create(mm_sno_trainer **out, int32_t nx, int32_t ny, int32_t batch, const float *weights,
                        int64_t nweights, void *hip_stream);
int mm_sno_train_grad(mm_sno_trainer *t, const float *m_dev, const float *target_dev, float *grad_dev,
                      double *loss_out);
int mm_sno_train_step(mm_sno_trainer *t, const float *m_dev, const float *target_dev, double lr, double *loss_out);
int mm_sno_train_get_weights(mm_sno_trainer *t, float *weights_host);
void mm_sno_train_destroy(mm_sno_trainer *t);

void mm_destroy(mm_ctx *c);
const char *mm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
