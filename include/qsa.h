/*
 * qsa.h -- C ABI of the MI355X quasistatic (QSA) particle-in-cell hot path.
 *
 * Physics and units (paper, "Quasistatic model" section): a relativistic beam
 * of species s (charge Z_s e, mass M_s m_e, density ratio alpha_s = n_bs/n_p,
 * common Lorentz factor gamma_b) crosses a plasma of initially cold or warm
 * electrons over ions (immobile unless qsa_params.ion_m > 0).  Comoving
 * coordinates (xi, tau) = (ct - z, t); the plasma/field response is
 * quasistatic in xi at fixed tau and the beam evolves slowly in tau.  All
 * quantities are normalized: lengths to c/omega_p, times to 1/omega_p,
 * densities to n_p, momenta u = p/(M m_e c), fields to m_e c omega_p/e.
 * The propagation axis is z (the paper's x); transverse boundaries are
 * periodic and xi is open ("PIC simulations" section).
 *
 * One context = one simulation box on one GPU.  Per xi slice the library
 * deposits the plasma charge and current, solves the transverse
 * Poisson/Helmholtz problems for psi = phi - A_z (minus the paper's Psi,
 * defined after its Eq. (2)), E_z, B_z and B_perp by FFT, and advances the
 * plasma macro-particles to the next slice with a predictor-corrector; the
 * beam is then advanced by one Boris step of length dt in the stored 3D
 * fields.  Beyond the paper's runs (its conclusion's outlook) a context can
 * add a uniform guide field along z (qsa_params.b0z), a plasma density
 * profile with matching immobile ions (per-particle weights and
 * qsa_load_ions), and mobile plasma ions (qsa_params.ion_z, ion_m).
 *
 * Memory and ownership
 *   - The caller owns one device workspace of qsa_workspace_bytes() bytes
 *     (256-byte aligned) and the HIP stream; the library carves all of its
 *     device state out of the workspace and allocates no device memory.
 *   - The library owns only the host-side qsa_ctx; qsa_destroy frees it and
 *     never touches the workspace.
 *   - Every call enqueues work and returns without waiting, except the
 *     calls documented as synchronizing.  The library runs its kernels on
 *     a stream of its own, ordered after the work enqueued on the caller's
 *     stream before the call, and the caller's stream is ordered after the
 *     call's work; the sweep and the single beam step are captured once
 *     into HIP graphs and replayed (QSA_OPT_GRAPHS); a group of steps in
 *     flight is enqueued directly on two streams of the library's (the beam
 *     work of each slice tick alongside the next ticks of the slice loop).
 *   - A context is used from one host thread at a time.
 *
 * Errors
 *   - Invalid arguments, an undersized workspace or a wrong call order are
 *     reported at once by the return code.
 *   - Conditions found on the device (1 + psi <= 1e-3 at a plasma particle,
 *     i.e. quasistatic breakdown, or a non-finite value there) set a sticky
 *     device flag; the next synchronizing call returns QSA_E_BREAKDOWN and
 *     every later call returns it too, until qsa_destroy.
 *   - qsa_last_error() gives a readable reason for the last failure.
 *
 * Layouts
 *   - Grids are row-major [xi][y][x] (x fastest), nx*ny values per slice.
 *   - Particle arrays are structure-of-arrays, one float64 array per
 *     component; the library converts to its working precision.
 */
#ifndef QSA_H
#define QSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsa_ctx qsa_ctx;

typedef enum {
  QSA_OK = 0,
  QSA_E_INVALID = -1,    /* bad parameter or argument                      */
  QSA_E_NOMEM = -2,      /* workspace smaller than qsa_workspace_bytes()   */
  QSA_E_DEVICE = -3,     /* a HIP runtime call failed                       */
  QSA_E_BREAKDOWN = -4,  /* 1 + psi <= 1e-3 or non-finite at a particle     */
  QSA_E_NONFINITE = -5,  /* non-finite value in loaded particle data        */
  QSA_E_STATE = -6       /* call out of order (e.g. no plasma loaded)       */
} qsa_status;

enum { QSA_FP64 = 0, QSA_FP32 = 1 };

/* Field identifiers for qsa_fields().  The library stores psi, d_x psi,
 * d_y psi, E_z, B_x, B_y, B_z per slice; E_x = -d_x psi + B_y and
 * E_y = -d_y psi - B_x are formed on output.  QSA_SRC_* are the beam
 * sources (rho - J_z, J_x, J_y, J_z) of the last sweep. */
enum {
  QSA_PSI = 0, QSA_EX = 1, QSA_EY = 2, QSA_EZ = 3, QSA_BX = 4, QSA_BY = 5,
  QSA_BZ = 6, QSA_DXPSI = 7, QSA_DYPSI = 8,
  QSA_SRC_S = 9, QSA_SRC_JX = 10, QSA_SRC_JY = 11, QSA_SRC_JZ = 12
};

#define QSA_MAX_SPECIES 4
#define QSA_MAX_PIPELINE 16

typedef struct {
  int32_t Z;        /* charge number: -1 electron, +1 positron              */
  int32_t pad_;
  double M;         /* mass in electron masses                              */
} qsa_species;

/* Problem statement in normalized units (see header comment). */
typedef struct {
  int32_t nx, ny;        /* transverse cells, powers of two; nx in [8, 512],
                            ny = 1 (slab in x) or ny in [8, 512]            */
  int32_t nxi;           /* xi slices (>= 2); the head of the box is xi = 0  */
  int32_t precision;     /* QSA_FP64 or QSA_FP32                             */
  double dx, dy, dxi;    /* cell sizes in c/omega_p (dy is the slab depth)   */
  double dt;             /* beam time step in 1/omega_p                      */
  int32_t n_corr;        /* predictor-corrector iterations for B_perp (>= 0) */
  int32_t n_species;     /* beam species, 1..QSA_MAX_SPECIES                 */
  double kappa2;         /* Helmholtz shift of the B_perp iteration (> 0)    */
  int64_t n_plasma;      /* plasma macro-particles per slice (> 0)           */
  double plasma_w;       /* their common weight: area per particle (> 0)     */
  qsa_species species[QSA_MAX_SPECIES];
  int64_t beam_capacity[QSA_MAX_SPECIES]; /* max particles per species (>= 0) */
  int32_t pipeline;      /* beam steps in flight in qsa_beam_step, 0..16 (0 and 1:
                            one step at a time).  With P > 1 the workspace holds
                            P working sets (sources, fields, plasma state) and,
                            unless lean_pipeline, a copy of the beam; see
                            qsa_beam_step.                                   */
  int32_t adjoint_steps; /* 0, or the most beam steps qsa_adjoint_sweep will
                            differentiate (the workspace then holds the beam
                            and the 7 field planes for every step, plasma
                            checkpoints every ckpt_every slices, and the
                            adjoint arrays; see qsa_adjoint_sweep)          */
  int32_t ckpt_every;    /* adjoint plasma checkpoint stride in xi slices,
                            1..nxi (0: 16).  Memory of the checkpoints falls
                            and of the recomputed segment grows with it.    */
  int32_t no_field_pack; /* 0: without steps in flight the workspace keeps
                            the beam push's six fields packed per node for
                            every slice (32 bytes per cell in float32, 48
                            in float64; the push then gathers 16-byte
                            records); 1: it does not (the push gathers from
                            the stored planes), for boxes that need the
                            memory                                          */
  int32_t plasma_weights; /* 0: every plasma macro-particle has weight
                            plasma_w; 1: the workspace keeps a weight per
                            particle (random macro-particle weights, the
                            noise control of the "Extending the QSA to
                            extreme blazar jet regimes" section), loaded
                            with qsa_load_plasma_weights (until then all
                            plasma_w).  qsa_adjoint_sweep requires 0.      */
  int32_t lean_pipeline; /* with pipeline > 1: 0 keeps a second copy of the
                            beam (the group's sort target, the state a group
                            that breaks the drift schedule is repeated from
                            one step at a time, and the load order that
                            qsa_read_beam returns); 1 keeps none, for beams
                            too large to hold twice: each group's sort by
                            cell row gathers every beam array through the
                            sources and stored fields of working set 0 (so
                            the largest beam_capacity times 8 bytes must fit
                            in (4 + 7) nxi ny nx working-precision values,
                            else the parameters are invalid), qsa_read_beam
                            returns the particles in storage order (cell-row
                            order after a group), qsa_autotune does not try
                            steps in flight, and a group that breaks the
                            drift schedule fails with QSA_E_STATE (the beam
                            is then lost: the context keeps the error).
                            Not with adjoint_steps > 0.  Ignored with
                            pipeline <= 1.                                  */
  double b0z;            /* uniform external magnetic field along the
                            propagation axis (a guide field, in units of
                            m_e c omega_p / e; 0: none).  Added to the wake's
                            B_z in the plasma push and in the beam's Boris
                            push; not a source of the wake, and not stored in
                            the B_z that qsa_fields returns.  A static field
                            along z exerts no force along z, so the plasma's
                            gamma - u_z = 1 + psi still holds (the outlook of
                            the paper's conclusion lists external magnetic
                            fields).  Must be finite; 0 with adjoint_steps > 0. */
  double ion_m;          /* mass of mobile plasma ions in electron masses, or
                            0 (the ions are an immobile background, density
                            1 or the grid of qsa_load_ions).  With ion_m > 0
                            (contexts with plasma_weights = 1) the plasma
                            template may hold ions next to the electrons: a
                            negative weight in qsa_load_plasma_weights marks
                            one.  An ion keeps gamma - u_z = 1 - (Z/M) psi,
                            is pushed with the electrons' equations scaled
                            by -Z/M and carries +Z w (ion motion is in the
                            outlook of the paper's conclusion).  Finite and
                            >= 0.                                           */
  int32_t ion_z;         /* their charge number, 1..64 (with ion_m > 0)      */
  int32_t pad2_;
} qsa_params;

/* Bytes of device workspace a context with these parameters needs; 0 if the
 * parameters are invalid. */
size_t qsa_workspace_bytes(const qsa_params* p);

/* Create a context.  dev_ws: device pointer to >= qsa_workspace_bytes(p)
 * bytes, 256-byte aligned; hip_stream: a hipStream_t (NULL = default
 * stream).  On success *out holds the context.  Synchronizing (it uploads
 * transform tables). */
qsa_status qsa_create(const qsa_params* p, void* dev_ws, size_t ws_bytes,
                      void* hip_stream, qsa_ctx** out);

/* Load the plasma template (the cold or warm plasma electrons of the
 * problem statement, "Quasistatic model" section): the n = p->n_plasma macro-particles that enter
 * every slice sweep at xi = 0 (positions x, y in [0, L), momenta u_x, u_y;
 * u_z follows from gamma - u_z = 1).  Arrays are float64, host memory when
 * on_device = 0 (the call then synchronizes), device memory otherwise.
 * Returns QSA_E_NONFINITE for a non-finite host value. */
qsa_status qsa_load_plasma(qsa_ctx* c, const double* x, const double* y,
                           const double* ux, const double* uy, int64_t n,
                           int32_t on_device);

/* Per-particle weights of the loaded plasma template (contexts created
 * with plasma_weights = 1; after qsa_load_plasma, which resets them to
 * plasma_w): w[i] is the weight of template particle i in the units of
 * plasma_w (area per particle times the local density, so that a uniform
 * plasma has w[i] = plasma_w); each particle deposits -w[i]/(dx dy) times
 * its shape.  n must equal n_plasma.  Float64, host (synchronizing; every
 * value finite and >= 0, else QSA_E_NONFINITE) or device memory.  With
 * mobile ions (ion_m > 0) a negative w[i] makes particle i an ion of weight
 * -w[i] (charge ion_z, mass ion_m); host values then need only be finite.
 * QSA_E_STATE without plasma_weights or before a template is loaded. */
qsa_status qsa_load_plasma_weights(qsa_ctx* c, const double* w, int64_t n, int32_t on_device);

/* Density of the immobile ions at the nodes, n_i[l * nx + i] at
 * (x_i, y_l) = (i dx, l dy), in units of the reference density (contexts
 * created with plasma_weights = 1; qsa_load_plasma resets it to 1
 * everywhere).  With the electrons' weights of qsa_load_plasma_weights
 * scaled by the same profile, this is an inhomogeneous plasma that enters
 * the box neutral (plasma inhomogeneity is in the outlook of the paper's
 * conclusion): the ions add n_i to rho - J_z of every slice.  Loading new
 * weights and ions between beam steps makes the density change along the
 * propagation distance.  n must equal nx * ny.  Float64, host
 * (synchronizing; every value finite and >= 0, else QSA_E_NONFINITE) or
 * device memory.  QSA_E_STATE without plasma_weights or before a template
 * is loaded. */
qsa_status qsa_load_ions(qsa_ctx* c, const double* n_i, int64_t n, int32_t on_device);

/* Load n (<= capacity) particles of beam species s (the beam species of
 * the problem statement; flat-top loading as in the "PIC simulations"
 * section): position (x, y, xi),
 * momentum (u_x, u_y, u_z) and weight w (number of physical particles per
 * unit n_p, i.e. alpha dV/ppc for a uniform beam).  A particle with w = 0 is
 * inert.  Float64 arrays, host (synchronizing) or device memory.  Any order;
 * with pipeline > 1 the library keeps the particles sorted by cell row
 * internally (each group of steps starts with that sort), and qsa_read_beam
 * still returns them in the order they were loaded (with pipeline = 1 too,
 * unless QSA_OPT_RESORT_EVERY reorders the storage). */
qsa_status qsa_load_beam(qsa_ctx* c, int32_t s, const double* x,
                         const double* y, const double* xi, const double* ux,
                         const double* uy, const double* uz, const double* w,
                         int64_t n, int32_t on_device);

/* Load a beam of species s in parts, for beams too large to stage at once
 * (the 512 x 512 x 2048 pair beam holds 2.1e9 particles per species):
 * particles [first, first + n) of the species, in the layout of
 * qsa_load_beam.  first = 0 starts a new beam of n particles; first equal
 * to the species' current count appends n; first + n <= capacity.  The
 * species then holds first + n particles, in load order.  With pipeline > 1
 * the sort by cell row is left to the next group of steps in flight (every
 * group starts with it).  Host arrays synchronize; QSA_E_INVALID for any
 * other first, QSA_E_NONFINITE for a non-finite host value. */
qsa_status qsa_load_beam_range(qsa_ctx* c, int32_t s, int64_t first, const double* x,
                               const double* y, const double* xi, const double* ux,
                               const double* uy, const double* uz, const double* w,
                               int64_t n, int32_t on_device);

/* Copy the current particles of species s out as float64 (7 arrays of at
 * least *n entries; cap = their length).  Synchronizing when on_device = 0. */
qsa_status qsa_read_beam(qsa_ctx* c, int32_t s, double* x, double* y,
                         double* xi, double* ux, double* uy, double* uz,
                         double* w, int64_t cap, int64_t* n, int32_t on_device);

/* One quasistatic sweep at the current tau (the field and plasma equations
 * at fixed tau of the "Quasistatic model" section, whose linearization is
 * Eqs. (1)-(2)): beam sources from the beam particles, then the plasma
 * response slice by slice from xi = 0 to the tail.  Fields of every slice
 * are kept until the next sweep. */
qsa_status qsa_slice_sweep(qsa_ctx* c);

/* n_steps x (qsa_slice_sweep; Boris push of every beam species by dt): the
 * slow evolution of the beam in tau in the quasistatic fields ("Quasistatic
 * model" section; linearized, Eq. (3)).
 *
 * With pipeline = P > 1 the steps run in groups of up to P steps in flight:
 * step n0 + k sweeps QSA_PIPE_LAG = 8 slices behind step n0 + k - 1 in the
 * same kernel launches.  This relies on the beam drifting only backwards in
 * xi by less than a few cells per step: each beam particle is pushed by step
 * n0 + k as soon as that step has finished the slices around the cell row it
 * was loaded in, and deposited for step n0 + k + 1 right away.  The results
 * are those of one step at a time (up to the order of floating-point
 * additions).  If a particle has moved too far from the cell row it was
 * loaded in, the group is detected on the device, the beam is restored from
 * the copy taken at the group's start, the group is repeated one step at a
 * time and pipelining stays off until the next qsa_load_beam.  Pipelined
 * calls synchronize once per group (to read that flag). */
qsa_status qsa_beam_step(qsa_ctx* c, int32_t n_steps);

/* Fields of the last sweep (psi is minus the paper's Psi of Eq. (2); the
 * transverse force on a v = c particle is -grad psi, the paper's F_perp).
 * Copy slices [xi0, xi1) of one field of the last sweep as float64 into dst
 * (count >= (xi1 - xi0) * nx * ny values), host or device memory.
 * Synchronizing; reports a pending device error. */
qsa_status qsa_fields(qsa_ctx* c, int32_t field, int32_t xi0, int32_t xi1,
                      double* dst, size_t count, int32_t dst_on_device);

/* Diagnostics of the last sweep, reduced on the device (no copy of the 3D
 * fields): the transverse field amplitudes and field energies the paper
 * follows at positions along the beam (Fig. 2; Fig. 3(d,e) and the
 * saturation estimates, which take eps_F = <F^2>/(4 n_b gamma_b) in these
 * units).  Slices are grouped in windows of `window` consecutive slices
 * (the last one may be shorter).  dst[w*6 + f] = the mean over window w's
 * slices of the transverse mean of F^2, F = (E_x, E_y, E_z, B_x, B_y, B_z)
 * in that order (E_x = -d_x psi + B_y, E_y = -d_y psi - B_x); count >=
 * 6 ceil(nxi/window) doubles, host or device memory (dst_on_device).
 * Accumulated in float64.  Synchronizing; QSA_E_STATE before any sweep. */
qsa_status qsa_field_moments(qsa_ctx* c, int32_t window, double* dst, size_t count, int32_t dst_on_device);

/* Beam momentum moments of species s (the spreads of the paper's Fig.
 * 3(f)): dst[w*7 + k] = the sum over the particles with w_p != 0 and slice
 * floor(xi/dxi) in window w (slices [0, nxi) only) of k = (w_p, w_p u_x,
 * w_p u_y, w_p u_z, w_p u_x^2, w_p u_y^2, w_p u_z^2); the weighted RMS
 * spread is sqrt(sum w u^2/sum w - (sum w u/sum w)^2).  count >=
 * 7 ceil(nxi/window) doubles, host or device memory.  Accumulated in float64
 * (atomic sums: the order of additions varies).  Synchronizing. */
qsa_status qsa_beam_moments(qsa_ctx* c, int32_t species, int32_t window, double* dst, size_t count,
                            int32_t dst_on_device);

/* Batched solver of the single-mode linear model, Eq. (5) of the paper,
 * [(d_xi^2 + 1) d_tau^2 - Gamma^2] dPsi = 0, the tool the paper compares its
 * simulations with (its Fig. 1(e)) and from which growth rates along the
 * beam are read.  It is solved as n = (d_xi^2 + 1) dPsi with the causal
 * inverse dPsi(xi) = int_0^xi sin(xi - xi') n(xi') dxi' (trapezoid rule on
 * xi_j = j dxi, j < nxi) and d_tau^2 n = Gamma^2 dPsi by classical RK4 in
 * tau with step dtau, from n(xi, 0) = n0 and d_tau n(xi, 0) = 0, for n_inst
 * independent instances (one Gamma and one seed each) at once.  A
 * longitudinal beam profile enters through Gamma(xi), the paper's
 * generalization of Eq. (5): d_tau^2 n = Gamma(xi)^2 dPsi point by point.
 *   gamma: device memory (float64), [n_inst] (gamma_per_point = 0) or the
 *     profiles [n_inst][nxi] (gamma_per_point = 1);
 *   n0 [n_inst][nxi]: device memory (float64);
 *   taus [n_tau]: host memory, output times (each reached in
 *     round((tau_m - tau_{m-1})/dtau) steps, ties to even; non-decreasing);
 *   n_out, psi_out [n_inst][n_tau][nxi]: device memory, n and dPsi at them.
 * Limits: nxi <= 4096, n_tau <= 256.  Enqueued on hip_stream (a hipStream_t,
 * null for the default stream) without synchronizing; QSA_E_INVALID for
 * arguments out of range (nothing launched), QSA_E_DEVICE if the launch
 * fails.  Needs no context. */
qsa_status qsa_linear_model(int32_t n_inst, int32_t nxi, double dxi, double dtau, const double* gamma,
                            int32_t gamma_per_point, const double* n0, int32_t n_tau, const double* taus, double* n_out, double* psi_out,
                            void* hip_stream);

/* Conducting-wall (Dirichlet) transverse solves by sine transforms, the
 * sine-transform form of the field equations' transverse solves (the
 * pseudo-potential's Poisson equation, Eq. (2) in its linear form, and the
 * Helmholtz-shifted B_perp iteration) for a box whose walls hold the
 * potential at zero.  For n_grid independent grids f[g][ny][nx] of values
 * at the interior nodes x_i = i dx (i = 1..nx, walls at 0 and (nx+1) dx) and
 * y_l = l dy (l = 1..ny), solve (-lap_perp + kappa2) u = f with u = 0 on the
 * walls, in the wall modes sin(m pi x/L_x) sin(n pi y/L_y) (m <= nx,
 * n <= ny; L = (N+1) d) with their exact eigenvalues (m pi/L_x)^2 +
 * (n pi/L_y)^2 + kappa2; ny = 1 is a slab with x walls only.
 *   precision: QSA_FP64 (f, u double) or QSA_FP32 (float);
 *   nx + 1 and (unless ny = 1) ny + 1 powers of two in [2, 512];
 *   dx, dy > 0; kappa2 >= 0 (0: Poisson);
 *   f, u: device memory [n_grid][ny][nx], row-major (x fastest); u may be f
 *     (in place) but must not overlap it otherwise.
 * Enqueued on hip_stream (a hipStream_t, null for the default stream)
 * without synchronizing: three launches (one for a slab).  QSA_E_INVALID for
 * arguments out of range (nothing launched), QSA_E_DEVICE if a launch
 * fails.  Needs no context. */
qsa_status qsa_dirichlet_solve(int32_t precision, int32_t n_grid, int32_t nx, int32_t ny, double dx, double dy,
                               double kappa2, const void* f, void* u, void* hip_stream);

/* Wait for the stream and report any pending device error. */
qsa_status qsa_sync(qsa_ctx* c);

/* Kernel classes that qsa_timing_begin can time. */
enum {
  QSA_K_PUSH_PRED = 0,   /* plasma predictor push + predicted J_perp deposit  */
  QSA_K_PUSH_FINAL = 1,  /* plasma advance to the next slice                  */
  QSA_K_DEP_S = 2,       /* plasma rho - J_z deposit                          */
  QSA_K_DEP_J = 3,       /* plasma J deposit                                  */
  QSA_K_ROW_R2C = 4,     /* row transforms, real -> half spectrum             */
  QSA_K_COL = 5,         /* column transforms with the spectral solves        */
  QSA_K_ROW_C2R = 6,     /* row transforms, half spectrum -> real             */
  QSA_K_BEAM_DEPOSIT = 7,/* beam source deposit                               */
  QSA_K_BEAM_PUSH = 8,   /* beam Boris push                                   */
  QSA_K_COUNT = 9
};

/* Start timing every launch of one kernel class with a pair of HIP events
 * recorded on the context's work stream around it (at most 1<<17 launches
 * per window; later launches run untimed).  Instrumentation for
 * measurement: while timing is on, the sweep and the beam step are enqueued
 * launch by launch (no graph replay). */
qsa_status qsa_timing_begin(qsa_ctx* c, int32_t kernel_class);

/* Stop timing; synchronizing.  *total_ms = summed kernel time of the timed
 * launches, *launches = their count. */
qsa_status qsa_timing_end(qsa_ctx* c, double* total_ms, int64_t* launches);

/* Options for qsa_set_option / qsa_get_option. */
enum {
  QSA_OPT_GRAPHS = 0,    /* 1 (default): replay a captured HIP graph of the sweep
                            and of the single beam step; 0: enqueue every
                            launch (groups of steps in flight, and single
                            steps with QSA_OPT_BEAM_BESIDE, always are)     */
  QSA_OPT_PIPELINE = 1,  /* beam steps in flight in qsa_beam_step: set 1..P
                            (values above the parameter's pipeline = P are
                            clamped to P; setting also re-enables pipelining
                            after a drift fallback); get: the depth in use,
                            1 when pipelining is off                        */
  QSA_OPT_PLASMA_THREADS = 2, /* threads per plasma cell-row block: 64, 128,
                            256, 512 (float32 only), or 0 for the default
                            (from the particles per row, at most 512 in
                            float32 and 256 in float64); get: the value in
                            use                                             */
  QSA_OPT_ROW_THREADS = 3, /* threads per row-transform block: 64, 128, 256
                            (a multiple of nx/4), or 0 for
                            min(256, max(64, nx/2));
                            get: the value in use                           */
  QSA_OPT_COL_THREADS = 4, /* threads per column transform: 16, 32 or 64 (a
                            wavefront takes 64 / value adjacent columns), or
                            0 for 64; at most ny/4 are used; get: the value
                            in use                                          */
  QSA_OPT_BEAM_BESIDE = 5, /* contexts without steps in flight (pipeline = 1):
                            1 runs a beam step's source deposit and
                            push on a second stream beside the slice loop, a
                            few slabs at a time (the deposit ahead of the
                            slice that needs it, the push once the fields it
                            gathers are final); 0 (default): deposit, sweep,
                            push one after the other.  The results agree up to the
                            order of the deposit's additions.              */
  QSA_OPT_BESIDE_BLOCKS = 6, /* workgroups per launch of the beam work beside
                            the slice loop: 0 (default) as many as the work
                            has; n > 0 caps every such launch at n (each
                            workgroup then loops over its share), leaving
                            the rest of the chip to the slice loop       */
  QSA_OPT_RESORT_EVERY = 7 /* contexts without steps in flight: n > 0
                            reorders the beam's storage by deposit key (cell
                            row, slab-major) before every n-th beam step of
                            qsa_beam_step, counted from the last beam load
                            (so the first step after a load re-sorts), which
                            keeps the deposit's and the push's memory access
                            coalesced as particles drift across cells; the
                            step's sources and stored fields serve as
                            scratch, so the largest beam_capacity times 8
                            bytes must fit in them (else the setting is
                            refused).  qsa_read_beam then returns particles
                            in storage order, no longer the load order; the
                            order within a cell row is unspecified.  0
                            (default): never.  Refused for contexts with
                            steps in flight (they sort the beam by cell row
                            themselves and keep the load order). */
};

/* Set a context option (see QSA_OPT_*). */
qsa_status qsa_set_option(qsa_ctx* c, int32_t option, int64_t value);

/* Read a context option (see QSA_OPT_*) into *value. */
qsa_status qsa_get_option(const qsa_ctx* c, int32_t option, int64_t* value);

/* Gradient of the transverse magnetic energy with respect to beam-amplitude
 * bins (requires adjoint_steps >= n_steps at create).  The paper has no
 * adjoint: this differentiates the discrete form of its quasistatic model
 * (the operations of qsa_slice_sweep and qsa_beam_step); the field energy is
 * the quantity behind its saturation estimates (discussion of Fig. 3).
 *
 * Starting from the beam as loaded (or as left by the last step), with every
 * particle's weight scaled by amps[bin] (bins[s][p] in [0, n_bins): the bin of
 * particle p of species s, host arrays of beam_n[s] entries; a particle with
 * a bin outside that range keeps its weight), the call runs n_steps beam
 * steps and one more sweep, *loss = 1/2 sum (B_x^2 + B_y^2) dx dy dxi over
 * every node of that last sweep, and grad[b] = d loss / d amps[b] (host
 * array of n_bins).  The derivative is that of the discrete scheme (sweeps,
 * deposits, Boris pushes), computed in reverse with the beam and fields of
 * every step kept and the plasma recomputed between checkpoints every 16
 * slices.  Its forward passes use their own simple kernels (no pipelining,
 * the plasma never reordered).  The context's beam, fields and options are
 * unchanged.  Synchronizing.  n_bins <= 4096. */
qsa_status qsa_adjoint_sweep(qsa_ctx* c, int32_t n_steps, int32_t n_bins, const double* amps,
                             const int32_t* const* bins, double* loss, double* grad);

/* Autotuner (launch shapes only, nothing the paper defines): times real work
 * on this context's data (direct launches, HIP events) and keeps the fastest
 * threads per plasma-row block (64/128/256), threads per row-transform block
 * (64/128/256, multiples of nx/4), threads per column transform and, with
 * pipeline > 1, beam steps in flight (2, 4, ... up to pipeline).  A trial is
 * a group of steps in flight, after which the beam is restored, or (pipeline
 * <= 1) one sweep.  The beam and the device flags are as before the call;
 * fields are invalid until the next sweep.  *ms_per_step (may be NULL)
 * receives the best time per step (per sweep without pipelining).
 * Synchronizing; about 10 trials.  The shapes chosen change the order of
 * floating-point additions only. */
qsa_status qsa_autotune(qsa_ctx* c, double* ms_per_step);

/* ---------------------------------------------------------------------------
 * Batches: many independent boxes (a growth-rate parameter scan: different
 * nx, ny, nxi, alpha, gamma_b, dt per box, as in the paper's comparison of
 * growth rates across beam parameters in its results section) advanced
 * together.  The slice
 * loops of all member contexts run as lanes of the same kernel launches (one
 * launch per phase per slice for the whole batch; a box with fewer slices
 * drops out), and the whole batched sweep or step is captured once into a
 * HIP graph and replayed.  Members keep their own workspaces, beams and
 * fields (read them with qsa_fields / qsa_read_beam on each context); they
 * must share precision and n_corr, have their plasma loaded, and not be used
 * on their own while the batch runs work.
 * ------------------------------------------------------------------------- */
typedef struct qsa_batch qsa_batch;

/* Device bytes of the batch's lane table (256-byte aligned). */
size_t qsa_batch_workspace_bytes(int32_t n_ctx);

/* Create a batch over n_ctx distinct contexts.  dev_ws: device memory of
 * qsa_batch_workspace_bytes(n_ctx) bytes; hip_stream: the caller's stream
 * (the batch orders its work after it and it after the batch's work).
 * Synchronizing. */
qsa_status qsa_batch_create(qsa_ctx* const* ctxs, int32_t n_ctx, void* dev_ws, size_t ws_bytes,
                            void* hip_stream, qsa_batch** out);

/* One sweep of every member (beam deposit + slice loop). */
qsa_status qsa_batch_sweep(qsa_batch* b);

/* n_steps x (sweep of every member; Boris push of every member's beam). */
qsa_status qsa_batch_step(qsa_batch* b, int32_t n_steps);

/* Wait for the batch's work and report any member's pending device error. */
qsa_status qsa_batch_sync(qsa_batch* b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one sweep
 * of every member context (their beam deposits, then their slice loops as
 * lanes of the same launches), the same work as qsa_batch_sweep, without a
 * batch object or its workspace.  The lane table (one descriptor per
 * member) lives in a static device array of the library, QSA_STATIC_MAX_CTX
 * descriptors (about 50 KB) per device, held until the process ends; the
 * members' fields, beams and scratch stay in their own workspaces.
 *   ctxs[n_ctx]: distinct contexts with plasma loaded, one precision and
 *     n_corr; 1 <= n_ctx <= QSA_STATIC_MAX_CTX (else QSA_E_INVALID with a
 *     message in qsa_last_error(ctxs[0])).
 *   hip_stream: the stream every launch is enqueued on (a hipStream_t, null
 *     for the default stream); nothing synchronizes.  Pass the stream the
 *     members were created with: each context call orders that stream after
 *     its own work, so this call then follows the members' earlier calls
 *     and their later calls follow it.
 * No device memory is allocated or freed, and no stream, event or graph is
 * created.  Every call on one device rewrites that device's table, so calls
 * that overlap on one device (enqueued on different streams) race; calls in
 * one stream order do not.  Read results with qsa_fields on each member.
 * Errors: QSA_E_INVALID / QSA_E_STATE for bad arguments (nothing enqueued),
 * a member's sticky status, QSA_E_DEVICE if a launch fails. */
#define QSA_STATIC_MAX_CTX 64
qsa_status qsa_batch_sweep_static(qsa_ctx* const* ctxs, int32_t n_ctx, void* hip_stream);

/* Free the batch (member contexts and workspaces are not touched). */
qsa_status qsa_batch_destroy(qsa_batch* b);

/* Free the host context (the workspace is not touched). */
qsa_status qsa_destroy(qsa_ctx* c);

const char* qsa_status_string(qsa_status s);
const char* qsa_last_error(const qsa_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* QSA_H */
