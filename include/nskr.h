/*
 * nskr.h -- C ABI of the MI355X (gfx950) library for the DGSEM right-hand side
 * and low-storage Runge-Kutta update of relaxation models 1 and 2 of the
 * non-isothermal Navier-Stokes-Korteweg equations with a van der Waals
 * equation of state (Keim, Munz, Rohde, arXiv 2208.05310).
 *
 * The system (Sec. 2.3.2, flux and source vectors of relaxation model 1;
 * model 2 replaces p by p_alpha = p + alpha/2 rho^2 in F^C, eq.
 * modified_pressure, and moves the matching terms out of S) is
 *   U_t + div(F^C(U) - F^V(U, grad U, lap c)) = S(U, grad U),
 *   U = (rho, rho u, rho v, rho w, rho e, c),
 * discretised as in Sec. 3.1: nodal DGSEM on Legendre-Gauss nodes with
 * collocated quadrature, Rusanov (model 2: HLLC) face flux for F^C, BR1
 * lifting for the gradients, point-wise sources, explicit low-storage RK4.
 * Walls follow the
 * relaxation-model boundary conditions of Sec. 2.4 (eq. bc_nsk_alpha) with the
 * cubic wall energy (eq. helmfreesurftot_derivative), enforced weakly through
 * the face flux (Sec. 3.2).
 *
 * Conventions
 *  - Every call returns an int status (NSKR_OK = 0).  Arguments are validated
 *    before anything is enqueued.  After NSKR_E_HIP the context is poisoned
 *    and later calls return NSKR_E_STATE until nskr_destroy.
 *  - A context is not thread-safe: one host thread per context.
 *  - State buffers U, R, U_t are caller-owned device memory (e.g. torch
 *    tensors), contiguous, structure-of-arrays [6][nelems][(N+1)^3] with the
 *    node index i + (N+1)(j + (N+1)k), i along the first reference direction.
 *    Element type is double for precision 0 (FP64) and float for precision 1
 *    (FP32-mixed).
 *  - Work is enqueued on the caller's stream and is asynchronous, except for
 *    the calls documented as synchronising (they return host values).
 *  - Only compute on the device: there is no CPU fallback.  If the device
 *    code is unavailable, nskr_create fails with NSKR_E_HIP.
 */
#ifndef NSKR_H
#define NSKR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSKR_ABI_VERSION 9  /* 9: nskr_mesh of geometry nodes (degree ngeo) with face orientations; 8: nskr_dt_noalloc; 7: batches advance the context time and admit walls that change in time; 6: nskr_bc.twall_rate, context time; 5: nskr_init.cylinder_axis; 4: twall_grad */

enum {
    NSKR_OK = 0,
    NSKR_E_ARG = 1,          /* invalid argument; nothing enqueued          */
    NSKR_E_STATE = 2,        /* call out of order or context poisoned       */
    NSKR_E_NOMEM = 3,        /* device allocation failed                    */
    NSKR_E_HIP = 4,          /* a HIP runtime call failed                   */
    NSKR_E_NONFINITE = 5,    /* non-finite or out-of-range state detected   */
    NSKR_E_UNSUPPORTED = 6   /* valid request the library does not implement */
};

typedef struct nskr_ctx nskr_ctx;
typedef void *nskr_stream; /* a hipStream_t; NULL is the default stream */

/* Physical and numerical parameters.  R, a, b: reduced van der Waals
 * constants (Sec. 2.1: 8/3, 3, 1/3); cv: c_v; mu: viscosity (Stokes
 * hypothesis); kappa: heat conductivity; gam: capillarity gamma_K; alpha:
 * Korteweg parameter; beta: relaxation parameter (Sec. 2.3.2); cfl: CFL number
 * (0.9, Sec. 4).  precision: 0 = FP64 everywhere; 1 = FP32-mixed (FP32 state
 * and bulk arithmetic; temperature recovery, pressure and sound speed in FP64;
 * time-step and integral reductions in FP64). */
typedef struct {
    double R, a, b, cv, mu, kappa, gam, alpha, beta, cfl;
    int precision;
    int kahan;   /* FP32-mixed only: 1 = compensated (Kahan) state update, which
                    carries the rounding error of U += B R from stage to stage */
    int model;   /* relaxation model (Sec. 2.3.2): 0 or 1 = model 1 (Rusanov
                    interior flux); 2 = model 2: pressure p_alpha = p + alpha/2
                    rho^2 in the convective flux (eq. modified_pressure), the
                    alpha rho grad rho source terms folded into it (eq.
                    navierstokeskorteweg_palpha), HLLC interior flux, sound
                    speed sqrt(c_s^2 + alpha rho) */
} nskr_params;

/* Wall boundary condition (Sec. 2.4, eq. bc_nsk_alpha; weak enforcement
 * through the face flux, Sec. 3.2).  All walls are impermeable.
 *   kind 1: no-slip isothermal wall at twall with a static contact angle
 *     theta_deg (cubic wall energy, eq. helmfreesurftot_derivative, Maxwell
 *     states and sigma_vl evaluated at twall), moving with the tangential
 *     velocity uwall (a lid; zero for a fixed wall).
 *   kind 2: slip adiabatic wall with neutral wetting (zero contact-angle flux,
 *     zero tangential traction).
 *   kind 3: generalized Navier-slip wall: tangential traction gamma1 div u
 *     grad_Gamma c - gamma2 (u_t - uwall) (eq. bc_navierstokes_alpha),
 *     contact-angle flux grad c . n = (gamma1 div u - dpsi/dc) / gamma at
 *     twall and theta_deg (eq. bc_contactangle_alpha), wall value zeta_c =
 *     -gamma1 gamma4 div u of the relaxation condition (eq.
 *     bc_relaxation_alpha), and heat flux k grad T . n = -gamma3 (1/twall -
 *     1/T) (eq. bc_energy_alpha); gamma3 = +infinity makes it isothermal at
 *     twall.
 * gamma1..gamma4 >= 0 and are read for kind 3 only; uwall must be tangential
 * to every face of the wall (NSKR_E_ARG otherwise) and is read for kinds 1
 * and 3.  twall_grad, twall_rate (kinds 1, 3): the wall temperature at a
 * wall point x and time t is twall + twall_grad . x + twall_rate t; when
 * either is non-zero, sigma_vl and the Maxwell states at that temperature
 * come from a table of Sec. 3.2 (10000 equidistant temperatures on [0.3, 1],
 * sigma by a 15-point Gauss rule, linear interpolation) at every wall face
 * point and stage, and the wall temperature must stay in [0.3, 0.99] on the
 * whole wall: at mesh upload for t = 0, and over the time span of every
 * call that evaluates the operator or admits the context into a batch
 * (NSKR_E_ARG otherwise). */
typedef struct {
    int kind;
    double twall;
    double theta_deg;
    double uwall[3];
    double gamma1, gamma2, gamma3, gamma4;
    double twall_grad[3];
    double twall_rate;
} nskr_bc;

/* Hexahedral mesh (Sec. 3.1: each element mapped from the reference cube
 * [-1,1]^3; curved elements with a geometry of degree N_geo <= N, e.g. the
 * N_geo = 2 elements of Sec. 4.5).
 *   ngeo: geometry degree, 1..N.
 *   xgeo[e][(ngeo+1)^3][3]: the element's geometry nodes on the Gauss-Lobatto
 *     points of degree ngeo, node a + (ngeo+1)(b + (ngeo+1)c) at reference
 *     coordinates (xi_a, xi_b, xi_c), a along the first reference direction
 *     (ngeo = 1: the 8 corners, v = i + 2j + 4k).  The element is the
 *     polynomial interpolant of these nodes; J > 0 is required at every node.
 *   Faces: 0 = xi^1 = -1, 1 = +1, 2/3 = xi^2, 4/5 = xi^3; face point p + (N+1) q
 *     with (p, q) the node indices along the two remaining directions in
 *     increasing order.
 *   nbr[e][f]: neighbour element, or -1 on a wall.
 *   nbr_face[e][f]: the neighbour's local face (any of 0..5).
 *   nbr_orient[e][f] (NULL: all 0): orientation o in 0..7 taking own face
 *     point (p, q) to the neighbour's point (a, b): (a, b) = (q, p) if o & 4,
 *     else (p, q); then a -> N - a if o & 1 and b -> N - b if o & 2.  The
 *     neighbour's entry for the same face must be the inverse map.
 *   bc[e][f]: 0 for interior faces, else a 1-based index into bcs.
 * The library checks that the connectivity is reciprocal, that each face and
 * its neighbour's face are the same surface (matching points differ by one
 * translation: zero, or a period of the domain) with opposite normals and
 * equal surface elements, and forms the metric terms Ja^d_m = J d xi^d/d x_m
 * itself in the conservative curl form (Kopriva 2006), in extended precision.
 * Meshes whose elements are all parallelepipeds keep per-element metrics;
 * otherwise every node carries its own (10 values) and every face point its
 * own normal.  All arrays are host memory; the library copies them. */
typedef struct {
    int nelems;
    int ngeo;
    const double *xgeo;
    const int *nbr;
    const int *nbr_face;
    const int *nbr_orient;
    const int *bc;
    int nbcs;
    const nskr_bc *bcs;
} nskr_mesh;

/* Droplet initial condition: rho = rho_v + sum_j (rho_l - rho_v)/2 (1 +
 * tanh((r_j - d_j)/width)) (the tanh profiles of Sec. 4.1.1, 4.2 and 4.3 with
 * their width given directly), d_j the distance to centre j, taken as the
 * minimum image along the axes flagged periodic (box extent length[]);
 * rho_v, rho_l are the Maxwell densities at T0 unless both fields below are
 * positive (e.g. the Young-Laplace adjusted densities of the collision cases,
 * Sec. 4.3, Table 5).  Velocity u = sum_j v_j (1 + tanh((r_j - d_j)/width))/2, each
 * droplet carrying its own velocity v_j (zero when velocities is NULL);
 * m = rho u; c = rho; rho e from eq. totalenergyalpha with the lifted grad c
 * and the kinetic energy, so that the recovered temperature is T0.
 * cylinder_axis in 0..2 makes every droplet a cylinder along that axis (the
 * liquid pillar of Sec. 4.4.1; d_j measured in the normal plane), -1 keeps
 * spheres.  centres: ndrop x 3, radii: ndrop, velocities: ndrop x 3 or NULL;
 * host memory. */
typedef struct {
    double T0;
    int ndrop;
    const double *centres;
    const double *radii;
    double width;
    double length[3];
    int periodic[3];
    const double *velocities;
    double rho_v, rho_l;
    int cylinder_axis;
} nskr_init;

/* Integrals returned by nskr_reduce (Gauss quadrature with the Jacobian, FP64
 * accumulation in a fixed order). */
enum {
    NSKR_SUM_MASS = 0, NSKR_SUM_MOMX = 1, NSKR_SUM_MOMY = 2, NSKR_SUM_MOMZ = 3,
    NSKR_SUM_ENERGY = 4, NSKR_SUM_C = 5, NSKR_SUM_KINETIC = 6,
    NSKR_SUM_GRADIENT_ENERGY = 7, /* gamma/2 |grad c|^2                 */
    NSKR_SUM_RELAX_ENERGY = 8,    /* alpha/2 (rho - c)^2                */
    NSKR_SUM_RHO_MINUS_C_SQ = 9,  /* (rho - c)^2                        */
    NSKR_SUM_MIN_RHO = 10, NSKR_SUM_MAX_RHO = 11,
    NSKR_SUM_MIN_T = 12, NSKR_SUM_MAX_T = 13,
    NSKR_CNT_NONFINITE = 14, NSKR_CNT_RHO_RANGE = 15, NSKR_CNT_T_NONPOS = 16,
    NSKR_CNT_CS2_NEG = 17,
    NSKR_SUM_ENTROPY = 18,        /* -int rho eta, eta = R c_v ln T - R ln(b rho/(1-b rho)) */
    NSKR_SUM_VOLUME = 19,
    NSKR_NSUMS = 20
};

/* ABI version (NSKR_ABI_VERSION). */
int nskr_version(void);

/* Create a context for polynomial degree N (2..5) on HIP device `device`.
 * No device memory is allocated yet.  Errors: NSKR_E_ARG (N out of range,
 * negative mu, kappa, gam, alpha or beta, b < 0, cv <= 0, R <= 0, cfl <= 0,
 * precision not 0/1, out == NULL); NSKR_E_HIP (device missing or no device code
 * for it). */
int nskr_create(const nskr_params *p, int N, int device, nskr_ctx **out);

/* Free library-owned device memory and the context.  Never frees caller
 * buffers.  Safe on NULL. */
int nskr_destroy(nskr_ctx *ctx);

/* Upload the mesh (see nskr_mesh): metric terms, outward face normals and
 * surface elements, connectivity and per-wall constants (Maxwell states,
 * sigma_vl of eq. surftenscoef read with the factor sqrt(2 gamma));
 * allocates the library's scratch (lifted gradients, face traces).  May be
 * called again to replace the mesh.  Errors: NSKR_E_ARG (null arrays, ngeo
 * outside 1..N, non-finite geometry, J <= 0, neighbour indices, faces or
 * orientations out of range, connectivity not reciprocal or orientations not
 * inverse, a face whose neighbour's face is not the same surface under the
 * given orientation or has a different normal or surface element, wall face
 * without a bc or bc index out of range, wall kind not 1, 2 or 3, negative
 * Navier-slip coefficients, a wall velocity that is not tangential at every
 * face point, supercritical wall temperature); NSKR_E_UNSUPPORTED (walls
 * whose temperature varies on a mesh with curved elements, or a mesh whose
 * node arrays (8 (N+1)^3 nelems bytes per field) or face-point arrays reach
 * 4 GiB, i.e. beyond about 500M nodes); NSKR_E_NOMEM; NSKR_E_HIP.
 * Synchronises the stream. */
int nskr_mesh_upload(nskr_ctx *ctx, const nskr_mesh *m, nskr_stream s);

/* Number of values in one state buffer: 6 nelems (N+1)^3.
 * Errors: NSKR_E_STATE before a mesh is uploaded. */
int nskr_state_size(const nskr_ctx *ctx, size_t *nvalues);

/* Bytes of library-owned device memory for the current mesh. */
int nskr_device_bytes(const nskr_ctx *ctx, size_t *bytes);

/* Write the droplet initial state into U (see nskr_init).  noise: host array
 * of nelems (N+1)^3 doubles added to rho in node order (before c = rho and
 * m = rho u), or NULL.  Errors: NSKR_E_ARG (null U or ic, ndrop < 0,
 * width <= 0, T0 not below the critical temperature when the Maxwell
 * densities are needed, densities outside (0, 1/b) or rho_l <= rho_v). */
int nskr_init_droplets(nskr_ctx *ctx, const nskr_init *ic, const double *noise, void *U, nskr_stream s);

/* Simulation time of the context: the time at which nskr_rhs, nskr_lift1
 * and nskr_lift2 evaluate walls whose temperature changes in time
 * (nskr_bc.twall_rate); nskr_rk_steps evaluates stage s of step n at t + n dt
 * + c_s dt (the stage times of the RK scheme) and advances t by nsteps dt;
 * a batch does the same for each of its instances (nskr_batch_admit).
 * Starts at 0.  Errors: NSKR_E_ARG (null ctx or output, non-finite t). */
int nskr_set_time(nskr_ctx *ctx, double t);
int nskr_get_time(const nskr_ctx *ctx, double *t);

/* U_t = L(U), the semi-discrete operator (Sec. 3.1).  Asynchronous.
 * Errors: NSKR_E_STATE, NSKR_E_ARG (null or aliasing buffers), NSKR_E_HIP. */
int nskr_rhs(nskr_ctx *ctx, const void *U, void *Ut, nskr_stream s);

/* Sub-operators for verification.  nskr_lift1 writes the BR1 gradients of
 * (rho, u, v, w, c): q[15][nelems (N+1)^3], field 3k+m = d w_k / d x_m.
 * nskr_lift2 writes out[5][...] = temperature, its lifted gradient (3) and
 * the divergence lifting of grad c (lap c).  Same element type as U. */
int nskr_lift1(nskr_ctx *ctx, const void *U, void *q, nskr_stream s);
int nskr_lift2(nskr_ctx *ctx, const void *U, void *out, nskr_stream s);

/* Stable time step (FP64) of the explicit scheme.  The paper fixes only the
 * CFL number 0.9 (Sec. 4, preamble) for its low-storage RK4 (Sec. 3.1); the
 * rule is the reading of that statement: the min of the advective limit
 * CFL T_N 2 / max_nodes sum_d (|u . Ja^d| + c~ |Ja^d|)/J (the Rusanov wave
 * speed of Sec. 3.1 with c~ = sqrt(|c_s^2|), eq. speedofsound) and the
 * parabolic/source limit CFL 4.6567 / (alpha beta + RHO_N nu_max max_nodes
 * sum_d (|Ja^d|/(2J))^2) (the relaxation source rate alpha beta and the
 * diffusivities of F^V, Sec. 2.3.2), nu_max = max(4 mu/(3 rho), kappa/(rho R
 * cv), gam beta); T_N and RHO_N are the 1D upwind-advection and BR1-diffusion
 * stability constants of the Gauss DGSEM under the RK scheme's stability
 * polynomial, 4.6567 its real stability interval.  A mesh with generalized
 * Navier-slip walls of gamma_1 > 0 (eq. bc_navierstokes_alpha,
 * eq. bc_contactangle_alpha) adds the wall limit CFL 3.3407 / max_nodes W
 * over the nodes of elements with such a face: per face of direction n,
 * W = SIGMA_N (Lambda a gamma_1 sum_d |grad c . Ja^d|/(J rho)
 * + sqrt(alpha beta gamma_1 Lambda a sum_d (|Ja^d|/J)^2)), d the two other
 * directions, a = |Ja^n|/J, Lambda = (N+1)^2/2, grad c the lifted gradient
 * and SIGMA_N the spectral radius of the lifted first derivative; the
 * traction gamma_1 div u grad_G c and the c-flux beta gamma_1 div u give
 * eigenvalues near the imaginary axis, whose stability interval under the
 * RK scheme is 3.3407.  Synchronises s.
 * Errors: NSKR_E_NONFINITE if a rate is not finite (dt not written). */
int nskr_dt(nskr_ctx *ctx, const void *U, double *dt, nskr_stream s);

/* nskr_dt for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same time step, bit for bit, with the reduction's partial maxima and
 * results in a static device array of 4 MiB instead of the context's
 * memory.  It calls no allocating routine; the traces and lifted gradients
 * it evaluates are the context's own, allocated at mesh upload.  Limit: a
 * mesh of at most 131072 element tiles of the 256-thread reduction kernel
 * (tiles = nelems / floor(256 / (N+1)^3), rounded up; the 32^3 N = 5 mesh
 * has 32768), else NSKR_E_ARG with nothing enqueued.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other host
 * threads, other streams) race and must be serialised by the caller.
 * Synchronises s.  Errors as nskr_dt; NSKR_E_STATE if the array's address
 * could not be set up on the context's device. */
int nskr_dt_noalloc(nskr_ctx *ctx, const void *U, double *dt, nskr_stream s);

/* nsteps steps of the 5-stage 2N-storage RK4(3)5 of Carpenter & Kennedy
 * (the low-storage fourth-order scheme family cited in Sec. 3.1): per stage
 * R <- A_s R + dt L(U) (assigned at stage 1, so R needs no initialisation),
 * U <- U + B_s R.  R is the scheme's scratch register: its content after
 * the call is unspecified (the last stage of a step does not store it, as
 * the next stage to read it assigns it).  Asynchronous.  Errors: NSKR_E_ARG
 * (dt not positive and finite, nsteps < 0, null or aliasing buffers),
 * NSKR_E_STATE, NSKR_E_HIP. */
int nskr_rk_steps(nskr_ctx *ctx, void *U, void *R, double dt, int nsteps, nskr_stream s);

/* Integrals and counters (the NSKR_SUM_* indices) into out[NSKR_NSUMS]:
 * the quantities the paper follows over time (Sec. 4.1.1: the relaxation
 * and gradient energies and L2(rho - c); Sec. 4.2-4.3: kinetic energy,
 * total energy, the mathematical entropy from the Helmholtz energy of
 * Sec. 2.1), plus mass, momentum, volume, extrema of rho and T and health
 * counters (non-finite values, rho outside (0, 1/b) where the van der Waals
 * pressure is defined, T <= 0, c_s^2 < 0 inside the spinodal, Sec. 2.3.1).
 * Gauss quadrature with the Jacobian, FP64 accumulation in a fixed order.
 * Synchronises s.  Returns NSKR_E_NONFINITE (out still filled) when a
 * non-finite value, rho outside (0, 1/b) or T <= 0 is found. */
int nskr_reduce(nskr_ctx *ctx, const void *U, double *out, nskr_stream s);

/* Per-kernel timing with HIP events recorded on the caller's stream around
 * every kernel launch of this context (off by default).  Kernel kinds:
 * 0 prolong, 1 lift1, 2 lift2, 3 update, 4 reductions/init.  nskr_profile
 * synchronises s, then writes the accumulated milliseconds and launch counts
 * of each kind (arrays of length NSKR_NKINDS) and resets them. */
#define NSKR_NKINDS 5
int nskr_set_profiling(nskr_ctx *ctx, int on);
int nskr_profile(nskr_ctx *ctx, double *ms, long *count, nskr_stream s);

/* Threads per workgroup of the stage kernels: 256, 512, or the degree's
 * tight size that packs whole elements into waves (N = 2: 192, N = 3 and 4:
 * 128, N = 5: 448); a block must hold at least one element.  Default: 128 at
 * N = 3, 256 otherwise.  This is the tile
 * shape (elements per workgroup) the autotuner chooses.  Results do not
 * depend on it (every element's arithmetic is the same in any tile).  A mesh
 * with curved elements runs 256 threads (its upload sets 256).
 * Errors: NSKR_E_ARG for other values; NSKR_E_UNSUPPORTED for another size on
 * a mesh with curved elements or where the kernels exceed the LDS per
 * workgroup. */
int nskr_set_block(nskr_ctx *ctx, int threads);
int nskr_get_block(const nskr_ctx *ctx, int *threads);

/* Message of the last failing call on this context (static storage valid
 * until the next call); a generic message for ctx == NULL. */
const char *nskr_last_error(const nskr_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batched execution of many independent instances (contexts), possibly with
 * different degrees, meshes, parameters, precisions and time steps.  Each
 * nskr_batch_step advances every active instance by one RK step: per group of
 * equal (degree, precision, block size) one launch per stage kernel covers all
 * member instances through a device table of instances and a block map, and
 * the whole step is captured once into a HIP graph and replayed until the set
 * of instances changes.  An instance's arithmetic is the same alone and in any
 * mix, so its results are bitwise identical.
 * ------------------------------------------------------------------------- */
typedef struct nskr_batch nskr_batch;

/* Batch on device `device` that admits instances while the sum of their
 * library memory and two state buffers stays within budget_bytes. */
int nskr_batch_create(int device, size_t budget_bytes, nskr_batch **out);
int nskr_batch_destroy(nskr_batch *b);

/* Capture steps into a HIP graph (default on).  Graph capture needs a stream
 * other than the legacy default stream. */
int nskr_batch_set_graph(nskr_batch *b, int on);

/* Admit ctx (mesh uploaded) with caller-owned state U and register R (borrowed
 * until retired), its time step dt and the number of steps to run.  The
 * instance starts from the context time t at admission: stage s of its step n
 * is evaluated at t + n dt + c_s dt, as nskr_rk_steps evaluates it, through a
 * device step counter of the context that the replayed steps advance; the
 * context time becomes t + nsteps dt when the instance finishes, or t + k dt
 * when it is retired after k steps.  Returns NSKR_E_NOMEM when the budget has
 * no room now (not fatal: retry after a retirement); NSKR_E_ARG for bad
 * arguments, an instance already admitted, or walls whose temperature would
 * leave [0.3, 0.99] during the admitted steps. */
int nskr_batch_admit(nskr_batch *b, nskr_ctx *ctx, void *U, void *R, double dt, int nsteps, int *slot);

/* One RK step of every active instance on stream s (asynchronous).  Instances
 * that reach their step count stop advancing (nskr_batch_poll reports them
 * once that step has run).  The first step after an instance is admitted also
 * clears its FP32 compensation and prolongs its state to its faces (direct
 * launches on s before the graph); later steps take the face traces the
 * previous step's last stage wrote, exactly as nskr_rk_steps does. */
int nskr_batch_step(nskr_batch *b, nskr_stream s);

/* Finished slots (up to cap written to slots, total count in *n): instances
 * whose last step has completed on the GPU (an event recorded after that
 * step), so their state can be read once the caller's stream is ordered
 * after it.  Does not block. */
int nskr_batch_poll(nskr_batch *b, int *slots, int cap, int *n);

/* Release a slot (finished or not).  Waits until every step queued so far
 * has completed, so that on return the slot's buffers are the caller's
 * again and its context may be admitted anew. */
int nskr_batch_retire(nskr_batch *b, int slot);

/* Budget in use, active instances, steps taken. */
int nskr_batch_info(const nskr_batch *b, size_t *used_bytes, int *active, long *steps);

const char *nskr_batch_last_error(const nskr_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* NSKR_H */
