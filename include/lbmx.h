/*
 * lbmx.h -- C-ABI of the MI355X double-MRT lattice Boltzmann library for
 * natural convection in a differentially heated cubic cavity
 * (Li, Yang & Zhang, arXiv:1511.04633).
 *
 * Problem (Sec. 2, Eqs. 1-10): a cube of edge H = n lattice cells, walls at
 * y = 0 (hot, theta_hot) and y = H (cold, theta_cold), no-slip everywhere
 * (Eq. 8); the four other walls are adiabatic (Type 1), carry the linear
 * profile theta_h + (theta_c - theta_h) y/H (Type 2, Eq. 9), or carry it on
 * x = 0, H and are adiabatic on z = 0, H (Type 3, Eq. 10).  Gravity points
 * along -z.
 *
 * Method (Sec. 3): D3Q19-MRT flow (Eqs. 11-26) with the Boussinesq force of
 * Eqs. (15)-(17), coupled to a D3Q7-MRT energy lattice (Eqs. 27-37);
 * parameters in lattice units from Ma, Pr, Ra (Sec. 4, Eq. 38).
 *
 * Conventions for every call:
 *   - Status codes only; no exception or abort crosses this boundary.  On a
 *     failure lbmx_last_error() returns a thread-local message.
 *   - Host arrays are caller-owned and hold n^3 values, x fastest:
 *     index = x + n*(y + n*z).  Population arrays are population-major:
 *     f[i*n^3 + index], i in the paper's order (Eqs. 12, 28), 0-based.
 *   - Device work is enqueued on the cavity's HIP stream; calls that return
 *     host data synchronise that stream before returning.
 *   - A cavity handle may be used by one host thread at a time.
 *   - Time: a fresh or re-initialised cavity is at t = 0; lbmx_step advances
 *     t.  Every read returns the state at the current t (pre-collision
 *     populations, i.e. after streaming and wall conditions).
 *   - Device memory: a cavity holds two lattices (the current state and
 *     the one the next step writes) and a small reduction scratch, all in
 *     its workspace.  Between steps the second lattice is spare, and the
 *     transfers and readbacks stage their data in it, so no call on a
 *     cavity after lbmx_create allocates device memory (lbmx_save and
 *     lbmx_load use a pinned host buffer of up to 64 MB).
 *   - Failed cavities: a cavity fails when a Nu evaluation finds non-finite
 *     values (LBMX_EUNSTABLE: the run diverged) or when a device call fails
 *     while its state is being changed.  Until an initialisation succeeds
 *     (lbmx_init_rest, lbmx_set_populations, lbmx_load, lbmx_init_fields,
 *     lbmx_init_from_cavity with it as the destination), lbmx_step,
 *     lbmx_step_timed, lbmx_run_to_steady, lbmx_save and
 *     lbmx_init_from_cavity with it as the source return LBMX_ESTATE; the
 *     reads (lbmx_read_macro, lbmx_get_populations, lbmx_nusselt,
 *     lbmx_time) still work, to inspect what went wrong.
 */
#ifndef LBMX_H
#define LBMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBMX_OK = 0,
    LBMX_EINVAL = 1,         /* invalid argument or parameter set            */
    LBMX_ENOMEM = 2,         /* device or host allocation failed             */
    LBMX_EDEVICE = 3,        /* a HIP runtime call failed                    */
    LBMX_EUNSTABLE = 4,      /* non-finite values found (run diverged)       */
    LBMX_ENOTCONVERGED = 5,  /* run_to_steady hit max_steps                  */
    LBMX_ESTATE = 6,         /* call not valid in the handle's current state */
    LBMX_EIO = 7,            /* a checkpoint file could not be read/written  */
    LBMX_STATUS_RANGE_ = 0x7fffffff  /* not a status: makes every non-negative  */
                                     /* 32-bit value a valid lbmx_status, so    */
                                     /* lbmx_strerror accepts any code          */
} lbmx_status;

/* Population storage in HBM.  Collision arithmetic is FP64 for LBMX_F64 and
 * FP32 otherwise.  D3Q19 (flow) populations are stored as offsets f_i - w_i
 * from the lattice weights (Eq. 18), D3Q7 (energy) populations as g_i; in a
 * 16-bit format a population is stored divided by its weight (1/w_i, 1/w_T,i).
 * The mixed formats keep the flow lattice in 16 bits and the energy lattice
 * in FP32, or (LBMX_F16_I16) the energy populations as g_i / (w_T,i Theta) in
 * signed 16-bit fixed point with 15 fraction bits (range +-1, saturating; the
 * code -32768 stands for NaN; Theta = the power of two at or above
 * 2 max(|theta_hot|, |theta_cold|), 1 for walls at +-1/2), rounded
 * stochastically by the step (a deterministic counter-based stream of node
 * and step, 16 random bits per population), so that increments below one
 * spacing are kept on average.  Bytes moved per node update: 416, 208, 104,
 * 104, 132, 132, 104. */
typedef enum {
    LBMX_F64 = 0,       /* flow FP64, energy FP64                      */
    LBMX_F32 = 1,       /* flow FP32, energy FP32                      */
    LBMX_F16 = 2,       /* flow FP16, energy FP16                      */
    LBMX_BF16 = 3,      /* flow BF16, energy BF16                      */
    LBMX_F16_F32 = 4,   /* flow FP16, energy FP32                      */
    LBMX_BF16_F32 = 5,  /* flow BF16, energy FP32                      */
    LBMX_F16_I16 = 6    /* flow FP16, energy 16-bit fixed point        */
} lbmx_storage;

typedef struct {
    int32_t n;              /* cells per edge, H = n; 4 <= n <= 1024              */
    int32_t wall_type;      /* 1, 2 or 3 (Sec. 2, Eqs. 6-10)                      */
    double ra;              /* Rayleigh number, > 0 (Eq. 38)                      */
    double pr;              /* Prandtl number, > 0 (paper: 0.71)                  */
    double ma;              /* Mach number u_c / c_s, in (0, 0.5] (paper: 0.1)    */
    double theta_hot;       /* wall value at y = 0, Eq. (6)  (+0.5)               */
    double theta_cold;      /* wall value at y = H, Eq. (7)  (-0.5)               */
    double theta_ref;       /* T_l of Eq. (16) (0.0, the mean of the two walls)   */
    double buoyancy_scale;  /* multiplies g beta; 1.0 normally, 0.0 = no force    */
    int32_t storage;        /* lbmx_storage                                       */
    int32_t custom_rates;   /* 0: rates of Eq. (26) and Sec. 3.2; 1: use s, tau   */
    double s[19];           /* diagonal of S (Eq. 23) when custom_rates = 1       */
    double tau[7];          /* diagonal of Q^-1 (Eq. 35) when custom_rates = 1    */
    int32_t force_model;    /* buoyancy term, LBMX_FORCE_* (0 = Eq. 15)           */
    int32_t nu_stencil;     /* hot-wall gradient for Nu, LBMX_NU_* (0 = default)  */
    double aniso[6];        /* A_xx, A_yy, A_zz, A_xy, A_xz, A_yz: diffusion      */
                            /* tensor D = alpha A of Eq. (27), entering Q^-1 by   */
                            /* Eq. (36); all zero = isotropic D = alpha I         */
} lbmx_params;

/* Force models: how the buoyancy G = g beta (theta - theta_ref) e_z of
 * Eq. (16) enters the flow lattice.
 *   LBMX_FORCE_EQ15: Eq. (15) with the density carried by f^eq of Eq. (17),
 *     F_i = 3 G.(e_i - V) f^eq_i, added after the collision (Eq. 14); the
 *     momentum gain per step is rho G.
 *   LBMX_FORCE_EQ15_RHO: the other reading of Eq. (15), divided by rho
 *     (momentum gain G).
 *   LBMX_FORCE_GUO: Guo's forcing in moment space: V = (j + rho G / 2) / rho
 *     in the flow and energy equilibria and in lbmx_read_macro, and
 *     M^-1 (I - S/2) M Fbar added, Fbar_i = w_i rho [3 (e_i - V) + 9 (e_i.V) e_i].G. */
enum { LBMX_FORCE_EQ15 = 0, LBMX_FORCE_EQ15_RHO = 1, LBMX_FORCE_GUO = 2 };

/* Nu stencils for the temperature gradient at the hot wall (Eq. 39); all
 * assume theta_hot - theta_cold = 1 as in Eq. (38).
 *   LBMX_NU_SECOND_ORDER: (9 theta_0 - theta_1 - 8 theta_hot)/3, exact for
 *     quadratic profiles (wall value and the first two nodes);
 *   LBMX_NU_FIRST_ORDER: 2 (theta_0 - theta_hot);
 *   LBMX_NU_WALL_FLUX: the energy crossing the hot wall's D3Q7 links in the
 *     last streaming, q = g_in - g*_out = 2 (g_+y - theta_hot / 8) at the
 *     wall node, as a gradient q / D_yy. */
enum { LBMX_NU_SECOND_ORDER = 0, LBMX_NU_FIRST_ORDER = 1, LBMX_NU_WALL_FLUX = 2 };

typedef struct {
    double nu3d;            /* Eq. (40): mean local Nu over the hot wall        */
    double nu2d;            /* Eq. (41): mean over the X = 0.5 line             */
    double numax;           /* maximum local Nu on the hot wall                 */
    int64_t step;           /* time t the values belong to                      */
    int32_t nonfinite;      /* count of non-finite local values (0 if healthy)  */
} lbmx_nu;

typedef struct lbmx_cavity lbmx_cavity;

/* Fill *p with the defaults: n = 16, Type 1, Ra = 1e3, Pr = 0.71, Ma = 0.1,
 * theta_hot = 0.5, theta_cold = -0.5, theta_ref = 0, buoyancy 1, LBMX_F32,
 * force model Eq. (15), second-order Nu stencil, isotropic diffusion. */
lbmx_status lbmx_params_default(lbmx_params *p);

/* Lattice-unit parameters (Sec. 4, Eq. 38; Eqs. 26, 36):
 * out[6] = {u_c = Ma c_s, g beta (per unit theta), nu, alpha = nu/Pr,
 *           s_nu = 1/(3 nu + 1/2), tau_T = 1/2 + alpha/epsilon (epsilon 1/4)}.
 * EINVAL if the set is invalid (including s_nu outside (0, 2) or tau_T <= 1/2,
 * an unknown force model or stencil, an aniso tensor that is not positive
 * definite, or aniso together with custom_rates). */
lbmx_status lbmx_derive(const lbmx_params *p, double *out);

/* Device bytes a cavity needs (two lattices plus reduction scratch). */
lbmx_status lbmx_workspace_bytes(const lbmx_params *p, size_t *bytes);

/* Algorithmic HBM bytes moved by one cell update of lbmx_step:
 * 26 populations read once and written once at their storage widths. */
lbmx_status lbmx_bytes_per_cell(int32_t storage, double *bytes);

/* Create a cavity.  dev_workspace: device memory of at least
 * lbmx_workspace_bytes() bytes, 256-byte aligned, borrowed for the handle's
 * life; NULL makes the library allocate (and free) its own.  stream: a
 * hipStream_t for all device work; NULL uses a stream the library creates.
 * The cavity starts at rest with theta = 0 (as lbmx_init_rest(h, NULL)). */
lbmx_status lbmx_create(const lbmx_params *p, void *dev_workspace, size_t ws_bytes,
                        void *stream, lbmx_cavity **out);

/* Destroy a cavity (NULL-safe).  Waits for its pending work. */
void lbmx_destroy(lbmx_cavity *h);

/* Set the state at t = 0 to fluid at rest, rho = 1: f_i = w_i, and
 * g_i = w_T,i theta0 (host array of n^3 doubles; NULL = theta 0 everywhere). */
lbmx_status lbmx_init_rest(lbmx_cavity *h, const double *theta0_host);

/* Set the state at time t from host populations: f (19 n^3) and g (7 n^3)
 * doubles, population-major (as returned by lbmx_get_populations).  Staged
 * in the spare lattice by opposite-direction pairs. */
lbmx_status lbmx_set_populations(lbmx_cavity *h, const double *f_host, const double *g_host,
                                 int64_t t);

/* Copy the populations of the current state to host (19 n^3 and 7 n^3
 * doubles; either pointer may be NULL), in passes of as many populations as
 * the spare lattice holds (1 pass FP64, 2 FP32, up to 5 for 16-bit). */
lbmx_status lbmx_get_populations(lbmx_cavity *h, double *f_host, double *g_host);

/* Checkpoints, for callers that resume long runs (the paper's runs to a
 * steady state take up to ~10^6 steps).  lbmx_save writes the cavity's
 * parameter set, its time t and its current lattice (the post-collision
 * populations of t - 1, in the storage format, bit for bit) to `path`;
 * lbmx_load reads such a file into a cavity created with the same parameter
 * set (the custom s, tau arrays are compared only when custom_rates = 1, the
 * Nu stencil not at all: it only reads the state), so
 * that stepping on continues bitwise as the saved cavity would.  lbmx_load
 * reads the lattice into the cavity's spare lattice and switches to it only
 * after the last byte has arrived, so a load that fails leaves the state as
 * it was (a successful load also clears a failed state).  The file is
 * a 376-byte header (magic "LBMXCKPT", version 1, sizeof(lbmx_params), the
 * parameters, t, lattice bytes, nodes per slab; host byte order) followed by
 * the lattice; it is tied to this library's lattice layout and is not meant
 * to be portable across versions.  Both calls synchronise the stream.
 * Errors: EIO when the file cannot be opened, written or read in full;
 * EINVAL when it is not a checkpoint, has another version, size, layout or
 * parameter set (checked before the cavity's state is touched). */
lbmx_status lbmx_save(lbmx_cavity *h, const char *path);
lbmx_status lbmx_load(lbmx_cavity *h, const char *path);

/* Set the state at t = 0 from velocity and temperature fields given on a
 * src_n^3 grid of node-centred device FP32 arrays (x fastest): each cavity
 * node samples them trilinearly (clamped at the walls) and takes
 * f = f^eq(rho = 1, u) of Eq. (17) and g = g^eq(theta, u) with
 * N g^eq = n^eq of Eq. (33).  Velocities in lattice units. */
lbmx_status lbmx_init_fields(lbmx_cavity *h, const float *dev_u, const float *dev_v,
                             const float *dev_w, const float *dev_theta, int32_t src_n);

/* Set dst's state at t = 0 from the current state of another cavity src of
 * any size, storage or parameter set (grid sequencing: a coarse cavity's
 * steady state as the start of a finer one; the paper fixes no initial
 * state).  src's fields rho, u = j / rho, theta (Eqs. 20, 25, 30; the
 * half-force velocity under Guo's forcing) are formed on the device in
 * FP64 and sampled trilinearly onto dst's nodes as in lbmx_init_fields;
 * with s = u_c(dst) / u_c(src) (Eq. 38: 1 unless Ma differs) dst takes
 * f = f^eq(rho', s u) of Eq. (17), rho' = 1 + s^2 (rho - 1) (the density
 * variations are pressure, of order u_c^2), and g = g^eq(theta, s u).  src
 * is only read; its fields (5 src_n^3 doubles) are staged in src's spare
 * lattice.  Both cavities must live on the current device.  Synchronises
 * both streams.  Errors: EINVAL for a NULL or identical handle or another
 * device, ESTATE for a failed src, EDEVICE for a HIP failure. */
lbmx_status lbmx_init_from_cavity(lbmx_cavity *dst, lbmx_cavity *src);

/* Set dst's state at t = 0 from the weighted sum of two other cavities'
 * fields (grid sequencing with extrapolation; the paper fixes no initial
 * state): u = wa s_a u_a + wb s_b u_b, theta = wa theta_a + wb theta_b
 * and rho = 1 + wa s_a^2 (rho_a - 1) + wb s_b^2 (rho_b - 1), where rho_k,
 * u_k = j / rho_k and theta_k (Eqs. 20, 25, 30) of cavity k are formed on
 * the device in FP64 and sampled trilinearly onto dst's nodes as in
 * lbmx_init_fields, and s_k = u_c(dst) / u_c(k) (Eq. 38); dst takes
 * f = f^eq(rho, u) of Eq. (17) and g = g^eq(theta, u).  With a and b the
 * steady states of the same case at 1/2 and 1/4 of dst's resolution, the
 * weights wa = 5/4, wb = -1/4 extrapolate their second-order grid error
 * to dst's grid.  a and b are only read; each stages its fields (5 n^3
 * doubles) in its own spare lattice.  All three cavities must live on the
 * current device.  Synchronises the three streams.  Errors: EINVAL for a
 * NULL handle, two identical handles, another device or a non-finite
 * weight, ESTATE for a failed source, EDEVICE for a HIP failure. */
lbmx_status lbmx_init_from_cavities(lbmx_cavity *dst, lbmx_cavity *a, double wa, lbmx_cavity *b,
                                    double wb);

/* Advance nsteps >= 0 time steps (fused streaming + double-MRT collision,
 * Eqs. 14 and 29, wall conditions of Eqs. 6-10).  Asynchronous. */
lbmx_status lbmx_step(lbmx_cavity *h, int64_t nsteps);

/* As lbmx_step, and also report the elapsed device time of the nsteps
 * kernels measured with HIP events on the cavity's stream (synchronises). */
lbmx_status lbmx_step_timed(lbmx_cavity *h, int64_t nsteps, double *ms);

/* Current time step t. */
lbmx_status lbmx_time(const lbmx_cavity *h, int64_t *t);

/* Macroscopic fields at the current t to host arrays (n^3 doubles each,
 * any may be NULL): rho = sum f (Eq. 20), u = j / rho with j = sum e_i f_i,
 * theta = sum g (Eq. 30).  Staged in the spare lattice. */
lbmx_status lbmx_read_macro(lbmx_cavity *h, double *rho, double *ux, double *uy, double *uz,
                            double *theta);

/* Hot-wall Nusselt numbers at the current t (Eqs. 39-41): local
 * Nu = -n (9 theta_0 - theta_1 - 8 theta_hot)/3 from the two wall-adjacent
 * nodes (second order, exact for quadratic profiles); map_host (n*n doubles,
 * x fastest then z) may be NULL.  Returns EUNSTABLE (with *out filled) if any
 * local value is not finite, and the cavity is then failed (see above). */
lbmx_status lbmx_nusselt(lbmx_cavity *h, lbmx_nu *out, double *map_host);

/* For callers that cannot allocate device memory, for instance code that
 * runs between captured graph launches or a serving loop with a fixed
 * memory budget: lbmx_nusselt without the cavity's workspace scratch.  The
 * reduction's partial sums and results live in a static device array of the
 * library (4 * 1024 + 8 doubles, 32.8 KB, one per GPU, held until the
 * process ends); the map (if requested) is staged in the spare lattice as
 * in lbmx_nusselt.  Allocates nothing.  The cavity must live on the current
 * device.  Calls that overlap on one GPU (two host threads, or cavities on
 * different streams with work in flight) share that array and race; calls
 * that follow each other do not interfere: every call rewrites all the
 * partial sums it reads.  Same results and errors as lbmx_nusselt, plus
 * EINVAL for n > 1024 or a cavity on another device. */
lbmx_status lbmx_nusselt_noalloc(lbmx_cavity *h, lbmx_nu *out, double *map_host);

/* Step in chunks of `every` and stop once |Nu_3D(t) - Nu_3D(t - every)| < tol
 * (the paper gives no criterion; this is the criterion the library uses).
 * ENOTCONVERGED if max_steps pass first; EUNSTABLE on divergence.  *out holds
 * the last Nu evaluation either way. */
lbmx_status lbmx_run_to_steady(lbmx_cavity *h, double tol, int64_t every, int64_t max_steps,
                               lbmx_nu *out);

/* Launch shape of the step kernel: block = (bx, by) threads over (x, y),
 * grid covers the cube.  Any bx, by >= 1 with bx*by <= 1024 gives the same
 * results (each thread finds its node and walls from its own indices);
 * shapes whose rows span whole wavefronts (bx a multiple of 64, or bx = n)
 * keep every load and store coalesced and run fastest.  EINVAL otherwise.
 * 0, 0 restores the default (bx = min(n, 256), by = min(n, max(1, 256 / bx))). */
lbmx_status lbmx_set_launch(lbmx_cavity *h, int32_t bx, int32_t by);
lbmx_status lbmx_get_launch(const lbmx_cavity *h, int32_t *bx, int32_t *by);

/* ------------------------------------------------------------------ batch
 * Many cavities (uneven n, Ra, wall type; one storage format) advanced
 * together: every time step is ONE kernel launch over a work list of
 * fixed-size node tiles drawn from all active cavities (each node update as
 * lbmx_step), replayed from a captured hipGraph of `graph_steps` launches.
 * Cavities that reach a steady Nu are retired from the work list.  All
 * active cavities share the batch's time step count since their last
 * (re)initialisation.  Device memory is allocated by the library. */
typedef struct lbmx_batch lbmx_batch;

/* Cavity states reported by lbmx_batch_info. */
enum { LBMX_ACTIVE = 0, LBMX_CONVERGED = 1, LBMX_MAXSTEPS = 2, LBMX_DIVERGED = 3 };

/* Create a batch of `count` cavities from p[0..count-1] (same storage for
 * all, 4 <= n <= 255).  Each cavity starts at rest with theta = 0.  stream
 * as in lbmx_create.  Size and parameter errors return LBMX_EINVAL before
 * any device call. */
lbmx_status lbmx_batch_create(const lbmx_params *p, int32_t count, void *stream, lbmx_batch **out);

/* Destroy a batch (NULL-safe). */
void lbmx_batch_destroy(lbmx_batch *b);

/* (Re)initialise cavity k at rest with theta0 (host, n_k^3 doubles; NULL =
 * 0), reset its step count, and make it active again. */
lbmx_status lbmx_batch_init_rest(lbmx_batch *b, int32_t k, const double *theta0_host);

/* Advance every active cavity by nsteps time steps (asynchronous). */
lbmx_status lbmx_batch_step(lbmx_batch *b, int64_t nsteps);

/* Step all active cavities in chunks of `every`; after each chunk evaluate
 * each active cavity's Nu_3D (Eq. 40) and retire it when
 * |Nu_3D(t) - Nu_3D(t - every)| < tol (LBMX_CONVERGED), when it has taken
 * max_steps steps in this call (LBMX_MAXSTEPS) or when Nu is not finite
 * (LBMX_DIVERGED).  Returns when no cavity is active; *n_converged (may be
 * NULL) counts converged cavities.  ENOTCONVERGED / EUNSTABLE if any cavity
 * ended that way. */
lbmx_status lbmx_batch_run_to_steady(lbmx_batch *b, double tol, int64_t every, int64_t max_steps,
                                     int32_t *n_converged);

/* State, step count and last Nu evaluation of cavity k (pointers may be NULL). */
lbmx_status lbmx_batch_info(const lbmx_batch *b, int32_t k, int32_t *state, int64_t *t,
                            lbmx_nu *last);

/* Nu (Eqs. 39-41) of cavity k now (synchronises). */
lbmx_status lbmx_batch_nusselt(lbmx_batch *b, int32_t k, lbmx_nu *out);

/* Cavity k starts at t = 0 from the current state of cavity ks of batch src
 * (src may be b itself, with ks != k), as lbmx_init_from_cavity does for
 * single cavities (grid sequencing: a batch of half-size cavities run to
 * steady starts the full-size batch); a retired cavity becomes active again.
 * Synchronises both batches' streams.  Errors as lbmx_init_from_cavity. */
lbmx_status lbmx_batch_init_from(lbmx_batch *b, int32_t k, lbmx_batch *src, int32_t ks);

/* Macroscopic fields of cavity k, as lbmx_read_macro (staged in cavity k's
 * spare lattice). */
lbmx_status lbmx_batch_read_macro(lbmx_batch *b, int32_t k, double *rho, double *ux, double *uy,
                                  double *uz, double *theta);

/* u, v, w (lattice units) and theta of cavity k resampled trilinearly onto
 * an out_n^3 node-centred grid of the same cube (clamped at the outermost
 * node centres): host_uvwt holds 4 out_n^3 floats, field-major, x fastest.
 * Allocates and frees device buffers of 32 n_k^3 + 16 out_n^3 bytes (a
 * dataset-export call, not part of the stepping). */
lbmx_status lbmx_batch_resample(lbmx_batch *b, int32_t k, int32_t out_n, float *host_uvwt);

/* Launch shape: `block` threads (= nodes per tile, multiple of 64, <= 1024),
 * `grid` blocks striding over the tiles (0 = one block per tile), and
 * `graph_steps` launches per captured graph (even; 0 = no graph). */
lbmx_status lbmx_batch_set_launch(lbmx_batch *b, int32_t block, int32_t grid, int32_t graph_steps);
lbmx_status lbmx_batch_get_launch(const lbmx_batch *b, int32_t *block, int32_t *grid,
                                  int32_t *graph_steps);

/* Time candidate (block, grid) shapes on the batch's current work list and
 * keep the fastest; with cache_path (a JSON file, created if missing) the
 * choice is looked up / stored under the GPU, storage, cavity count and node
 * count.  Timing advances the cavities, so every cavity is afterwards reset
 * to rest with theta = 0 at step 0: call it before initialising.
 * *us_per_step (may be NULL) receives the chosen shape's time per step. */
lbmx_status lbmx_batch_autotune(lbmx_batch *b, const char *cache_path, double *us_per_step);

/* ------------------------------------------------------------ surrogate
 * Kernels of the 3-D convolutional U-Net that maps (log10 Ra, wall type) to
 * steady u, v, w, theta and warm-starts a cavity (lbmx_init_fields).  Not a
 * step of the paper's method: it is trained on steady fields the batched
 * solver produces.  All pointers are device pointers; every call enqueues on
 * `stream` (a hipStream_t, NULL = the null stream) and returns at once.
 * Activations are channel-last BF16 [B][D][H][W][C], C a multiple of 16;
 * convolution weights BF16 [Co][27][Ci], tap = (kz*3 + ky)*3 + kx at offset
 * (kx-1, ky-1, kz-1), zero padding; biases, gradients and optimiser state
 * FP32.  Products on the matrix cores (BF16 in, FP32 accumulate). */

/* out[p][co] = bias[co] + sum_{tap,ci} w[co][tap][ci] in[p + off(tap)][ci];
 * out is BF16 (out_f32 = 0) or FP32 [B][D][H][W][Co].  bias may be NULL.
 * 16 <= Ci, Co <= 1024, multiples of 16; B D H W < 2^31 and 6 (H + 1) (W + 2)
 * Ci < 2^31 (32-bit element offsets within a few planes).  EINVAL otherwise. */
lbmx_status lbmx_nn_conv3d_fwd(const void *in, const void *w, const float *bias, void *out,
                               int32_t out_f32, int32_t B, int32_t D, int32_t H, int32_t W,
                               int32_t Ci, int32_t Co, void *stream);

/* lbmx_nn_conv3d_fwd with a BF16 output (out, [B][D][H][W][Co] unless
 * split) and fused epilogue options, each NULL / 0 when unused:
 *   act:   also write a = silu(z) (BF16, [.][Co]) beside z = the convolution
 *          plus bias in out: a forward layer without a separate SiLU pass;
 *   gate:  BF16 [.][Co] pre-activations z' of the previous layer: out gets
 *          bf16(bf16(conv) * silu'(z')) instead of the convolution, i.e. with
 *          the flipped weights of lbmx_nn_conv3d_flip, that layer's gradient
 *          dL/dz' without a separate SiLU-backward pass;
 *   out2, split: output channels c >= split go to out2 ([.][Co - split],
 *          channel c - split) and the others to out ([.][split]): the two
 *          parts of the gradient of a concatenated input.
 * act and gate exclude each other and out2; split is a multiple of 16 in
 * (0, Co).  Results equal the separate kernels' bit for bit (same roundings
 * to BF16 in the same order).  EINVAL otherwise, as lbmx_nn_conv3d_fwd. */
lbmx_status lbmx_nn_conv3d_fwd_ep(const void *in, const void *w, const float *bias, void *out,
                                  void *act, const void *gate, void *out2, int32_t split, int32_t B,
                                  int32_t D, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                                  void *stream);

/* A decoder layer's forward convolution with the upsample-and-concatenate
 * input read in place: the input is cat = [nearest x2 upsampling of low
 * [B][D/2][H/2][W/2][Cu] | skip [B][D][H][W][Cs]] (what lbmx_nn_upcat would
 * write), never materialised; w is [Co][27][Cu + Cs]; out (and act, if not
 * NULL) as lbmx_nn_conv3d_fwd_ep.  Cu, Cs multiples of 16, D H W even.
 * Equals lbmx_nn_upcat followed by lbmx_nn_conv3d_fwd_ep bit for bit.
 * EINVAL otherwise. */
lbmx_status lbmx_nn_conv3d_fwd_upcat(const void *low, const void *skip, const void *w, const float *bias,
                                     void *out, void *act, int32_t B, int32_t D, int32_t H, int32_t W,
                                     int32_t Cu, int32_t Cs, int32_t Co, void *stream);

/* cat [B][2D][2H][2W][Ch + Cs] = [nearest x2 upsampling of h [B][D][H][W][Ch]
 * | skip [B][2D][2H][2W][Cs]] in one pass (lbmx_nn_up2 then lbmx_nn_concat).
 * Ch, Cs multiples of 16. */
lbmx_status lbmx_nn_upcat(const void *h, const void *skip, void *cat, int32_t B, int32_t D, int32_t H,
                          int32_t W, int32_t Ch, int32_t Cs, void *stream);

/* Gradient through 2x2x2 average pooling with the optional extras of the
 * U-Net's encoder outputs: gin [B][D][H][W][C] (even extents) =
 * silu'(gate) * (bf16(gout[parent] / 8) + add), BF16 after each step as
 * lbmx_nn_pool2 (backward), lbmx_nn_add and lbmx_nn_silu_bwd in sequence
 * would round; add and gate may be NULL.  C a multiple of 16. */
lbmx_status lbmx_nn_pool2_bwd_gate(const void *gout, const void *add, const void *gate, void *gin,
                                   int32_t B, int32_t D, int32_t H, int32_t W, int32_t C, void *stream);

/* Gradient through nearest x2 upsampling (sum over the 8 copies of each
 * coarse voxel; gout on the 2D x 2H x 2W grid, gin on D x H x W) times the
 * optional silu'(gate), BF16 after each step.  C a multiple of 16. */
lbmx_status lbmx_nn_up2_bwd_gate(const void *gout, const void *gate, void *gin, int32_t B, int32_t D,
                                 int32_t H, int32_t W, int32_t C, void *stream);

/* wt[ci][26 - tap][co] = w[co][tap][ci]: with it, lbmx_nn_conv3d_fwd of an
 * output gradient (Co channels) gives the input gradient (Ci channels). */
lbmx_status lbmx_nn_conv3d_flip(const void *w, void *wt, int32_t Ci, int32_t Co, void *stream);

/* lbmx_nn_conv3d_flip for `count` (<= 32) layers in one launch: layer l's
 * weights [co[l]][27][ci[l]] start at element offsets[l] of w and its
 * flipped copy at the same offset of wt (offsets, ci, co: host arrays). */
lbmx_status lbmx_nn_conv3d_flip_many(const void *w, void *wt, int32_t count, const int64_t *offsets,
                                     const int32_t *ci, const int32_t *co, void *stream);

/* gw[co][tap][ci] += sum_p gout[p][co] in[p + off(tap)][ci] and, if gb is
 * not NULL, gb[co] += sum_p gout[p][co] (FP32, accumulated atomically, so
 * the summation order varies between runs).  16 <= Ci, Co <= 1024,
 * multiples of 16; B D H W max(Ci, Co) < 2^31 and 6 (H + 1) (W + 2) max(Ci,
 * Co) < 2^31.  EINVAL otherwise. */
lbmx_status lbmx_nn_conv3d_wgrad(const void *in, const void *gout, float *gw, float *gb, int32_t B,
                                 int32_t D, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                                 void *stream);

/* lbmx_nn_conv3d_wgrad of a decoder layer whose input is the concatenation
 * of lbmx_nn_conv3d_fwd_upcat (low, skip, Cu, Cs, D H W even), read in
 * place; gw is [Co][27][Cu + Cs]. */
lbmx_status lbmx_nn_conv3d_wgrad_upcat(const void *low, const void *skip, const void *gout, float *gw,
                                       float *gb, int32_t B, int32_t D, int32_t H, int32_t W, int32_t Cu,
                                       int32_t Cs, int32_t Co, void *stream);

/* a = z sigmoid(z) elementwise (n BF16 values), and its gradient
 * gz = ga sigmoid(z) (1 + z (1 - sigmoid(z))). */
lbmx_status lbmx_nn_silu(const void *z, void *a, int64_t n, void *stream);
lbmx_status lbmx_nn_silu_bwd(const void *z, const void *ga, void *gz, int64_t n, void *stream);

/* 2x2x2 average pooling of in [B][D][H][W][C] (even extents) into out;
 * backward = 1: in is the pooled gradient, out the input gradient. */
lbmx_status lbmx_nn_pool2(const void *in, void *out, int32_t B, int32_t D, int32_t H, int32_t W,
                          int32_t C, int32_t backward, void *stream);

/* Nearest-neighbour x2 upsampling of in [B][D][H][W][C] into out
 * [B][2D][2H][2W][C]; backward = 1: in is the upsampled gradient, out the
 * input gradient (sum over the 8 copies). */
lbmx_status lbmx_nn_up2(const void *in, void *out, int32_t B, int32_t D, int32_t H, int32_t W,
                        int32_t C, int32_t backward, void *stream);

/* out[p] = [a[p] | b[p]] (Ca + Cb channels, nvox voxels); backward = 1
 * splits the gradient `out` into a and b. */
lbmx_status lbmx_nn_concat(void *a, void *b, void *out, int64_t nvox, int32_t Ca, int32_t Cb,
                           int32_t backward, void *stream);

/* The network head and its loss in one pass (the convolution epilogue
 * computes the loss, and the FP32 head output is never stored unless pred
 * is not NULL): z = lbmx_nn_conv3d_fwd(in, w, bias) in FP32 registers,
 * nvox = B D H W; for channels c < K, e = z[p][c] - target[p][c] (target
 * FP32 [nvox][K]) and grad[p][c] = bf16(2 e / (nvox K)); grad[p][c] = 0 for
 * K <= c < Co (grad BF16 [nvox][Co]); partial[0 .. npartial) receives
 * per-block sums of e^2 (their sum / (nvox K) is the loss; entries past the
 * last block are zeroed); pred (FP32 [nvox][Co]) receives z if not NULL.
 * grad equals lbmx_nn_conv3d_fwd (FP32) followed by lbmx_nn_mse bit for bit;
 * the partial sums differ only in FP64 summation order.  16 <= Ci, Co <=
 * 1024, multiples of 16, 1 <= K <= Co, npartial >= Co / 16 (the grid has at
 * most npartial blocks, at least one per 16 output channels), nvox Co <
 * 2^31 and 6 (H + 1) (W + 2) Ci < 2^31.  EINVAL otherwise. */
lbmx_status lbmx_nn_conv3d_mse(const void *in, const void *w, const float *bias, const float *target,
                               int32_t K, void *grad, double *partial, int32_t npartial, float *pred,
                               int32_t B, int32_t D, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                               void *stream);

/* Squared error of the first K of C channels of pred [nvox][C] against
 * target [nvox][K] (both FP32): grad [nvox][C] BF16 = 2 (pred - target) /
 * (nvox K) (0 for channels >= K); partial[0..npartial) receives per-block
 * sums of squared errors (their sum / (nvox K) is the loss). */
lbmx_status lbmx_nn_mse(const float *pred, const float *target, void *grad, double *partial,
                        int32_t npartial, int64_t nvox, int32_t C, int32_t K, void *stream);

/* Adam step (bias-corrected, decoupled weight decay wd) on FP32 master
 * weights w with gradient g (cleared afterwards) and moments m, v; writes
 * the BF16 copy w_bf16 (may be NULL).  step >= 1 counts updates. */
lbmx_status lbmx_nn_adam(float *w, float *g, float *m, float *v, void *w_bf16, int64_t n, float lr,
                         float b1, float b2, float eps, int64_t step, float wd, void *stream);

/* lbmx_nn_adam that also writes the flipped BF16 copies of `count` (<= 32)
 * layers, as lbmx_nn_conv3d_flip_many of w_bf16 would (bit for bit): layer
 * l's weights [co[l]][27][ci[l]] start at element offsets[l] of w, its
 * flipped copy at the same offset of w_flip; the layers ascend, do not
 * overlap and lie in [0, n); elements outside them get no flipped copy.
 * w_bf16 and w_flip are required.  EINVAL otherwise. */
lbmx_status lbmx_nn_adam_flip(float *w, float *g, float *m, float *v, void *w_bf16, void *w_flip,
                              int64_t n, float lr, float b1, float b2, float eps, int64_t step, float wd,
                              int32_t count, const int64_t *offsets, const int32_t *ci, const int32_t *co,
                              void *stream);

/* FP32 -> BF16 (round to nearest even). */
lbmx_status lbmx_nn_to_bf16(const float *a, void *b, int64_t n, void *stream);

/* Network input on an m^3 node-centred grid, BF16 [B][m][m][m][16]:
 * channel 0 = cond[2b] (normalised log10 Ra), 1..3 = one-hot of the wall
 * type cond[2b+1] in {1, 2, 3}, 4..6 = node coordinates in [-1, 1], rest 0. */
lbmx_status lbmx_nn_make_input(const float *cond, void *out, int32_t B, int32_t m, void *stream);

/* out = a + b for n BF16 values (sums of gradients of a tensor used twice). */
lbmx_status lbmx_nn_add(const void *a, const void *b, void *out, int64_t n, void *stream);

/* FP32 layout change between channel-first [B][K][V] (a) and channel-last
 * [B][V][C] (b, first K of C channels, others zero): to_channel_last = 1
 * reads a and writes b; 0 reads a as channel-last and writes b channel-first.
 * Each of the K channels is multiplied by scale[k] (device, may be NULL). */
lbmx_status lbmx_nn_layout(const float *a, float *b, int32_t B, int64_t V, int32_t K, int32_t C,
                           int32_t to_channel_last, const float *scale, void *stream);

/* lbmx_nn_layout (channel-first a [B][K][m^3] -> channel-last b [B][m^3][C])
 * on a cubic grid, transformed by a symmetry of the cavity: output voxel
 * (x, y, z) (x fastest) takes input voxel (x', y', z') with x' = m - 1 - x if
 * flip & 1, y' likewise if flip & 2, z' if flip & 4; channel k is multiplied
 * by signs[k] (host array of K floats) and scale[k] (device, may be NULL).
 * For the fields (u, v, w, theta) of the cavity (Sec. 2): flip 1 with signs
 * (-1, 1, 1, 1) is the spanwise mirror, flip 7 with (-1, -1, -1, -1) the
 * inversion about the centre (hot and cold walls exchanged, theta negated).
 * 1 <= K <= min(C, 8), 0 <= flip <= 7.  EINVAL otherwise. */
lbmx_status lbmx_nn_layout_flip(const float *a, float *b, int32_t B, int32_t m, int32_t K, int32_t C,
                                int32_t flip, const float *signs, const float *scale, void *stream);

const char *lbmx_strerror(lbmx_status s);
const char *lbmx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMX_H */
