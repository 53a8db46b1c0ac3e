/*
 * nm.h -- C ABI of the MI355X nodal finite-difference micromagnetics library.
 *
 * The library evaluates the effective field of the nodal finite-difference
 * scheme of Abert et al., "NeuralMag: an open-source nodal finite-difference
 * code for inverse micromagnetics" (Sec. 3), and advances the
 * Landau-Lifshitz-Gilbert equation (Sec. 2, Eq. llg) with RK4 or the adaptive
 * Dormand-Prince 5(4) pair (Sec. 5.3).  All compute runs in hand-written HIP
 * kernels for gfx950 in float32; float64 is used only for the demagnetisation
 * tensor set-up and for the adaptive step's error norm.
 *
 * Conventions shared by every call
 *  - Grid: N1 x N2 x N3 cells of size h1 x h2 x h3 (metres); nodes
 *    n = c + i with i in {0,1}^3 (Sec. 3.1), i.e. (N1+1)(N2+1)(N3+1) nodes.
 *  - Layout: structure of arrays, x fastest.  A nodal vector field is
 *    float[3][N3+1][N2+1][N1+1]; a cell scalar float[N3][N2][N1]; a cell
 *    vector float[3][N3][N2][N1].
 *  - Pointers named "device" must point to GPU memory of the current device.
 *    The caller owns every pointer it passes; the library owns its internal
 *    buffers (allocated in nm_mesh_create, released in nm_mesh_destroy).  No
 *    hot call (nm_heff, nm_llg_rhs, nm_llg_step) allocates.
 *  - Streams: work is enqueued on the stream given at mesh creation
 *    (hipStream_t cast to void*; NULL means the null stream).  Calls return
 *    without synchronising unless stated otherwise.
 *  - Units: SI; fields in A/m, mu0 = 4 pi 1e-7 exactly.
 *  - Errors: every call returns an nm_status; NM_OK is 0.  On error nothing
 *    has been enqueued and nm_last_error() returns a message (per thread).
 *  - Threads: a mesh must not be used by two threads at once.
 */
#ifndef NM_H
#define NM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NM_OK = 0,
    NM_EINVAL = -1,        /* bad argument (sizes, NULL pointer, unknown flag) */
    NM_ENOMEM = -2,        /* device allocation failed */
    NM_EHIP = -3,          /* a HIP runtime call failed */
    NM_ENOTREADY = -4,     /* result not available yet */
    NM_ENONFINITE = -5,    /* the state or the step error became NaN/Inf */
    NM_ESTEPSIZE = -6,     /* adaptive step fell below dt_min */
    NM_EBUDGET = -7,       /* a solve can never fit in the server's memory budget */
    NM_EUNSUPPORTED = -8   /* valid request the library does not handle */
} nm_status;

/* Energy / field terms (bit mask). */
enum {
    NM_T_EXCHANGE = 1,     /* int A |grad m|^2, Eq. exchange_energy */
    NM_T_DEMAG = 2,        /* cuboid-cell FFT demagnetisation, Sec. 3.2 */
    NM_T_ANIS = 4,         /* uniaxial -int Ku (m.e)^2 */
    NM_T_ZEEMAN = 8,       /* -mu0 int Ms m.H_ext */
    NM_T_DMI = 16,         /* antisymmetric exchange (Sec. 2), of the kind
                            * nm_material.dmi_type names: interfacial
                            * (normal z) int D [m_z div m - (m.grad) m_z], or
                            * bulk int D m . curl m */
    NM_T_CUBIC = 32,       /* cubic anisotropy int Kc (a1^2 a2^2 + a2^2 a3^2 +
                            * a3^2 a1^2), a_i = m . c_i, by the 2-point Gauss
                            * rule per axis (Sec. 5.1's quadrature of the
                            * integrand) */
    NM_T_ALL = 63
};

/* Kinds of antisymmetric exchange (nm_material.dmi_type). */
enum { NM_DMI_INTERFACIAL = 0, NM_DMI_BULK = 1 };

/* Time integrators (Sec. 5.3). */
enum { NM_RK4 = 1, NM_DP45 = 2 };

typedef struct nm_mesh nm_mesh;

/* Nodal bases (Sec. 3.1 and Sec. 3.3, low-dimensional geometries). */
enum {
    NM_BASIS_3D = 0,   /* trilinear functions: (N1+1)(N2+1)(N3+1) nodes */
    NM_BASIS_FILM = 1  /* bilinear in-plane functions constant along z, the weak
                        * form still integrated over the full cells: one cell
                        * layer (N3 = 1) and (N1+1)(N2+1) nodes, every nodal
                        * array laid out as [3][1][N2+1][N1+1] */
};

/* Optional device-memory hooks: when alloc is set, every device buffer of
 * the mesh (its state, stage and FFT workspaces, the k-space tensor and the
 * tensor set-up's float64 temporaries) comes from alloc(bytes, ctx) and goes
 * back through free(ptr, ctx) when the mesh is destroyed (the temporaries at
 * the end of nm_demag_tensor_init), so that a framework's caching allocator
 * (torch's, for instance) owns the memory.  The memory is used on the mesh's
 * stream only; alloc returns NULL on failure (nm_mesh_create then fails with
 * NM_ENOMEM) and must return 256-byte aligned pointers.  Both are called from
 * the thread that calls nm_mesh_create / nm_demag_tensor_init /
 * nm_mesh_destroy.  A zero-initialised struct selects the library's own
 * allocation. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} nm_allocator;

/* Grid and constants.  n[k] >= 2 for k = 0, 1 and n[2] >= 1 (= 1 for the
 * film basis); every padded FFT length (next power of two >= 2 n[k] - 1)
 * must not exceed 1024.  A zero-initialised descriptor selects the 3D
 * basis and the library's own allocation. */
typedef struct {
    int n[3];          /* cells N1, N2, N3 */
    double h[3];       /* cell edges (m), > 0 */
    double gamma;      /* reduced gyromagnetic ratio, m/(A s), > 0 */
    void *stream;      /* hipStream_t for all work on this mesh */
    int basis;         /* NM_BASIS_3D or NM_BASIS_FILM */
    nm_allocator alloc; /* optional device-memory hooks (see above) */
} nm_mesh_desc;

/* Cell-wise material parameters (Eqs. ms_discrete, cell_basis) and applied
 * field; all pointers are device pointers to float cell arrays, copied by
 * nm_mesh_create (the caller may free them afterwards).
 *   H_ext,c(t) = h_uniform + h_cell[c] + drive_mask[c] drive_amp sin(2 pi f t + phase) */
typedef struct {
    const float *Ms;          /* required, A/m, >= 0 (0 marks vacuum cells) */
    const float *A;           /* required, J/m */
    const float *alpha;       /* required, Gilbert damping */
    const float *Ku;          /* optional, J/m^3 (uniaxial); with easy */
    const float *easy;        /* optional, 3*N unit easy axes; with Ku */
    const float *h_cell;      /* optional, 3*N per-cell applied field */
    float h_uniform[3];       /* uniform applied field */
    const float *drive_mask;  /* optional, per-cell weight of the drive */
    float drive_amp[3];       /* drive amplitude (A/m) */
    double drive_freq;        /* Hz */
    double drive_phase;       /* rad */
    const float *D;           /* optional, J/m^2, DMI constant */
    int dmi_type;             /* NM_DMI_INTERFACIAL (0) or NM_DMI_BULK */
    const float *Kc;          /* optional, J/m^3, cubic anisotropy constant; with cubic */
    const float *cubic;       /* optional, 6*N: cubic axes c1 (3*N) then c2 (3*N),
                               * orthonormal per cell; c3 = c1 x c2; with Kc */
} nm_material;

/* Adaptive / fixed stepping parameters. */
typedef struct {
    int method;            /* NM_RK4 or NM_DP45 */
    unsigned terms;        /* field terms, NM_T_* mask */
    double rtol, atol;     /* DP45 tolerances (RMS norm, float64) */
    double dt_min, dt_max; /* DP45 bounds on the step (dt_max <= 0: none) */
    double stop_torque;    /* > 0: DP45 stops once max_n |dm/dt| < stop_torque (1/s) */
    double *log;           /* optional device buffer, 3 doubles (t, dt, accepted)
                              per DP45 attempt */
    long log_capacity;     /* attempts that fit in log */
} nm_integrator;

/* Integrator clock, read and written by nm_llg_step. */
typedef struct {
    double t;              /* current time (s) */
    double dt;             /* RK4: the step; DP45: the next step proposal */
    long accepted, rejected, rhs_evals;
    double max_torque;     /* DP45: max_n |dm/dt| after the last accepted step */
} nm_clock;

/* Create a mesh: validates desc and mat, allocates every internal buffer
 * (FFT workspace, tensor, per-node coefficients) and computes the lumped
 * mass M_n = mu0 sum_{c containing n} Ms_c V/8 (Eq. mass_lumping) and the
 * nodal damping.  Synchronises the stream before returning. */
nm_status nm_mesh_create(const nm_mesh_desc *desc, const nm_material *mat, nm_mesh **out);

/* Release a mesh and all its buffers (synchronises its stream).  NULL is ignored. */
nm_status nm_mesh_destroy(nm_mesh *mesh);

/* Sizes: nodes, cells and the padded FFT grid (any output may be NULL). */
nm_status nm_mesh_info(const nm_mesh *mesh, int64_t *n_nodes, int64_t *n_cells, int pad[3]);

/* Device bytes nm_mesh_create would allocate for this grid. */
size_t nm_mesh_footprint_bytes(const nm_mesh_desc *desc, int integrator);

/* Replace the per-cell applied-field map (device, 3*N floats; NULL clears it). */
nm_status nm_mesh_set_field(nm_mesh *mesh, const float *h_cell);

/* Demagnetisation tensor (Sec. 3.2): float64 Newell closed form near the
 * source cell, tent-weighted Gauss-Legendre integral of the dipole kernel
 * further out, transformed in float64 to the real k-space tensor of the
 * zero-padded grid and stored in float32.  Idempotent; must precede any call
 * with NM_T_DEMAG. */
nm_status nm_demag_tensor_init(nm_mesh *mesh);

/* The same tensor for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * float64 temporaries of the set-up live in a static device array of 96 MiB
 * (100663296 bytes) that the library holds on every device it runs on until
 * the process ends; nothing is allocated.  The temporaries of an
 * N1 x N2 x N3 grid take, rounded up to 256 bytes each,
 *   48 N1 N2 N3 + 48 N3 N2 KP + 48 N3 (P2/2+1) KP + 16 (P1 + P2 + P3) + 3840
 * bytes (P the padded lengths, KP = P1/2 + 1 rounded up to a multiple of 16):
 * a 128 x 128 x 32 block needs about 82 MB.  A larger grid is refused with
 * NM_EINVAL (use nm_demag_tensor_init).  The mesh's device must be the
 * current device (else NM_EINVAL).  Synchronous: returns when the tensor is
 * ready.  Calls on one device share the array and are serialised by a lock
 * held for the whole call (the array keeps the last call's contents, every
 * part of which a call writes before reading it).  The tile widths of the FFT
 * passes are left as they are (nm_mesh_tuning sets them): the tuner, which
 * creates timing events, does not run.  Idempotent like nm_demag_tensor_init;
 * the resulting tensor is bitwise the one nm_demag_tensor_init builds. */
nm_status nm_demag_tensor_init_noalloc(nm_mesh *mesh);

/* The float64 real-space tensor N(d) for 0 <= d_k < n[k], written to the
 * device buffer out[6][n3][n2][n1] (xx, yy, zz, xy, xz, yz).  Stand-alone:
 * no mesh needed; enqueued on stream. */
nm_status nm_newell_octant(const int n[3], const double h[3], double *out, void *stream);

/* Block widths of the register-FFT y passes and z convolution of this mesh:
 * 0 the widest column tile, 1 half of it, 2 a quarter.  nm_demag_tensor_init
 * chooses them by timing every width on the mesh (a few launches each on the
 * mesh stream; the choice is cached per padded shape and device).  Every
 * width computes each column identically, so results do not depend on it.
 * With set == 0 this only reads the choice into *y_width, *z_width; with
 * set != 0 it imposes them first (-1 keeps one; values outside -1..2 are
 * NM_EINVAL; a width a length cannot use falls back to 0). */
nm_status nm_mesh_tuning(nm_mesh *mesh, int set, int *y_width, int *z_width);

/* Effective field (Eq. heff with Eq. mass_lumping) of the selected terms at
 * time t: m and h are device nodal vector fields (3 * n_nodes floats). */
nm_status nm_heff(nm_mesh *mesh, const float *m, float *h, unsigned terms, double t);

/* Cell-centred demagnetisation field H_c = -sum N(c-c') Ms_c' mbar_c'
 * (device, 3 * n_cells floats). */
nm_status nm_demag_cell_field(nm_mesh *mesh, const float *m, float *h_cell_out);

/* LLG right-hand side dm/dt (Eq. llg) of the selected terms at time t. */
nm_status nm_llg_rhs(nm_mesh *mesh, const float *m, float *dmdt, unsigned terms, double t);

/* Energies in J: e[0] exchange, e[1] demag, e[2] anisotropy, e[3] Zeeman,
 * e[4] total, e[5] DMI (host array of 6).  Synchronises the stream. */
nm_status nm_energy(nm_mesh *mesh, const float *m, unsigned terms, double t, double e[6]);

/* Advance m (device, in place) from clk->t to t_end with at most max_steps
 * steps (RK4: steps of clk->dt, the last one shortened to land on t_end;
 * DP45: accepted steps, starting from the proposal clk->dt).  Updates *clk.
 * RK4 returns once the steps are queued on the mesh stream (the clock is
 * advanced on the host exactly as the device advances it; kernel errors
 * surface at the next synchronisation).  DP45 synchronises the stream and
 * returns NM_ENONFINITE / NM_ESTEPSIZE when its controller fails; m then
 * holds the last accepted state. */
nm_status nm_llg_step(nm_mesh *mesh, float *m, nm_clock *clk, const nm_integrator *integ,
                      double t_end, long max_steps);

/* Discrete adjoint of nsteps fixed RK4 steps of size dt from the checkpoint
 * m0 (device, 3 * n_nodes) at time t0, for the inverse problems of Sec. 4
 * (gradient of a trajectory objective, Eqs. adjoint_forward and
 * adjoint_objective, taken on the discrete map rather than by reverse
 * integration of the continuous adjoint system).  The forward states of the
 * segment are recomputed into `work`, then the exact reverse recurrence of
 * the four stages runs back to m0.
 *   terms       field terms of the forward run (NM_T_*)
 *   dl_dm       optional device array of per-step loss gradients: entry i
 *               (3 * n_nodes floats) is dl/dm at the state after step
 *               (i + 1) * dl_every of this segment; NULL for none
 *   lambda      device, in: dL/dm at the segment end (from later segments);
 *               out: dL/dm0
 *   grad_hcell  optional device array (3 * n_cells) to which dL/d(per-cell
 *               applied field map) is ADDED; needs NM_T_ZEEMAN
 *   work        device workspace of nm_adjoint_workspace_bytes(mesh, nsteps)
 *               bytes, owned by the caller
 * Asynchronous on the mesh stream; returns NM_EINVAL on bad arguments. */
nm_status nm_adjoint_step(nm_mesh *mesh, const float *m0, double t0, double dt, int nsteps,
                          unsigned terms, const float *dl_dm, int dl_every, float *lambda,
                          float *grad_hcell, float *work);

/* Workspace bytes nm_adjoint_step needs for a segment of nsteps steps. */
size_t nm_adjoint_workspace_bytes(const nm_mesh *mesh, int nsteps);

/* The continuous adjoint of Sec. 4 (Eq. adjoint_system): the joint system
 *   dm/dt = f(t, m),  da/dt = -(df/dm)^T a,  du/dt = -(df/dtheta)^T a
 * integrated backwards with nsteps classical RK4 steps of -dt from t_end,
 * with theta the per-cell applied field map.  No forward state is stored:
 * m is rebuilt by integrating the LLG equation backwards, which costs
 * accuracy (O(dt^4) against the discrete adjoint of nm_adjoint_step) and,
 * for damped dynamics, limits how far back the reconstruction stays close.
 *   m           device, 3 * n_nodes: m(t_end) in, m(t_end - nsteps dt) out
 *   a           device, 3 * n_nodes: dL/dm(t_end) in, a at the earlier time
 *               out (dL/dm there)
 *   grad_hcell  device, 3 * n_cells or NULL: u, the gradient with respect to
 *               the field map, added to what it holds; needs NM_T_ZEEMAN
 * The mesh's stepping buffers serve as scratch (an integration in progress
 * restarts its first stage at the next nm_llg_step).  Asynchronous on the
 * mesh stream; NM_EINVAL for NULL arguments, nsteps < 1, dt <= 0, unknown
 * term bits, NM_T_DEMAG before nm_demag_tensor_init, or a gradient without
 * NM_T_ZEEMAN. */
nm_status nm_adjoint_continuous(nm_mesh *mesh, float *m, double t_end, double dt, int nsteps,
                                unsigned terms, float *a, float *grad_hcell);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of independent LLG solves of uneven
 * size.  Requests wait in a FIFO queue; a scheduler thread admits them while
 * the device memory of admitted solves (nm_mesh_footprint_bytes plus the
 * state) stays within hbm_budget and fewer than max_active run.  Admitted
 * solves stay resident on the device and advance by replays of their own
 * captured DP45 graph on a pool of streams, so many solves' kernels are in
 * flight at once; finished solves leave and waiting ones join between
 * replays.  Each solve runs the same kernels on its own buffers, so results
 * do not depend on the mix.  max_active = 1 is the plain one-at-a-time loop.
 * A server may be used from any thread.
 * ---------------------------------------------------------------------- */
typedef struct nm_server nm_server;

typedef struct {
    size_t hbm_budget;        /* device bytes admitted solves may hold (0: 80% of free) */
    int max_active;           /* most solves admitted at once (>= 1) */
    int n_streams;            /* HIP streams the solves are spread over (1..16) */
    int attempts_per_launch;  /* DP45 attempts per graph replay (1..64) */
} nm_server_desc;

/* One solve: DP45 from t = 0 to t_end; all pointers are HOST memory, copied
 * by nm_serve_submit (the caller may free them on return). */
typedef struct {
    int n[3];
    double h[3];
    double gamma;
    const float *Ms, *A, *alpha;   /* cell arrays, N floats each */
    const float *m0;               /* nodal initial state, 3 * n_nodes floats */
    float h_uniform[3];            /* uniform applied field (A/m) */
    unsigned terms;                /* NM_T_* */
    double rtol, atol, dt0, t_end;
    /* optional cell arrays as in nm_material (NULL: absent; zero-initialise
     * the request so that callers unaware of them leave them absent) */
    const float *Ku, *easy;        /* N and 3*N floats, given together */
    const float *h_cell;           /* 3*N per-cell applied field (A/m) */
    const float *D;                /* N floats, DMI constant (J/m^2) */
    int dmi_type;                  /* NM_DMI_INTERFACIAL (0) or NM_DMI_BULK */
    const float *Kc, *cubic;       /* N and 6*N floats, given together */
} nm_solve_request;

typedef struct {
    int status;                    /* NM_OK, NM_ENOTREADY or the solve's error */
    double t;                      /* time reached */
    long accepted, rejected, rhs_evals;
    double t_submit, t_admit, t_done;  /* nm_server_clock() seconds */
} nm_solve_result;

nm_status nm_server_create(const nm_server_desc *desc, nm_server **out);

/* Stop the scheduler, release every solve (waiting, running or unpolled). */
nm_status nm_server_destroy(nm_server *server);

/* Queue a request (non-blocking); *ticket identifies it for nm_serve_poll. */
nm_status nm_serve_submit(nm_server *server, const nm_solve_request *req, uint64_t *ticket);

/* Wait up to timeout_ms for the solve: NM_OK fills *res (and the host array
 * m_out, 3 * n_nodes floats, when not NULL) and forgets the ticket;
 * NM_ENOTREADY if still running; NM_EINVAL for an unknown ticket. */
nm_status nm_serve_poll(nm_server *server, uint64_t ticket, nm_solve_result *res, float *m_out,
                        int timeout_ms);

/* Seconds on the server clock (steady, process-wide). */
double nm_server_clock(void);

/* Per-kernel timing (measurement only).  While enabled, every kernel the
 * mesh launches is bracketed by a pair of HIP events on the mesh stream and
 * its duration is accumulated in one of these slots. */
enum {
    NM_PROF_XFWD = 0,      /* nodal -> cell average, R2C along x */
    NM_PROF_YFWD = 1,      /* FFT along y (3D) */
    NM_PROF_CONV = 2,      /* fused FFT + k-space product + inverse (z in 3D, y in films) */
    NM_PROF_YINV = 3,      /* inverse FFT along y (3D) */
    NM_PROF_XINV = 4,      /* C2R along x -> cell field */
    NM_PROF_STENCIL = 5,   /* local terms + LLG + stage epilogue */
    NM_PROF_CONTROL = 6,   /* step controller / bookkeeping */
    NM_PROF_OTHER = 7,
    NM_PROF_SLOTS = 8
};

/* on != 0: start profiling (clears the accumulators); on == 0: stop. */
nm_status nm_profile_enable(nm_mesh *mesh, int on);

/* Synchronise the stream and return, per slot, the summed kernel time (ms)
 * and the number of launches since profiling was enabled (host arrays of
 * NM_PROF_SLOTS entries). */
nm_status nm_profile_read(nm_mesh *mesh, double ms[NM_PROF_SLOTS], long long counts[NM_PROF_SLOTS]);

/* Message describing the last error on the calling thread. */
const char *nm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NM_H */
