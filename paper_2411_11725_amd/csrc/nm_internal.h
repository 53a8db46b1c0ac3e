// Internal declarations of the MI355X nodal finite-difference library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "nm.h"

namespace nm {

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;  // mu0 = 4 pi 1e-7
constexpr int kTwN = 4096;        // twiddle table: tw[t] = exp(-2 pi i t / kTwN)
constexpr int kMaxFFT = 1024;     // longest padded axis handled
constexpr int kBlock = 256;       // threads per block of the pointwise kernels

// Device-resident integrator state (read by every stepping kernel so that a
// whole attempt can be replayed without host round trips).
struct Ctrl {
    double t, dt, dt_prop, t_end;
    double rtol, atol, dt_min, dt_max, stop_torque;
    double err, max_torque;
    double norm_scale;       // 1 / (3 * active nodes): RMS over node components
    long long accepted, rejected, rhs_evals, attempts, max_accepted;
    int done, status, rejected_last, accept;
    double *log;
    long long log_cap;
};

// Block partials written by the last DP45 stage and reduced by the controller.
struct ErrPartial {
    double sumsq;
    float maxf;
    int nonfinite;
};

// Arguments of the fused node kernel (mesh constants) and of one of its
// stages (buffers, clock).
struct StencilParams {
    int N1, N2, N3, NX, NY, NZ;
    long long nn, nc;
    float Kp[8], Mp[8];
    // node kernel: packed cell data and the pre-weighted cell-field source
    const float4 *cellP;           // {2A with the sign bit of Ku, sqrt|Ku| e}
    // {mu0 Ms V/8 (H_d [+ static H_ext]), mu0 Ms V/8 drive mask} per cell, or NULL
    const float4 *src;
    int drive;                     // add the drive (the w component times sin and its amplitude)
    int W;                         // LDS window length per z offset: 256 + 2 NX + 2
    int faces;                     // K^e couples face neighbours (cells are not cubes)
    unsigned zcols;                // node kernel: 256-node ranges per node layer
    const float *Dc;               // DMI constant per cell, or NULL
    int dmi_bulk;                  // bulk (m . curl m) rather than interfacial DMI
    float gx[4], gy[4], gz[4];     // DMI weights (see the node kernel)
    const float4 *cubP;            // cubic anisotropy per cell {Kc, c1}, {c2, 0}, or NULL
    float gq[2], gw;               // Gauss-point basis values and weight
    float rNX, rNY;                // 1 / NX, 1 / NY
    // energy kernel: raw cell data
    const float *wc, *A2, *Ku, *easy, *hcell, *dmask, *hd;
    float hu[3], damp[3];
    double dfreq, dphase;
    const float *inv_mass, *alpha_n, *gp_n;
    unsigned terms;
};

struct StageArgs {
    const float *in;
    float *out, *y_next, *mstate, *acc;
    float *lo;               // RK4: the state's compensation (low part), or null
    float *k[7];
    const Ctrl *ctrl;
    ErrPartial *partials;
    double t0, dt0;
};

// One solve of a batched launch: everything the batched kernels read about
// it, in device memory (one descriptor per slot of a batch group).  Slots
// with active = 0 are empty: every batched kernel returns at once there.
struct BatchSlot {
    int active;
    // demag passes
    int N1, N2, N3, NZ, P2, K1, KP, P2h, P3h, src_mode;
    const float *Ms;
    float2 *spec;
    const float *tensor;
    float *hd;
    const float *wc;
    const float4 *wstat;
    const float *stage_in[8];    // input of DP45 stage s (2..7)
    // controller and stage epilogue
    Ctrl *ctrl;
    ErrPartial *partials;
    int np;                      // node-kernel blocks = error partials
    float *mstate, *y0, *y1, *k1, *k7;
    long long n3;                // 3 n_nodes
    // node kernel
    StencilParams P;
    StageArgs S[8];              // DP45 stages 2..7
};

// Shape class of a batch group: solves with equal padded lengths, node
// window, basis and terms run the same kernel instantiations; grids cover the
// largest mesh of the class, blocks beyond a solve's own range return.
struct BatchClass {
    int P1, P2, P3, nit;
    unsigned terms;
    int xt;                      // node-kernel term instantiation (node_xt)
    int tune_y, tune_z;          // column-tile widths of the register FFT passes
    // grid extents, fitted to the members a group's graphs were captured
    // for: the most rows (gN2) and cell layers (gN3) and node-kernel blocks
    // of any of them; blocks past a member's own extent return at once
    int gN2, gN3;
    unsigned node_blocks;
};

struct ProfState;  // per-kernel event timing (measurement only)

// Neighbour-weight tables of the node kernel, generated from the element
// matrices of the quadratic terms (terms.hip).
struct ElementTables {
    float Kp[8], Mp[8];      // stiffness and mass by axis-difference pattern
    float gx[4], gy[4], gz[4];   // antisymmetric first-derivative parts per axis
    float gq[2], gw;         // psi_1 at the two Gauss points; weight of a point
};
bool generate_element_tables(const double h[3], ElementTables *out, std::string *why);

// Element access by 32-bit byte offset from a uniform base pointer: the loads
// and stores then take the scalar-base form with one 32-bit offset register.
// Callers keep each offset below 4 GiB (a component array of the largest
// mesh, 512 cells per axis, is well below).
template <class T>
__device__ __forceinline__ T ldo(const T *base, unsigned byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void sto(T *base, unsigned byte_off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

// XCD-aware block order: the dispatcher hands consecutive workgroups to the 8
// XCDs in turn, each with its own L2.  Renumbering so that XCD x works through
// one contiguous range of logical blocks keeps neighbouring blocks (which
// share halo rows) in the same L2.  A bijection of [0, nb).
constexpr unsigned kXCDs = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned q = nb / kXCDs, r = nb % kXCDs, x = b % kXCDs, k = b / kXCDs;
    return x * q + (x < r ? x : r) + k;
}

// device memory: hipMalloc / hipFree, or a pool (see pool.hip)
struct DevPool;
constexpr size_t kPoolHostBlock = 4096;   // pinned host blocks recycled by a pool
DevPool *pool_create();
DevPool *pool_create_user(const nm_allocator &a);   // every block from the caller's hooks
void pool_destroy(DevPool *P);
void set_thread_pool(DevPool *P);   // allocations of the calling thread come from P
DevPool *thread_pool();
hipError_t dev_alloc(void **p, size_t bytes, DevPool *P);
void dev_free(void *p, DevPool *P);
hipError_t host_alloc(void **p, size_t bytes, DevPool *P);
void host_free(void *p, DevPool *P);
}  // namespace nm

struct nm_mesh {
    int N1, N2, N3;          // cells
    int NX, NY, NZ;          // nodes per axis (N + 1)
    int P1, P2, P3;          // padded FFT lengths (powers of two)
    int K1;                  // P1 / 2 + 1 complex x-frequencies
    int KP;                  // row pitch of spectrum and tensor: K1 rounded up to 16
    int P2h, P3h;            // P2 / 2 + 1, P3 / 2 + 1 stored tensor frequencies
    double h[3], V, gamma;
    int64_t n_nodes, n_cells;
    hipStream_t stream;
    int device;
    nm::DevPool *pool;       // where the buffers came from (NULL: hipMalloc)
    bool owns_pool;          // pool wraps the caller's allocator hooks (freed with the mesh)

    // owned material copies (cell arrays) and derived quantities
    float *Ms, *A2, *Ku, *easy, *h_cell, *drive_mask;
    float *Dc;               // interfacial DMI constant per cell (when given)
    float *wc;               // mu0 Ms_c V / 8: weight of a cell-constant field
    float4 *cellP;           // packed per cell: {2A with the sign of Ku, sqrt|Ku| e}
    float4 *wstat;           // per cell: mu0 Ms V/8 {h_uniform + h_cell, drive mask}
    float h_uniform[3], drive_amp[3];
    double drive_freq, drive_phase;
    bool has_anis, has_hcell, has_drive, has_dmi;
    float Kp[8], Mp[8];      // element matrices by axis-difference pattern
    // DMI: the antisymmetric part of int phi_a d_k phi_b between nodes that
    // differ by d is d_k gx[(d_y != 0) + 2 (d_z != 0)] (k = x) and
    // d_y gy[(d_x != 0) + 2 (d_z != 0)] (k = y): products of 1D mass factors
    float gx[4], gy[4], gz[4];
    bool dmi_bulk;           // bulk DMI (m . curl m) instead of interfacial
    bool has_cubic;
    float4 *cubP;            // per cell: {Kc, c1}, {c2, 0} (cubic anisotropy)
    float gq[2], gw;         // 1D basis value psi_1 at the two Gauss points; point weight V / 8

    // nodal coefficients
    float *inv_mass, *alpha_n, *gp_n;

    // demagnetisation
    float2 *spec;            // [3][N3][P2][KP] complex workspace
    float *tensor;           // [6][P3h][P2h][KP] real k-space tensor / (P1 P2 P3)
    float *hd;               // demag cell field: [3][n_cells] H_d, or the node
                             // kernel's source, float4 [n_cells] (see demag_forward_conv_inverse)
    bool tensor_ready;

    // integrator buffers
    float *y[2], *acc, *k[7];
    // RK4 state compensation: the low part of a two-sum of every state update,
    // carried from step to step (and from call to call while the caller
    // continues the same state: same buffer, t where the last call ended)
    float *mlo;
    const float *lo_mag;
    double lo_t;
    bool lo_valid;
    nm::Ctrl *ctrl;          // device controller state
    nm::Ctrl *ctrl_host;     // pinned mirror for read-back
    int64_t n_active;        // nodes with positive lumped mass
    nm::ErrPartial *partials;
    int n_partials;
    double *ered;            // energy block partials [4][n_eblocks]
    int n_eblocks;
    nm::ProfState *prof;     // non-null while profiling is enabled

    // captured stepping graph (one batch of attempts / steps), launched on
    // `stream`; captured on the private `cap_stream`.  gtail[k] holds the
    // same graph with 2^k attempts (< g_batch) for the end of an integration
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    hipGraphExec_t gtail[6];
    // tile choices of the register-FFT passes (see the tuner)
    int tune_y, tune_z;
    // recorded adjoint segment and its key
    hipGraphExec_t adj_gexec;
    int adj_nsteps, adj_every;
    unsigned adj_terms;
    bool adj_gather;
    double adj_dt;
    float *adj_work;
    // recorded step of the continuous adjoint and its key
    hipGraphExec_t cadj_gexec;
    unsigned cadj_terms;
    double cadj_dt;
    bool cadj_gather;
    const float *cadj_m, *cadj_a;
    int g_method;
    unsigned g_terms;
    float *g_mag;
    int g_batch;
};

namespace nm {

void set_error(const std::string &msg);

// Kernel launch on the mesh stream.  While the mesh is being profiled the
// launch carries a start / stop event pair (recorded by the dispatch itself,
// so the pair brackets exactly the kernel's execution) accumulated in `slot`.
void prof_pair(nm_mesh *m, int slot, hipEvent_t *start, hipEvent_t *stop);
void prof_free(nm_mesh *m);
#define NM_LAUNCH(mesh, slot, kernel, grid, block, shmem, ...)                                   \
    do {                                                                                          \
        hipEvent_t ev_a_ = nullptr, ev_b_ = nullptr;                                              \
        if ((mesh)->prof) prof_pair((mesh), (slot), &ev_a_, &ev_b_);                              \
        if (ev_a_ && ev_b_)                                                                       \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, (mesh)->stream, ev_a_, ev_b_, 0,    \
                                  __VA_ARGS__);                                                   \
        else                                                                                      \
            hipLaunchKernelGGL(kernel, grid, block, shmem, (mesh)->stream, __VA_ARGS__);          \
    } while (0)

const float2 *twiddles(int device);   // per-device table (built at mesh creation)

// demag FFT pipeline: m (nodal, stage input) -> mesh->hd (cell field); the
// ctrl variant skips its kernels once the device controller reports done
// src_mode 0: hd = H_d, [3][n_cells]; 1 and 2: hd = the source the node kernel
// gathers, one float4 per cell: {mu0 Ms V/8 H_d, 0} (1) or
// {mu0 Ms V/8 (H_d + h_uniform + h_cell), mu0 Ms V/8 drive mask} (2)
hipError_t demag_forward_conv_inverse(nm_mesh *m, const float *mag, int src_mode);
hipError_t tune_passes(nm_mesh *m);   // block widths of the register-FFT passes
int tile_widths(int L);               // how many column-tile widths (0, 1, 2) length L has
hipError_t demag_forward_conv_inverse_ctrl(nm_mesh *m, const float *mag, const Ctrl *ctrl,
                                           int src_mode);

// tensor set-up: octant in float64 and the k-space transform
hipError_t launch_newell_octant(int n1, int n2, int n3, const double h[3], double *out,
                                hipStream_t s);
hipError_t build_kspace_tensor(nm_mesh *m);
size_t kspace_scratch_bytes(const nm_mesh *m);          // float64 temporaries of the set-up
size_t kspace_scratch_bytes(int N1, int N2, int N3, int P1, int P2, int P3);
hipError_t build_kspace_tensor_with(nm_mesh *m, void *work);   // temporaries in work; no allocation

// stencil / LLG / stage kernels
// kModeAdjFwd: store H(y_s) and form the next RK4 stage input (adjoint recompute)
enum StencilMode { kModeField = 0, kModeRhs = 1, kModeRK4 = 2, kModeDP45 = 3, kModeAdjFwd = 4 };

struct StageSpec {
    int mode;
    int stage;               // 1-based stage index
    const float *in;         // stage input (nodal m)
    float *out;              // field / rhs output (modes 0, 1)
    float *y_next;           // next stage input
    float *mstate;           // state at the start of the step (stepping modes)
    double t0;               // start-of-step time when ctrl is null
    double dt0;              // step when ctrl is null (RK4 / adjoint recompute)
    bool use_ctrl;           // stepping modes: t, dt from the device controller
    float *lo;               // RK4 stage 4: compensation of the state (null: plain update)
};

hipError_t launch_stencil(nm_mesh *m, unsigned terms, const StageSpec &sp);

// batched launches over the cap slots of a group (grid z = slot)
int window_items(int NX, int NZ);          // node-kernel LDS window items (0: direct loads)
int node_xt(const nm_mesh *m, unsigned terms);   // node-kernel term instantiation of a mesh
void batch_slot_fill(const nm_mesh *m, unsigned terms, Ctrl *ctrl, float *mstate, BatchSlot *out);
hipError_t launch_batch_demag(const BatchClass &bc, const BatchSlot *slots, int cap, int stage, hipStream_t st);
hipError_t launch_batch_node(const BatchClass &bc, const BatchSlot *slots, int cap, int stage, hipStream_t st);
hipError_t launch_batch_control(const BatchSlot *slots, int cap, hipStream_t st);
hipError_t launch_batch_finish(const BatchClass &bc, const BatchSlot *slots, int cap, hipStream_t st);
dim3 stencil_grid(const nm_mesh *m);   // blocks of the fused node kernel
hipError_t launch_energy(nm_mesh *m, const float *mag, unsigned terms, double t, double e[6]);
hipError_t launch_dp45_control(nm_mesh *m);
hipError_t launch_dp45_finish(nm_mesh *m, float *mstate);
hipError_t launch_cell_pack(nm_mesh *m);   // cellP, wstat from the raw copies
// attempts for the next replay of a DP45 integration: the full batch while
// the host mirror of the controller says at least that many steps are left
// (by step count and by time at the proposed step), else the largest power
// of two not above what is left, so that no attempt of the replay is idle
int next_batch(const nm_mesh *m, int batch);
int batch_for(double est, int batch);   // batch if est >= batch, else the largest power of two <= est (>= 1)
void mesh_release(nm_mesh *m);             // free a mesh whose stream work has completed
hipError_t launch_rk4_advance(nm_mesh *m);

// stepping building blocks shared by nm_llg_step and the solve server
nm_status step_begin(nm_mesh *m, float *mag, const nm_clock *clk, const nm_integrator *in,
                     double t_end, long max_steps, int *batch);
// one replay of `batch` steps / attempts (batch == full, or a power of two
// below it) from the graphs keyed on `full`
hipError_t step_batch(nm_mesh *m, float *mag, int method, unsigned terms, int full, int batch);
hipError_t ctrl_readback(nm_mesh *m);
nm_status step_finish(nm_mesh *m, int method, nm_clock *clk);

}  // namespace nm
