// Internal declarations of the gfx950 FDTD-PIC library: kernel argument
// blocks and launchers.  Device state is FP32 in normalised units:
//   lengths in cells, time in steps,
//   E in V/m, Ht = eta0 H in V/m, Jt = (dt/eps0) J in V/m,
//   particle u = gamma v / c (dimensionless), positions in cells.
// With S = c dt / dx the field updates read
//   Ht -= S curl E,      E += S curl Ht - Jt_pol - Jt_b,
//   Jt_pol += cbt E - d Jt_pol,  cbt = 2 (wp dt)^2/(2 + g dt), d = 2 g dt/(2 + g dt),
// which is Eq. 6 / Eq. 8 of the paper rescaled (the increment form keeps
// the small damping d exact when rounded to FP32).
//
// Everything that changes from step to step (which H buffer is current,
// steps since the last sort, which particle buffer set is current, the step
// number) lives in a DevState in device memory and is advanced by the
// kernels themselves.  The argument blocks are therefore fixed for the life
// of a simulation, so a sequence of steps can be captured once in a HIP
// graph, and one launch can serve many simulations (an array of argument
// blocks in device memory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int PBLOCK = 256;  // particle sort kernels
// Push / deposit: one wavefront per workgroup. Wavefronts of one window take
// very different numbers of reduction rounds, and a workgroup's slot on the
// compute unit is freed only when its last wavefront ends, so single-wave
// workgroups keep the units fuller (8 % faster than 256 threads).
constexpr int PUSH_BLOCK = 64;
constexpr int FX = 64;       // default field tile: 64 x 4 cells of one z plane
constexpr int FY = 4;

// Field-kernel tile shapes (cells along x, y of one z plane per workgroup)
// and tile orders the autotuner chooses from; shape 0 is the default.
// Order 0 numbers tiles x, then y, then z (a plane at a time); order 1 x,
// then z, then y (a band of rows marches through all planes, so the next
// plane's values are still in L2 when its tiles run).
constexpr int N_TILE_SHAPES = 16;
constexpr int TILE_FX[N_TILE_SHAPES] = {64, 64, 128, 256, 32, 64, 128, 32, 64, 64, 128, 256, 32, 64, 128, 32};
constexpr int TILE_FY[N_TILE_SHAPES] = {4, 2, 2, 1, 8, 8, 4, 4, 4, 2, 2, 1, 8, 8, 4, 4};
constexpr int TILE_ZO[N_TILE_SHAPES] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1};
// A batched field launch gives each workgroup this many consecutive tiles of
// one member.  One: a workgroup's tiles run one after another (the next
// tile's loads wait for the last one's stores, which may alias them as far
// as the compiler knows), which costs more than the member lookup (work-unit
// table, argument block, device state) it would share.
constexpr int BATCH_TILES = 1;

struct DevState {
    int parity;      // H[parity] holds H^{n-1/2} at the start of step n
    int since_sort;  // steps since the last cell sort
    int pcur;        // particle buffer set in use
    int pad;
    long long step;  // steps taken
    float *P[6];     // set pcur's arrays (x, y, z, ux, uy, uz), written with pcur by the sort
};

// CPML data of one axis.  Coefficients are per position along the axis:
// E-type at node i, H-type at i + 1/2; k* hold 1/kappa.  psi arrays cover
// the two absorbing slabs (2*npml planes) of that axis:
//   x: idx = p + 2npml*(j + ny*k)   y: idx = i + nx*(p + 2npml*k)
//   z: idx = i + nx*(j + ny*p),     p = q < npml ? q : q - (n - 2npml).
// psi[a][0] / psi[a][1] belong to the lower / higher numbered updated
// component whose curl differentiates along a (x: y,z   y: x,z   z: x,y):
// psiE[x][0] is the memory of dHz/dx in the Ey update, psiH[z][1] that of
// dEx/dz in the Hy update, and so on.
struct PmlAxis {
    int on;
    int npml;
    const float *bE, *cE, *kE;
    const float *bH, *cH, *kH;
    float *psiE[2];
    float *psiH[2];
};

struct FieldArgs {
    int nx, ny, nz;
    int tile;    // tile shape index (TILE_FX / TILE_FY)
    int gx, gy;  // tiles along x and y
    int per[3];
    float S;
    float *E[3];
    float *H[2][3];  // ping-pong: the H update reads H[parity], writes H[parity ^ 1]
    float *Havg[3];  // (H^{n-1/2} + H^{n+1/2})/2 inside the particle box, or null
    PmlAxis pml[3];
    // Drude polarization current on the metal bounding box [lo, hi)
    int mlo[3], mhi[3];
    float *Jp[3];
    const float2 *coef;  // (cbt, d) per box cell
    // when set, the E update also copies E^n and J_pol^{n-1/2} of the metal
    // box here ([6][box cells], E then J_pol): the reverse pass's snapshot
    float *snap;
    // bunch current: read and cleared inside the particle box (+ margin)
    float *Jb[3];
    unsigned long long *Jq[3];  // the fixed-point form instead of Jb, or null
    double qinv;                // V/m per fixed-point unit
    const int *pbox;  // device [6]: lo x,y,z, hi x,y,z (cells, inclusive), or null
    int *nan_flag;
    DevState *st;
};

// One-pass field sweep (E update of step n, then H update of step n + 1).
// Every field is one block with its components FIELD_STRIDE apart; the E-side
// state (E, J_pol, the E-side CPML memories) is read from the *in blocks and
// written to the *out blocks, since a workgroup recomputes its neighbours'
// new E at its edges from their old values.
constexpr int FUSED_ROWS = 2;    // y rows per lane
constexpr int FUSED_PLANES = 16;  // z planes per workgroup
struct FusedArgs {
    int nx, ny, nz;
    int per[3];
    float S;
    int N;                       // cells: component stride of E, H, Havg, J_b
    const float *Ein;            // [3][N] E^n
    float *Eout;                 // [3][N] E^{n+1}
    const float *Hin;            // [3][N] H^{n+1/2}
    float *Hout;                 // [3][N] H^{n+3/2}
    float *Havg;                 // [3][N] (H^{n+1/2} + H^{n+3/2}) / 2 in the particle box, or null
    int pon[3], npml[3];
    const float *tab[3];         // per axis [6][n]: bE, cE, kE, bH, cH, kH
    int slab[3];                 // psi cells per component of an axis
    const float *psiEin[3];      // per axis [2][slab]
    float *psiEout[3];
    float *psiH[3];              // updated in place (one owner per H cell)
    int mlo[3], mhi[3];          // metal box [lo, hi)
    int nbox;                    // metal-box cells: component stride of J_pol
    const float *Jpin;           // [3][nbox] J_pol^{n-1/2}
    float *Jpout;                // [3][nbox] J_pol^{n+1/2}
    const float2 *coef;          // (cbt, d) per metal-box cell
    const float *Jb;             // [3][N] bunch current, or null (read only: cleared afterwards)
    const int *pbox;             // device [6] live-cell box of the last sort, or null
    int *nan_flag;
    DevState *st;
    int gy;                      // y blocks of FUSED_ROWS rows
};

struct PartArgs {
    int n;  // particles; their arrays are the device state's P (the current buffer set)
    int nx, ny, nz;
    int per[3];
    const float *E[3];
    const float *B[3];  // (Ht^{n-1/2} + Ht^{n+1/2}) / 2, valid inside the particle box
    float *Jb[3];
    // fixed-point bunch current (deterministic deposit): integer atomics of
    // round(current * qscale) per particle and slot, or null for the FP32
    // atomics into Jb
    unsigned long long *Jq[3];
    float qscale;
    float S;   // c dt / dx
    float ah;  // q dt / (2 m c), per V/m
    float qd;  // -q w / (eps0 dx^2), V/m
    unsigned long long *pushes;  // one counter per wavefront: [ceil(n / 64)]
    DevState *st;
};

struct SortArgs {
    int n;
    int nx, ny, nz;
    int ncell;
    float *P[2][6];
    int *id[2];
    int *key;
    int *rank;
    int *counts;  // [ncell + 1]
    // per key: runs of that key in the array's current order, and where the
    // (last recorded) run starts; a key with one run is contiguous and keeps
    // its order in the scatter
    int *runs;    // [ncell + 1]
    int *first;   // [ncell + 1]
    int *box;     // [6] bounding box of live cells (lo x, y, z, hi x, y, z)
    int *boxpart; // [6 * count workgroups] each count workgroup's box, reduced into box
    int *scan_tmp;  // [scan_tmp_size(ncell + 1)] the scans' tile sums
    DevState *st;
};

struct ProbeArgs {
    int nprobe, nfreq;
    const int *pidx;      // linear Ez index per probe
    const double *omega;  // rad/s
    double *fre, *fim;
    float *series;        // [series_len * nprobe] or null
    long long series_len;
    double dt;
    const float *Ez;
    // optional FP64 record of Ez at the probes for steps g0+1 .. g0+gn
    // (gser[(n - g0 - 1) * nprobe + p]), used by the gradient's objective
    double *gser;
    long long g0, gn;
    DevState *st;
};

// A particle is live when every coordinate is finite and inside [0, n) (cell
// units); a lost particle stores x = -1.  Every kernel indexes the grid from
// a position only after this test, so non-finite values never become indices.
__device__ __forceinline__ bool live_pos(float x, float y, float z, int nx, int ny, int nz)
{
    return x >= 0.f && x < (float)nx && y >= 0.f && y < (float)ny && z >= 0.f && z < (float)nz;
}

// Cells the particle box is widened by: a particle moves less than S cells
// per step, and its gather / deposit stencil reaches two cells past its own.
__device__ __forceinline__ int box_margin(int since_sort, float S)
{
    return 3 + (int)ceilf((float)(since_sort + 1) * S);
}

inline int field_tiles(int nx, int ny, int nz, int shape = 0)
{
    const int fx = TILE_FX[shape], fy = TILE_FY[shape];
    return ((nx + fx - 1) / fx) * ((ny + fy - 1) / fy) * nz;
}

// Work units of one member in a batched field launch.
inline long long batch_field_units(int nx, int ny, int nz, int shape)
{
    return ((long long)field_tiles(nx, ny, nz, shape) + BATCH_TILES - 1) / BATCH_TILES;
}

// Linear offset to the neighbour at distance d = +-1 along an axis of n
// cells with stride st: wraps on a periodic axis; across a wall it points
// at the cell itself and clears `ok` (the neighbour value is then 0).
__device__ __forceinline__ int nb_off(int i, int d, int n, int per, int st, bool &ok)
{
    const int r = i + d;
    const bool in = r >= 0 && r < n;
    ok = in || per;
    const int w = r < 0 ? r + n : r - n;
    return in ? d * st : (per ? (w - i) * st : 0);
}

// Global-memory pointers.  A pointer the kernels read from device memory (the
// batched entry points' argument blocks) or pass through a scalar-register
// pin is generic to the compiler, which then emits flat loads, stores and
// atomics: 64-bit vector addresses, and counted with the scalar loads, so a
// wait for either waits for both.  Every pointer the library hands its kernels
// addresses global memory (the same bits), so accesses go through G(p).
template <class T>
using gp = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gp<T> G(T *p)
{
    return (gp<T>)p;
}
// Two floats as a plain vector (HIP's float2 is a class, which C++ cannot
// copy out of a global-typed lvalue).
typedef float fvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void gatomic_add(gp<float> p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gatomic_add(gp<unsigned long long> p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup -> tile with XCD locality: the 8 XCDs receive workgroups round
// robin, so workgroup b runs on XCD b % 8; give each XCD a contiguous block
// of tiles.
__device__ __forceinline__ int xcd_tile()
{
    const int B = gridDim.x;
    const int b = blockIdx.x;
    return (B % 8 == 0) ? (b % 8) * (B / 8) + b / 8 : b;
}

// xcd_tile() with each XCD walking its range from the end: a launch that
// follows one in the forward order starts on the tiles the other wrote last,
// which are still in the Infinity Cache.
__device__ __forceinline__ int xcd_tile_rev()
{
    const int B = gridDim.x, b = blockIdx.x;
    const int x = b & 7, i = b >> 3, q = B >> 3, r = B & 7;
    const int len = q + (x < r ? 1 : 0);
    return x * q + min(x, r) + (len - 1 - i);
}

// Position of plane q inside the two absorbing slabs of an axis.
__device__ __forceinline__ int slab_p(int q, int n, int np) { return q < np ? q : q - (n - 2 * np); }

// launchers (stream-ordered, no synchronisation)
void launch_fused(const FusedArgs &a, hipStream_t s);
void launch_jb_clear(float *Jb, int N, int nx, int ny, int nz, const int *per, const int *pbox, float S,
                     const DevState *st, hipStream_t s);
void launch_h_update(const FieldArgs &a, hipStream_t s);
void launch_e_update(const FieldArgs &a, hipStream_t s);
void launch_push_deposit(const PartArgs &a, int mode, hipStream_t s);
void launch_probe(const ProbeArgs &a, hipStream_t s);  // also advances the DevState
void launch_fill_i32(int *p, int v, long long n, hipStream_t s);
void launch_sort(const SortArgs &a, int *scan_tmp, hipStream_t s);
// The sorts of nmem simulations (every one with particles) in one launch per
// kernel: args[nmem] on the device, own[nown] the count and scatter
// workgroups (member << 24 | workgroup index in that member).
void launch_sort_batch(const SortArgs *args, const int *own, int nown, int nmem, hipStream_t s);
int scan_tmp_size(long long n);

// Batched forms: one launch over many simulations.  `args` is a device array
// of per-simulation argument blocks; `own` a device table with one entry per
// work unit of the launch (field tile / particle workgroup, `total` of them):
// simulation index << 24 | the unit's index within that simulation.
void launch_h_update_batch(const FieldArgs *args, const int *own, int total, int shape, hipStream_t s);
void launch_e_update_batch(const FieldArgs *args, const int *own, int total, int shape, hipStream_t s);
void launch_push_deposit_batch(const PartArgs *args, const int *own, int total, int mode, hipStream_t s);
void launch_probe_batch(const ProbeArgs *args, int n, hipStream_t s);

// ---- reverse-time adjoint of the linear field step (bunch current fixed) ----
//
// Adjoint state in the same normalised units and compact layout as the
// forward fields: Ea = dL/dE, Ha = dL/dHt, Ja = dL/dJt_pol (metal box);
// psiEa / psiHa are the adjoint CPML memories (same slab layout as psiE /
// psiH), DE / DH per-step scratch holding the adjoint weight of each slab
// difference.
struct AdjArgs {
    int nx, ny, nz;
    int gx, gy;
    int per[3];
    float S;
    float *Ea[3];
    float *Ha[3];
    PmlAxis pml[3];  // forward coefficient tables (b, c, 1/kappa) and slab sizes
    float *psiEa[3][2], *psiHa[3][2];
    float *DE[3][2], *DH[3][2];
    int mlo[3], mhi[3];
    float *Ja[3];
    const float2 *coef;  // (cbt, d) per metal-box cell
    const float *traj;   // this step's E^n (3 comps) then Jt^{n-1/2} (3 comps), metal box
    double *gcb, *gd;    // per metal-box cell: dL/dcbt and dL/dd summed over its edges
    int nprobe;
    const int *pidx;
    const float *seed;   // dL/dEz at the probes for E^n, or null
    int mode;            // bit 0: reverse the step; bit 1: add seed and prepare the CPML weights
};

// Copy of a box [lo, lo + w) of three grid arrays to / from a packed buffer.
struct BoxCopyArgs {
    float *grid[3];
    float *packed;  // [3][w0*w1*w2], x fastest
    int nx, ny;
    int lo[3], w[3];
    int to_grid;
};

// Forward values the gradient needs at step n on the metal box.
void launch_adj_face(const AdjArgs &a, hipStream_t s);
void launch_adj_edge(const AdjArgs &a, hipStream_t s);
void launch_box_copy(const BoxCopyArgs &a, hipStream_t s);

// FP64 diagnostics
struct DiagArgs {
    int nx, ny, nz;
    int per[3];
    int npml[3];
    int mlo[3], mhi[3];
    const float *E[3];
    const float *H[3];
    int np;
    const float *x, *y, *z, *ux, *uy, *uz;
    double *rho;        // (nx+1)(ny+1)(nz+1) nodes, x fastest
    const double *rho0; // same layout or null
    double qw_over_vol; // q w / dx^3
    double eps0_over_dx;
    double *acc;        // reduction outputs
};
void launch_rho(const DiagArgs &a, hipStream_t s);
void launch_diag_reduce(const DiagArgs &a, hipStream_t s);

}  // namespace pic
