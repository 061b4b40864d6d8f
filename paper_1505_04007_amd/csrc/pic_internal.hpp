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

constexpr int PBLOCK = 256;  // particle kernels
constexpr int FX = 64;       // field tile: 64 x 4 cells of one z plane
constexpr int FY = 4;

struct DevState {
    int parity;      // H[parity] holds H^{n-1/2} at the start of step n
    int since_sort;  // steps since the last cell sort
    int pcur;        // particle buffer set in use
    int pad;
    long long step;  // steps taken
};

// CPML data of one axis.  Coefficients are per position along the axis:
// E-type at node i, H-type at i + 1/2; k* hold 1/kappa.  psi arrays cover
// the two absorbing slabs (2*npml planes) of that axis:
//   x: idx = p + 2npml*(j + ny*k)   y: idx = i + nx*(p + 2npml*k)
//   z: idx = i + nx*(j + ny*p),     p = q < npml ? q : q - (n - 2npml).
// psi[a][0] / psi[a][1] belong to the lower / higher numbered component
// that is differentiated along a (x: y,z   y: x,z   z: x,y).
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
    // bunch current: read and cleared inside the particle box (+ margin)
    float *Jb[3];
    const int *pbox;  // device [6]: lo x,y,z, hi x,y,z (cells, inclusive), or null
    int *nan_flag;
    DevState *st;
};

struct PartArgs {
    int n;
    float *P[2][6];  // x, y, z, ux, uy, uz for each buffer set
    int nx, ny, nz;
    int per[3];
    const float *E[3];
    const float *B[3];  // (Ht^{n-1/2} + Ht^{n+1/2}) / 2, valid inside the particle box
    float *Jb[3];
    float S;   // c dt / dx
    float ah;  // q dt / (2 m c), per V/m
    float qd;  // -q w / (eps0 dx^2), V/m
    unsigned long long *pushes;  // one counter per wavefront: [gridDim * PBLOCK / 64]
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
    int *box;     // [6] bounding box of live cells, written by the count kernel
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

inline int field_tiles(int nx, int ny, int nz)
{
    return ((nx + FX - 1) / FX) * ((ny + FY - 1) / FY) * nz;
}

// launchers (stream-ordered, no synchronisation)
void launch_h_update(const FieldArgs &a, hipStream_t s);
void launch_e_update(const FieldArgs &a, hipStream_t s);
void launch_push_deposit(const PartArgs &a, int mode, hipStream_t s);
void launch_probe(const ProbeArgs &a, hipStream_t s);  // also advances the DevState
void launch_fill_i32(int *p, int v, long long n, hipStream_t s);
void launch_sort(const SortArgs &a, int *scan_tmp, hipStream_t s);
int scan_tmp_size(int n);

// Batched forms: one launch over many simulations.  `args` is a device array
// of per-simulation argument blocks; `start` a device prefix table of work
// units (field tiles / particle workgroups) per simulation, start[n] = total.
void launch_h_update_batch(const FieldArgs *args, const int *start, int n, int total, hipStream_t s);
void launch_e_update_batch(const FieldArgs *args, const int *start, int n, int total, hipStream_t s);
void launch_push_deposit_batch(const PartArgs *args, const int *start, int n, int total, int mode,
                               hipStream_t s);
void launch_probe_batch(const ProbeArgs *args, int n, hipStream_t s);

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
