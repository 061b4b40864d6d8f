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
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int PBLOCK = 256;  // particle kernels

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
    int per[3];
    float S;
    float *E[3];
    const float *Hin[3];
    float *Hout[3];
    float *Havg[3];  // H kernel: (Hin + Hout)/2 written inside the particle box, or null
    PmlAxis pml[3];
    // Drude polarization current on the metal bounding box [lo, hi)
    int mlo[3], mhi[3];
    float *Jp[3];
    const float2 *coef;  // (cbt, d) per box cell
    // bunch current: read and cleared inside the particle box (+ margin)
    float *Jb[3];
    const int *pbox;     // device [6]: lo x,y,z, hi x,y,z (cells, inclusive)
    int margin;
    int *nan_flag;
};

struct PartArgs {
    int n;
    float *x, *y, *z, *ux, *uy, *uz;
    int nx, ny, nz;
    int per[3];
    const float *E[3];
    const float *B[3];  // (Ht^{n-1/2} + Ht^{n+1/2}) / 2, valid inside the particle box
    float *Jb[3];
    float S;   // c dt / dx
    float ah;  // q dt / (2 m c), per V/m
    float qd;  // -q w / (eps0 dx^2), V/m
    unsigned long long *pushes;  // one counter per wavefront: [gridDim * PBLOCK / 64]
};

struct SortArgs {
    int n;
    int nx, ny, nz;
    int ncell;
    const float *src[6];
    float *dst[6];
    const int *id_src;
    int *id_dst;
    int *key;
    int *rank;
    int *counts;  // [ncell + 1]
    int *box;     // [6] bounding box of live cells, written by the count kernel
};

struct ProbeArgs {
    int nprobe, nfreq;
    const int *pidx;      // linear Ez index per probe
    const double *omega;  // rad/s
    double *fre, *fim;
    float *series;        // [series_len * nprobe] or null
    long long series_len;
    long long step;       // index n of the E^n just computed
    double dt;
    const float *Ez;
    int *nan_flag;
};

// A particle is live when every coordinate is finite and inside [0, n) (cell
// units); a lost particle stores x = -1.  Every kernel indexes the grid from
// a position only after this test, so non-finite values never become indices.
__device__ __forceinline__ bool live_pos(float x, float y, float z, int nx, int ny, int nz)
{
    return x >= 0.f && x < (float)nx && y >= 0.f && y < (float)ny && z >= 0.f && z < (float)nz;
}

// launchers (stream-ordered, no synchronisation)
void launch_h_update(const FieldArgs &a, hipStream_t s);
void launch_e_update(const FieldArgs &a, hipStream_t s);
void launch_push_deposit(const PartArgs &a, int mode, hipStream_t s);
void launch_probe(const ProbeArgs &a, hipStream_t s);
void launch_fill_i32(int *p, int v, long long n, hipStream_t s);
void launch_sort(const SortArgs &a, int *scan_tmp, int scan_tmp_len, hipStream_t s);
int scan_tmp_size(int n);

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
