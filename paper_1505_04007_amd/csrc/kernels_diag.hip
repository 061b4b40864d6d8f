// Probe DFT (FP64 accumulators) and FP64 check-path diagnostics.
#include "pic_internal.hpp"

namespace pic {

// F_p(w_m) += dt Ez_p^n exp(-i w_m n dt) for the E^n just computed (Sec. IV,
// Figs. 6-7: Ez at the film surface and its spectrum).  The phase is
// evaluated directly in FP64 each step.
// The last kernel of a step: after sampling, it advances the step clock
// (H parity, steps since the sort, step number) for the next step.
__device__ __forceinline__ void probe_body(const ProbeArgs &a)
{
    const int t = threadIdx.x;
    const gp<DevState> st = G(a.st);
    const gp<const float> Ez = G(a.Ez);
    const gp<const int> pidx = G(a.pidx);
    const long long n1 = st->step + 1;  // E^{n+1} was just computed
    const double tn = (double)n1 * a.dt;
    for (int q = t; q < a.nprobe * a.nfreq; q += blockDim.x) {
        const int p = q / a.nfreq, f = q - p * a.nfreq;
        const double ez = (double)Ez[pidx[p]];
        double sn, cs;
        sincos(G(a.omega)[f] * tn, &sn, &cs);
        G(a.fre)[q] += a.dt * ez * cs;
        G(a.fim)[q] -= a.dt * ez * sn;
    }
    if (a.series && t < a.nprobe && n1 - 1 < a.series_len)
        G(a.series)[(n1 - 1) * a.nprobe + t] = Ez[pidx[t]];
    if (a.gser && t < a.nprobe && n1 > a.g0 && n1 <= a.g0 + a.gn)
        G(a.gser)[(n1 - a.g0 - 1) * a.nprobe + t] = (double)Ez[pidx[t]];
    __syncthreads();  // every thread has read the clock before it moves
    if (t == 0) {
        st->parity ^= 1;
        st->since_sort += 1;
        st->step = n1;
    }
}
__global__ void k_probe(ProbeArgs a) { probe_body(a); }

__global__ void k_probe_batch(const ProbeArgs *args) { probe_body(args[blockIdx.x]); }

void launch_probe(const ProbeArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_probe, dim3(1), dim3(256), 0, s, a);
}

void launch_probe_batch(const ProbeArgs *args, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_probe_batch, dim3(n), dim3(256), 0, s, args);
}

// Node-centred cloud-in-cell charge density in FP64 (nodes (nx+1)(ny+1)(nz+1)).
__global__ void k_rho(DiagArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.np) return;
    if (!live_pos(a.x[p], a.y[p], a.z[p], a.nx, a.ny, a.nz)) return;
    const double X[3] = {(double)a.x[p], (double)a.y[p], (double)a.z[p]};
    int i0[3];
    double fr[3];
    const int n[3] = {a.nx, a.ny, a.nz};
    for (int d = 0; d < 3; ++d) {
        const double f = floor(X[d]);
        i0[d] = (int)f;
        fr[d] = X[d] - f;
    }
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) {
                int id[3] = {i0[0] + q, i0[1] + b, i0[2] + c};
                bool skip = false;
                for (int d = 0; d < 3; ++d) {
                    if (a.per[d]) id[d] = id[d] >= n[d] ? id[d] - n[d] : id[d];
                    if (id[d] < 0 || id[d] > n[d]) skip = true;
                }
                if (skip) continue;
                const double w = (q ? fr[0] : 1 - fr[0]) * (b ? fr[1] : 1 - fr[1]) * (c ? fr[2] : 1 - fr[2]);
                atomicAdd(&a.rho[id[0] + (a.nx + 1) * (id[1] + (a.ny + 1) * id[2])], a.qw_over_vol * w);
            }
}

void launch_rho(const DiagArgs &a, hipStream_t s)
{
    if (a.np <= 0) return;
    hipLaunchKernelGGL(k_rho, dim3((unsigned)(((long long)a.np + 255) / 256)), dim3(256), 0, s, a);
}

__device__ __forceinline__ double warp_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double warp_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void atomic_max_pos(double *addr, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

// acc layout: [0] sum (E^2 + Ht^2), [1] count, [2..4] sum x, [5..7] sum x^2,
// [8..10] sum u, [11] max |G|, [12] max |rho0|, [13] checked nodes
__global__ void k_diag_fields(DiagArgs a)
{
    const long long n = (long long)a.nx * a.ny * a.nz;
    double s = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            const double e = a.E[c][q], h = a.H[c][q];
            s += e * e + h * h;
        }
    }
    s = warp_sum(s);
    if ((threadIdx.x & 63) == 0) atomicAdd(&a.acc[0], s);
}

// Grid-stride sums over the live particles, reduced per wavefront, then per
// workgroup in LDS, then one FP64 atomic per workgroup and quantity (a fixed
// grid keeps the same-address atomics to a few thousand).
__global__ __launch_bounds__(256) void k_diag_particles(DiagArgs a)
{
    __shared__ double part[4][10];
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < a.np;
         p += (long long)gridDim.x * blockDim.x) {
        if (!live_pos(a.x[p], a.y[p], a.z[p], a.nx, a.ny, a.nz)) continue;
        const double X[3] = {a.x[p], a.y[p], a.z[p]};
        const double U[3] = {a.ux[p], a.uy[p], a.uz[p]};
        v[0] += 1.0;
        for (int d = 0; d < 3; ++d) {
            v[1 + d] += X[d];
            v[4 + d] += X[d] * X[d];
            v[7 + d] += U[d];
        }
    }
    const int w = threadIdx.x >> 6;
    for (int q = 0; q < 10; ++q) {
        const double t = warp_sum(v[q]);
        if ((threadIdx.x & 63) == 0) part[w][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const double t = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                         part[3][threadIdx.x];
        if (t != 0.0) atomicAdd(&a.acc[1 + threadIdx.x], t);
    }
}

// G = eps0 div E - rho at interior nodes away from CPML layers and the metal
// box, compared with its initial value -rho0 (E^0 = 0).
__global__ void k_diag_gauss(DiagArgs a)
{
    const long long n = (long long)(a.nx + 1) * (a.ny + 1) * (a.nz + 1);
    double gm = 0.0, rm = 0.0, cnt = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % (a.nx + 1));
        const int j = (int)((q / (a.nx + 1)) % (a.ny + 1));
        const int k = (int)(q / ((long long)(a.nx + 1) * (a.ny + 1)));
        if (a.rho0) rm = fmax(rm, fabs(a.rho0[q]));
        const int id[3] = {i, j, k};
        const int nn[3] = {a.nx, a.ny, a.nz};
        bool ok = true;
        for (int d = 0; d < 3; ++d)
            if (id[d] < 1 + a.npml[d] || id[d] > nn[d] - 1 - a.npml[d]) ok = false;
        if (ok && i >= a.mlo[0] - 1 && i <= a.mhi[0] && j >= a.mlo[1] - 1 && j <= a.mhi[1] &&
            k >= a.mlo[2] - 1 && k <= a.mhi[2])
            ok = false;
        if (!ok) continue;
        const long long c0 = i + (long long)a.nx * (j + (long long)a.ny * k);
        const double dE = ((double)a.E[0][c0] - (double)a.E[0][c0 - 1]) +
                          ((double)a.E[1][c0] - (double)a.E[1][c0 - a.nx]) +
                          ((double)a.E[2][c0] - (double)a.E[2][c0 - (long long)a.nx * a.ny]);
        double g = a.eps0_over_dx * dE - a.rho[q];
        if (a.rho0) g += a.rho0[q];
        gm = fmax(gm, fabs(g));
        cnt += 1.0;
    }
    gm = warp_max(gm);
    rm = warp_max(rm);
    cnt = warp_sum(cnt);
    if ((threadIdx.x & 63) == 0) {
        atomic_max_pos(&a.acc[11], gm);
        atomic_max_pos(&a.acc[12], rm);
        atomicAdd(&a.acc[13], cnt);
    }
}

void launch_diag_reduce(const DiagArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_fields, dim3(1024), dim3(256), 0, s, a);
    if (a.np > 0) hipLaunchKernelGGL(k_diag_particles, dim3(1024), dim3(256), 0, s, a);
    if (a.rho) hipLaunchKernelGGL(k_diag_gauss, dim3(1024), dim3(256), 0, s, a);
}

}  // namespace pic
