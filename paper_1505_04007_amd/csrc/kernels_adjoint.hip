// Reverse-time adjoint of the linear field step on gfx950: the transpose of
// the H update, the Drude current recursion (Eq. 6) and the E update (Eq. 8)
// with their CPML memories, the bunch current held fixed.  It carries the
// derivative of the probe spectral power back through time and accumulates,
// in FP64, its derivative with respect to each metal cell's Drude
// coefficients cbt and d.
//
// The forward E update adds S (H(m) - H(m - e_a)) terms (CPML-stretched in
// the slabs); its transpose sends the edge's adjoint weight to the two faces
// it read.  Both transposes are written as gathers (one thread per cell, no
// atomics), in two kernels per step:
//   face kernel: Ha += sum over the edges that read the face of their
//                weights; then the face's own CPML adjoint for the H update
//                (the weights of its slab differences into DH).
//   edge kernel: the Drude transpose and gradient accumulation, Ea += sum
//                over the faces that read the edge; then the seed of the
//                probe objective and the edge's CPML adjoint for the next
//                (earlier) step (weights into DE).
// Outside the slabs a weight is +-S times the adjoint value itself and is
// recomputed where it is gathered; inside, it depends on the adjoint CPML
// memory and is read from DE / DH, written by the previous kernel.
#include "pic_internal.hpp"

namespace pic {

__device__ __forceinline__ bool adj_tile_cell(const AdjArgs &a, int t, int &i, int &j, int &k)
{
    const int bx = t % a.gx, by = (t / a.gx) % a.gy;
    k = t / (a.gx * a.gy);
    i = bx * FX + threadIdx.x;
    j = by * FY + threadIdx.y;
    return i < a.nx && j < a.ny && k < a.nz;
}

template <int AX>
__device__ __forceinline__ bool in_slab(const AdjArgs &a, int i, int j, int k)
{
    const PmlAxis &P = a.pml[AX];
    const int p = AX == 0 ? i : AX == 1 ? j : k;
    const int n = AX == 0 ? a.nx : AX == 1 ? a.ny : a.nz;
    return P.on && (p < P.npml || p >= n - P.npml);
}

template <int AX>
__device__ __forceinline__ int slab_sid(const AdjArgs &a, int i, int j, int k)
{
    const int np = a.pml[AX].npml;
    if (AX == 0) return slab_p(i, a.nx, np) + 2 * np * (j + a.ny * k);
    if (AX == 1) return i + a.nx * (slab_p(j, a.ny, np) + 2 * np * k);
    return i + a.nx * (j + a.ny * slab_p(k, a.nz, np));
}

// E component C is never written on the stored lower PEC wall planes across it.
template <int C>
__device__ __forceinline__ bool e_masked(const AdjArgs &a, int i, int j, int k)
{
    const bool wx = !a.per[0] && i == 0, wy = !a.per[1] && j == 0, wz = !a.per[2] && k == 0;
    return C == 0 ? (wy || wz) : C == 1 ? (wx || wz) : (wx || wy);
}

// A weight in two halves, so that a thread issues every load it needs before
// it uses any (a slab value loaded and used weight by weight would be one
// round trip to memory each): load() reads the weight's CPML value where the
// weight is one, use() gives the weight.
struct Weight {
    bool zero, slab;
    float v;
};

// Adjoint weight of the H difference along AX taken by the update of E
// component C (sign SGN in that update, CPML memory slot Q) at edge (i,j,k):
// 0 where the edge is never written, the stored slab weight inside the slab,
// else +-S times the edge's adjoint value.
template <int C, int AX, int Q>
__device__ __forceinline__ Weight e_weight_load(const AdjArgs &a, int i, int j, int k)
{
    Weight w;
    w.zero = e_masked<C>(a, i, j, k);
    w.slab = !w.zero && in_slab<AX>(a, i, j, k);
    w.v = 0.f;
    if (w.slab) w.v = a.DE[AX][Q][slab_sid<AX>(a, i, j, k)];
    return w;
}

// Adjoint weight of the E difference along AX taken by an H update (sign SGN,
// slot Q) at face (i,j,k).
template <int AX, int Q>
__device__ __forceinline__ Weight h_weight_load(const AdjArgs &a, int i, int j, int k)
{
    Weight w;
    w.zero = false;
    w.slab = in_slab<AX>(a, i, j, k);
    w.v = 0.f;
    if (w.slab) w.v = a.DH[AX][Q][slab_sid<AX>(a, i, j, k)];
    return w;
}

template <int SGN>
__device__ __forceinline__ float weight(const AdjArgs &a, const Weight &w, float bar)
{
    if (w.zero) return 0.f;
    if (w.slab) return w.v;
    return (SGN > 0 ? a.S : -a.S) * bar;
}

// Transpose of  psi' = b psi + c d,  d_eff = d / kappa + psi'  given the
// adjoint t of d_eff: the memory's adjoint moves back one step and the
// adjoint of the raw difference d is stored.
__device__ __forceinline__ void pml_adj(float *__restrict__ psib, float *__restrict__ D, int sid, float b,
                                        float c, float ik, float t)
{
    const float tot = psib[sid] + t;
    psib[sid] = b * tot;
    D[sid] = t * ik + c * tot;
}

template <int AX, int Q>
__device__ __forceinline__ void e_prep(const AdjArgs &a, float t, int i, int j, int k)
{
    const int p = AX == 0 ? i : AX == 1 ? j : k;
    const PmlAxis &P = a.pml[AX];
    pml_adj(a.psiEa[AX][Q], a.DE[AX][Q], slab_sid<AX>(a, i, j, k), P.bE[p], P.cE[p], P.kE[p], t);
}

template <int AX, int Q>
__device__ __forceinline__ void h_prep(const AdjArgs &a, float t, int i, int j, int k)
{
    const int p = AX == 0 ? i : AX == 1 ? j : k;
    const PmlAxis &P = a.pml[AX];
    pml_adj(a.psiHa[AX][Q], a.DH[AX][Q], slab_sid<AX>(a, i, j, k), P.bH[p], P.cH[p], P.kH[p], t);
}

// Forward E update, per edge (differences H(m) - H(m - e_a)):
//   Ex += S dHz/dy [y,0] - S dHy/dz [z,0]
//   Ey += S dHx/dz [z,1] - S dHz/dx [x,0]
//   Ez += S dHy/dx [x,1] - S dHx/dy [y,1]
// so face m of Hx is read with + by the Ey edge at m and the Ez edge at m
// (through their weights) and with - by the Ey edge at m + z and the Ez edge
// at m + y; likewise for Hy and Hz.
__global__ __launch_bounds__(FX *FY) void k_adj_face(AdjArgs a)
{
    int i, j, k;
    if (!adj_tile_cell(a, xcd_tile(), i, j, k)) return;
    const int id = i + a.nx * (j + a.ny * k);
    bool okx, oky, okz;
    const int ox = nb_off(i, 1, a.nx, a.per[0], 1, okx);
    const int oy = nb_off(j, 1, a.ny, a.per[1], a.nx, oky);
    const int oz = nb_off(k, 1, a.nz, a.per[2], a.nx * a.ny, okz);
    const int ip = i + 1 < a.nx ? i + 1 : 0;
    const int jp = j + 1 < a.ny ? j + 1 : 0;
    const int kp = k + 1 < a.nz ? k + 1 : 0;
    const float *__restrict__ Ex = a.Ea[0];
    const float *__restrict__ Ey = a.Ea[1];
    const float *__restrict__ Ez = a.Ea[2];
    const float ex = Ex[id], ey = Ey[id], ez = Ez[id];
    const float eyx = Ey[id + ox], ezx = Ez[id + ox];
    const float exy = Ex[id + oy], ezy = Ez[id + oy];
    const float exz = Ex[id + oz], eyz = Ey[id + oz];
    const float hx0 = a.Ha[0][id], hy0 = a.Ha[1][id], hz0 = a.Ha[2][id];
    // (ip, jp, kp are valid cells whether or not the neighbour takes part)
    const Weight wx0 = e_weight_load<1, 2, 1>(a, i, j, k), wx1 = e_weight_load<2, 1, 1>(a, i, j, k);
    const Weight wx2 = e_weight_load<1, 2, 1>(a, i, j, kp), wx3 = e_weight_load<2, 1, 1>(a, i, jp, k);
    const Weight wy0 = e_weight_load<0, 2, 0>(a, i, j, k), wy1 = e_weight_load<2, 0, 1>(a, i, j, k);
    const Weight wy2 = e_weight_load<0, 2, 0>(a, i, j, kp), wy3 = e_weight_load<2, 0, 1>(a, ip, j, k);
    const Weight wz0 = e_weight_load<0, 1, 0>(a, i, j, k), wz1 = e_weight_load<1, 0, 0>(a, i, j, k);
    const Weight wz2 = e_weight_load<0, 1, 0>(a, i, jp, k), wz3 = e_weight_load<1, 0, 0>(a, ip, j, k);

    float gx = weight<+1>(a, wx0, ey) + weight<-1>(a, wx1, ez);
    if (okz) gx -= weight<+1>(a, wx2, eyz);
    if (oky) gx -= weight<-1>(a, wx3, ezy);
    float gy = weight<-1>(a, wy0, ex) + weight<+1>(a, wy1, ez);
    if (okz) gy -= weight<-1>(a, wy2, exz);
    if (okx) gy -= weight<+1>(a, wy3, ezx);
    float gz = weight<+1>(a, wz0, ex) + weight<-1>(a, wz1, ey);
    if (oky) gz -= weight<+1>(a, wz2, exy);
    if (okx) gz -= weight<-1>(a, wz3, eyx);

    const float hx = hx0 + gx;
    const float hy = hy0 + gy;
    const float hz = hz0 + gz;
    a.Ha[0][id] = hx;
    a.Ha[1][id] = hy;
    a.Ha[2][id] = hz;

    // Forward H update (differences E(m + e_a) - E(m)):
    //   Hx -= S dEz/dy [y,0] - S dEy/dz [z,0]
    //   Hy -= S dEx/dz [z,1] - S dEz/dx [x,0]
    //   Hz -= S dEy/dx [x,1] - S dEx/dy [y,1]
    const float S = a.S;
    if (in_slab<0>(a, i, j, k)) {
        h_prep<0, 0>(a, S * hy, i, j, k);
        h_prep<0, 1>(a, -S * hz, i, j, k);
    }
    if (in_slab<1>(a, i, j, k)) {
        h_prep<1, 0>(a, -S * hx, i, j, k);
        h_prep<1, 1>(a, S * hz, i, j, k);
    }
    if (in_slab<2>(a, i, j, k)) {
        h_prep<2, 0>(a, S * hx, i, j, k);
        h_prep<2, 1>(a, -S * hy, i, j, k);
    }
}

__global__ __launch_bounds__(FX *FY) void k_adj_edge(AdjArgs a)
{
    int i, j, k;
    if (!adj_tile_cell(a, xcd_tile(), i, j, k)) return;
    const int id = i + a.nx * (j + a.ny * k);
    const bool mx = e_masked<0>(a, i, j, k), my = e_masked<1>(a, i, j, k), mz = e_masked<2>(a, i, j, k);
    const float ex1 = a.Ea[0][id], ey1 = a.Ea[1][id], ez1 = a.Ea[2][id];
    float ex = ex1, ey = ey1, ez = ez1;
    if (a.mode & 1) {
        bool okx, oky, okz;
        const int ox = nb_off(i, -1, a.nx, a.per[0], 1, okx);
        const int oy = nb_off(j, -1, a.ny, a.per[1], a.nx, oky);
        const int oz = nb_off(k, -1, a.nz, a.per[2], a.nx * a.ny, okz);
        const int im = i > 0 ? i - 1 : a.nx - 1;
        const int jm = j > 0 ? j - 1 : a.ny - 1;
        const int km = k > 0 ? k - 1 : a.nz - 1;
        const float *__restrict__ Hx = a.Ha[0];
        const float *__restrict__ Hy = a.Ha[1];
        const float *__restrict__ Hz = a.Ha[2];
        const float hx = Hx[id], hy = Hy[id], hz = Hz[id];
        const float hyx = Hy[id + ox], hzx = Hz[id + ox];
        const float hxy = Hx[id + oy], hzy = Hz[id + oy];
        const float hxz = Hx[id + oz], hyz = Hy[id + oz];
        // (im, jm, km are valid cells whether or not the neighbour takes part)
        const Weight vx0 = h_weight_load<2, 1>(a, i, j, k), vx1 = h_weight_load<1, 1>(a, i, j, k);
        const Weight vx2 = h_weight_load<2, 1>(a, i, j, km), vx3 = h_weight_load<1, 1>(a, i, jm, k);
        const Weight vy0 = h_weight_load<2, 0>(a, i, j, k), vy1 = h_weight_load<0, 1>(a, i, j, k);
        const Weight vy2 = h_weight_load<2, 0>(a, i, j, km), vy3 = h_weight_load<0, 1>(a, im, j, k);
        const Weight vz0 = h_weight_load<1, 0>(a, i, j, k), vz1 = h_weight_load<0, 0>(a, i, j, k);
        const Weight vz2 = h_weight_load<1, 0>(a, i, jm, k), vz3 = h_weight_load<0, 0>(a, im, j, k);
        // each face m reads E(m + e_a) with + and E(m) with -
        ex -= weight<-1>(a, vx0, hy) + weight<+1>(a, vx1, hz);
        if (okz) ex += weight<-1>(a, vx2, hyz);
        if (oky) ex += weight<+1>(a, vx3, hzy);
        ey -= weight<+1>(a, vy0, hx) + weight<-1>(a, vy1, hz);
        if (okz) ey += weight<+1>(a, vy2, hxz);
        if (okx) ey += weight<-1>(a, vy3, hzx);
        ez -= weight<-1>(a, vz0, hx) + weight<+1>(a, vz1, hy);
        if (oky) ez += weight<-1>(a, vz2, hxy);
        if (okx) ez += weight<+1>(a, vz3, hyx);

        if (i >= a.mlo[0] && i < a.mhi[0] && j >= a.mlo[1] && j < a.mhi[1] && k >= a.mlo[2] &&
            k < a.mhi[2]) {
            // Jt' = Jt + cbt E - d Jt, and E' takes - Jt': the adjoint of Jt'
            // is Ja - Ea' (E' written) and flows to E^n (cbt) and Jt (1 - d)
            const int wx = a.mhi[0] - a.mlo[0], wy = a.mhi[1] - a.mlo[1];
            const int nb = wx * wy * (a.mhi[2] - a.mlo[2]);
            const int bi = (i - a.mlo[0]) + wx * ((j - a.mlo[1]) + wy * (k - a.mlo[2]));
            const float2 cd = a.coef[bi];
            const float tx = a.Ja[0][bi] - (mx ? 0.f : ex1);
            const float ty = a.Ja[1][bi] - (my ? 0.f : ey1);
            const float tz = a.Ja[2][bi] - (mz ? 0.f : ez1);
            const float *__restrict__ T = a.traj;
            const double sE = (double)tx * T[bi] + (double)ty * T[nb + bi] + (double)tz * T[2 * nb + bi];
            const double sJ = (double)tx * T[3 * nb + bi] + (double)ty * T[4 * nb + bi] +
                              (double)tz * T[5 * nb + bi];
            a.gcb[bi] += sE;
            a.gd[bi] -= sJ;
            a.Ja[0][bi] = tx - cd.y * tx;
            a.Ja[1][bi] = ty - cd.y * ty;
            a.Ja[2][bi] = tz - cd.y * tz;
            ex += cd.x * tx;
            ey += cd.x * ty;
            ez += cd.x * tz;
        }
    }
    if (a.mode & 2) {
        if (a.seed)
            for (int p = 0; p < a.nprobe; ++p)
                if (a.pidx[p] == id) ez += a.seed[p];
        // CPML adjoint of the E update this adjoint value now enters
        const float S = a.S;
        if (!mx) {
            if (in_slab<1>(a, i, j, k)) e_prep<1, 0>(a, S * ex, i, j, k);
            if (in_slab<2>(a, i, j, k)) e_prep<2, 0>(a, -S * ex, i, j, k);
        }
        if (!my) {
            if (in_slab<2>(a, i, j, k)) e_prep<2, 1>(a, S * ey, i, j, k);
            if (in_slab<0>(a, i, j, k)) e_prep<0, 0>(a, -S * ey, i, j, k);
        }
        if (!mz) {
            if (in_slab<0>(a, i, j, k)) e_prep<0, 1>(a, S * ez, i, j, k);
            if (in_slab<1>(a, i, j, k)) e_prep<1, 1>(a, -S * ez, i, j, k);
        }
    }
    a.Ea[0][id] = ex;
    a.Ea[1][id] = ey;
    a.Ea[2][id] = ez;
}

__global__ void k_box_copy(BoxCopyArgs a)
{
    const long long nb = (long long)a.w[0] * a.w[1] * a.w[2];
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long t = t0; t < 3 * nb; t += st) {
        const int c = (int)(t / nb);
        const long long b = t - c * nb;
        const int bi = (int)(b % a.w[0]);
        const int bj = (int)((b / a.w[0]) % a.w[1]);
        const int bk = (int)(b / ((long long)a.w[0] * a.w[1]));
        const long long g = (long long)(a.lo[0] + bi) +
                            (long long)a.nx * ((long long)(a.lo[1] + bj) + (long long)a.ny * (a.lo[2] + bk));
        if (a.to_grid)
            a.grid[c][g] = a.packed[t];
        else
            a.packed[t] = a.grid[c][g];
    }
}

void launch_adj_face(const AdjArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_face, dim3(field_tiles(a.nx, a.ny, a.nz)), dim3(FX, FY), 0, s, a);
}

void launch_adj_edge(const AdjArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_edge, dim3(field_tiles(a.nx, a.ny, a.nz)), dim3(FX, FY), 0, s, a);
}

void launch_box_copy(const BoxCopyArgs &a, hipStream_t s)
{
    const long long n = 3LL * a.w[0] * a.w[1] * a.w[2];
    if (n <= 0) return;
    long long nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_box_copy, dim3((unsigned)nb), dim3(256), 0, s, a);
}

}  // namespace pic
