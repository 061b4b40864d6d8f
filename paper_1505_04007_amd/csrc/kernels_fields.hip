// Yee curl updates for gfx950: H update (vacuum form) and the fused Drude
// polarization-current + E update.
//
// Tiling: a 64 x 8 workgroup covers an (x, y) tile, x fastest so one
// wavefront reads one 256-byte row, and marches DZ consecutive z planes.
// The current plane of the differentiated field is staged in LDS with a
// one-cell halo (+x/+y for the H update's forward differences, -x/-y for
// the E update's backward differences); the z neighbour is carried in
// registers from the previous plane.  Each cell's three old values are read
// once and its three new values written once.
#include "pic_internal.hpp"

namespace pic {

__device__ __forceinline__ int lin(const FieldArgs &a, int i, int j, int k)
{
    return i + a.nx * (j + a.ny * k);
}

// Value at (i, j, k) where an index may lie one tile past either end of its
// axis: wraps on a periodic axis, reads 0 beyond a PEC / CPML wall.
__device__ __forceinline__ float ldb(const float *__restrict__ f, const FieldArgs &a, int i, int j,
                                     int k)
{
    if (i >= a.nx) {
        if (!a.per[0] || i >= 2 * a.nx) return 0.f;
        i -= a.nx;
    } else if (i < 0) {
        if (!a.per[0]) return 0.f;
        i += a.nx;
    }
    if (j >= a.ny) {
        if (!a.per[1] || j >= 2 * a.ny) return 0.f;
        j -= a.ny;
    } else if (j < 0) {
        if (!a.per[1]) return 0.f;
        j += a.ny;
    }
    if (k >= a.nz) {
        if (!a.per[2] || k >= 2 * a.nz) return 0.f;
        k -= a.nz;
    } else if (k < 0) {
        if (!a.per[2]) return 0.f;
        k += a.nz;
    }
    return f[lin(a, i, j, k)];
}

// One CPML recursion psi = b psi + c d, returning d / kappa + psi.
__device__ __forceinline__ float cpml(float *__restrict__ psi, int sid, float b, float c, float ik,
                                      float d)
{
    const float s = b * psi[sid] + c * d;
    psi[sid] = s;
    return d * ik + s;
}

__device__ __forceinline__ int slab_p(int q, int n, int np) { return q < np ? q : q - (n - 2 * np); }

// H^{n+1/2} = H^{n-1/2} - S curl E^n  (vacuum form for every cell).
__global__ __launch_bounds__(TX *TY) void k_h_update(FieldArgs a)
{
    __shared__ float sEx[TY + 1][TX];
    __shared__ float sEy[TY][TX + 1];
    __shared__ float sEz[TY + 1][TX + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = blockIdx.x * TX + tx, j = blockIdx.y * TY + ty;
    const int k0 = blockIdx.z * DZ;
    const int k1 = min(k0 + DZ, a.nz);
    const bool own = i < a.nx && j < a.ny;
    const float S = a.S;
    const float *__restrict__ Ex = a.E[0];
    const float *__restrict__ Ey = a.E[1];
    const float *__restrict__ Ez = a.E[2];

    float ex = ldb(Ex, a, i, j, k0), ey = ldb(Ey, a, i, j, k0), ez = ldb(Ez, a, i, j, k0);
    for (int k = k0; k < k1; ++k) {
        sEx[ty][tx] = ex;
        sEy[ty][tx] = ey;
        sEz[ty][tx] = ez;
        if (tx == TX - 1) {
            sEy[ty][TX] = ldb(Ey, a, i + 1, j, k);
            sEz[ty][TX] = ldb(Ez, a, i + 1, j, k);
        }
        if (ty == TY - 1) {
            sEx[TY][tx] = ldb(Ex, a, i, j + 1, k);
            sEz[TY][tx] = ldb(Ez, a, i, j + 1, k);
        }
        const float exn = ldb(Ex, a, i, j, k + 1);
        const float eyn = ldb(Ey, a, i, j, k + 1);
        const float ezn = ldb(Ez, a, i, j, k + 1);
        const int id = own ? lin(a, i, j, k) : 0;
        float hx = 0.f, hy = 0.f, hz = 0.f;
        if (own) {
            hx = a.Hin[0][id];
            hy = a.Hin[1][id];
            hz = a.Hin[2][id];
        }
        __syncthreads();
        if (own) {
            float dyEz = sEz[ty + 1][tx] - ez;
            float dzEy = eyn - ey;
            float dzEx = exn - ex;
            float dxEz = sEz[ty][tx + 1] - ez;
            float dxEy = sEy[ty][tx + 1] - ey;
            float dyEx = sEx[ty + 1][tx] - ex;
            if (a.pml[0].on) {
                const PmlAxis &P = a.pml[0];
                if (i < P.npml || i >= a.nx - P.npml) {
                    const int sid = slab_p(i, a.nx, P.npml) + 2 * P.npml * (j + a.ny * k);
                    const float b = P.bH[i], c = P.cH[i], ik = P.kH[i];
                    dxEz = cpml(P.psiH[0], sid, b, c, ik, dxEz);
                    dxEy = cpml(P.psiH[1], sid, b, c, ik, dxEy);
                }
            }
            if (a.pml[1].on) {
                const PmlAxis &P = a.pml[1];
                if (j < P.npml || j >= a.ny - P.npml) {
                    const int sid = i + a.nx * (slab_p(j, a.ny, P.npml) + 2 * P.npml * k);
                    const float b = P.bH[j], c = P.cH[j], ik = P.kH[j];
                    dyEz = cpml(P.psiH[0], sid, b, c, ik, dyEz);
                    dyEx = cpml(P.psiH[1], sid, b, c, ik, dyEx);
                }
            }
            if (a.pml[2].on) {
                const PmlAxis &P = a.pml[2];
                if (k < P.npml || k >= a.nz - P.npml) {
                    const int sid = i + a.nx * (j + a.ny * slab_p(k, a.nz, P.npml));
                    const float b = P.bH[k], c = P.cH[k], ik = P.kH[k];
                    dzEy = cpml(P.psiH[0], sid, b, c, ik, dzEy);
                    dzEx = cpml(P.psiH[1], sid, b, c, ik, dzEx);
                }
            }
            a.Hout[0][id] = hx - S * (dyEz - dzEy);
            a.Hout[1][id] = hy - S * (dzEx - dxEz);
            a.Hout[2][id] = hz - S * (dxEy - dyEx);
        }
        __syncthreads();
        ex = exn;
        ey = eyn;
        ez = ezn;
    }
}

// Fused step: J_pol^{n+1/2} = J_pol^{n-1/2} + cbt E^n - d J_pol^{n-1/2} on
// metal edges, then E^{n+1} = E^n + S curl H^{n+1/2} - J_pol^{n+1/2} -
// J_b^{n+1/2}; J_b is cleared after use.  Tangential E on PEC walls is
// never written.
__global__ __launch_bounds__(TX *TY) void k_e_update(FieldArgs a)
{
    __shared__ float sHx[TY + 1][TX];
    __shared__ float sHy[TY][TX + 1];
    __shared__ float sHz[TY + 1][TX + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = blockIdx.x * TX + tx, j = blockIdx.y * TY + ty;
    const int k0 = blockIdx.z * DZ;
    const int k1 = min(k0 + DZ, a.nz);
    const bool own = i < a.nx && j < a.ny;
    const float S = a.S;
    const float *__restrict__ Hx = a.Hin[0];
    const float *__restrict__ Hy = a.Hin[1];
    const float *__restrict__ Hz = a.Hin[2];

    int blo[3] = {0, 0, 0}, bhi[3] = {-1, -1, -1};
    if (a.pbox) {
        const int nn[3] = {a.nx, a.ny, a.nz};
        for (int d = 0; d < 3; ++d) {
            // deposits wrap on a periodic axis: clear the whole axis there
            blo[d] = a.per[d] ? 0 : a.pbox[d] - a.margin;
            bhi[d] = a.per[d] ? nn[d] - 1 : a.pbox[3 + d] + a.margin;
        }
    }
    const bool jb_ij = a.pbox && i >= blo[0] && i <= bhi[0] && j >= blo[1] && j <= bhi[1];
    const bool m_ij = i >= a.mlo[0] && i < a.mhi[0] && j >= a.mlo[1] && j < a.mhi[1];
    const bool wx = !a.per[0] && i == 0, wy = !a.per[1] && j == 0;

    float hxm = ldb(Hx, a, i, j, k0 - 1), hym = ldb(Hy, a, i, j, k0 - 1);
    for (int k = k0; k < k1; ++k) {
        const float hx = ldb(Hx, a, i, j, k);
        const float hy = ldb(Hy, a, i, j, k);
        const float hz = ldb(Hz, a, i, j, k);
        sHx[ty + 1][tx] = hx;
        sHy[ty][tx + 1] = hy;
        sHz[ty + 1][tx + 1] = hz;
        if (tx == 0) {
            sHy[ty][0] = ldb(Hy, a, i - 1, j, k);
            sHz[ty + 1][0] = ldb(Hz, a, i - 1, j, k);
        }
        if (ty == 0) {
            sHx[0][tx] = ldb(Hx, a, i, j - 1, k);
            sHz[0][tx + 1] = ldb(Hz, a, i, j - 1, k);
        }
        const int id = own ? lin(a, i, j, k) : 0;
        float ex = 0.f, ey = 0.f, ez = 0.f;
        if (own) {
            ex = a.E[0][id];
            ey = a.E[1][id];
            ez = a.E[2][id];
        }
        __syncthreads();
        if (own) {
            float dyHz = hz - sHz[ty][tx + 1];
            float dzHy = hy - hym;
            float dzHx = hx - hxm;
            float dxHz = hz - sHz[ty + 1][tx];
            float dxHy = hy - sHy[ty][tx];
            float dyHx = hx - sHx[ty][tx];
            if (a.pml[0].on) {
                const PmlAxis &P = a.pml[0];
                if (i < P.npml || i >= a.nx - P.npml) {
                    const int sid = slab_p(i, a.nx, P.npml) + 2 * P.npml * (j + a.ny * k);
                    const float b = P.bE[i], c = P.cE[i], ik = P.kE[i];
                    dxHz = cpml(P.psiE[0], sid, b, c, ik, dxHz);
                    dxHy = cpml(P.psiE[1], sid, b, c, ik, dxHy);
                }
            }
            if (a.pml[1].on) {
                const PmlAxis &P = a.pml[1];
                if (j < P.npml || j >= a.ny - P.npml) {
                    const int sid = i + a.nx * (slab_p(j, a.ny, P.npml) + 2 * P.npml * k);
                    const float b = P.bE[j], c = P.cE[j], ik = P.kE[j];
                    dyHz = cpml(P.psiE[0], sid, b, c, ik, dyHz);
                    dyHx = cpml(P.psiE[1], sid, b, c, ik, dyHx);
                }
            }
            if (a.pml[2].on) {
                const PmlAxis &P = a.pml[2];
                if (k < P.npml || k >= a.nz - P.npml) {
                    const int sid = i + a.nx * (j + a.ny * slab_p(k, a.nz, P.npml));
                    const float b = P.bE[k], c = P.cE[k], ik = P.kE[k];
                    dzHy = cpml(P.psiE[0], sid, b, c, ik, dzHy);
                    dzHx = cpml(P.psiE[1], sid, b, c, ik, dzHx);
                }
            }
            float nex = ex + S * (dyHz - dzHy);
            float ney = ey + S * (dzHx - dxHz);
            float nez = ez + S * (dxHy - dyHx);
            if (m_ij && k >= a.mlo[2] && k < a.mhi[2]) {
                const int wx_ = a.mhi[0] - a.mlo[0], wy_ = a.mhi[1] - a.mlo[1];
                const int bi = (i - a.mlo[0]) + wx_ * ((j - a.mlo[1]) + wy_ * (k - a.mlo[2]));
                const float2 cd = a.coef[bi];
                float jx = a.Jp[0][bi], jy = a.Jp[1][bi], jz = a.Jp[2][bi];
                jx += cd.x * ex - cd.y * jx;
                jy += cd.x * ey - cd.y * jy;
                jz += cd.x * ez - cd.y * jz;
                a.Jp[0][bi] = jx;
                a.Jp[1][bi] = jy;
                a.Jp[2][bi] = jz;
                nex -= jx;
                ney -= jy;
                nez -= jz;
            }
            if (jb_ij && k >= blo[2] && k <= bhi[2]) {
                nex -= a.Jb[0][id];
                ney -= a.Jb[1][id];
                nez -= a.Jb[2][id];
                a.Jb[0][id] = 0.f;
                a.Jb[1][id] = 0.f;
                a.Jb[2][id] = 0.f;
            }
            const bool wz = !a.per[2] && k == 0;
            if (!(wy || wz)) a.E[0][id] = nex;
            if (!(wx || wz)) a.E[1][id] = ney;
            if (!(wx || wy)) a.E[2][id] = nez;
            if (!(isfinite(nex) && isfinite(ney) && isfinite(nez))) atomicOr(a.nan_flag, 1);
        }
        __syncthreads();
        hxm = hx;
        hym = hy;
    }
}

static dim3 field_grid(const FieldArgs &a)
{
    return dim3((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + DZ - 1) / DZ);
}

void launch_h_update(const FieldArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_h_update, field_grid(a), dim3(TX, TY), 0, s, a);
}

void launch_e_update(const FieldArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_e_update, field_grid(a), dim3(TX, TY), 0, s, a);
}

}  // namespace pic
