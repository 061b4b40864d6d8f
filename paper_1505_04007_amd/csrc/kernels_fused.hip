// One-pass field sweep for gfx950: the E update of step n (Drude and bunch
// currents fused, Eqs. 6 and 8) and the H update of step n + 1 in one pass
// over the grid.  E^n and H^{n+1/2} are read from HBM once and E^{n+1} and
// H^{n+3/2} written once: 48 B/cell of field traffic, where the separate H
// and E launches move 72.
//
// A workgroup spans the whole x extent (one wavefront per 64 cells), holds
// FUSED_ROWS rows of y per lane and marches FUSED_PLANES planes of z.  In
// plane k it computes E^{n+1}(k) for its rows and for one row above them (a
// halo: that row belongs to the next block, which computes it again as its
// own), then H^{n+3/2}(k - 1) from the new E of planes k - 1 and k.  The +x
// neighbour of the new E comes from the next lane (DPP), or for a
// wavefront's last lane from the next wavefront's first lane through LDS
// (triple-buffered, one barrier per plane); +y from the next row in
// registers; +z from the next plane, and the plane past the chunk is
// computed again the same way.  Recomputing a neighbour's E takes its old E,
// J_pol and E-side CPML memories, so those are read from one block and
// written to another (the host swaps them after the sweep); the bunch
// current is only read (a small kernel clears the particle box afterwards).
// The y and z memberships (CPML slabs, metal box, particle box) are uniform
// across a wavefront, the x ones are per lane.  Per cell the arithmetic is
// that of the separate update kernels, so the fields agree bitwise.
#include "pic_internal.hpp"

namespace pic {

namespace {

constexpr int R = FUSED_ROWS;
constexpr int MAX_WAVES = 16;  // nx <= 1024

// psi' = b psi + c d, d' = d / kappa + psi' (the separate kernels' recursion)
__device__ __forceinline__ float cpml_step(float p, float d, float b, float c, float ik, float &out)
{
    const float s = b * p + c * d;
    out = s;
    return d * ik + s;
}

// CPML coefficients of one position along an axis: E-type (b, c, 1/kappa),
// H-type (b, c, 1/kappa).
struct Coef6 {
    float bE, cE, kE, bH, cH, kH;
};

__device__ __forceinline__ Coef6 coef6(const float *tab, int n, int q)
{
    const gp<const float> t = G(tab);
    return Coef6{t[q], t[n + q], t[2 * n + q], t[3 * n + q], t[4 * n + q], t[5 * n + q]};
}

// Row or plane of the sweep: its grid index after wrapping and its role.
enum { ZERO = 0, OWN = 1, HALO = 2 };
struct Line {
    int q;     // grid index (wrapped on a periodic axis)
    int mode;  // OWN: this block's; HALO: a neighbour block's, computed again; ZERO: outside the grid
};

__device__ __forceinline__ Line line_at(int q, bool owned, int n, int per)
{
    if (q < n) return Line{q, owned ? OWN : HALO};
    if (q == n && per) return Line{0, HALO};
    return Line{0, ZERO};
}

// Inclusive [lo, hi] of the particle box widened by m along an axis (the
// whole axis when periodic).
__device__ __forceinline__ void box_axis(const int *pbox, int d, int n, int per, int m, int &lo, int &hi)
{
    if (per) {
        lo = 0;
        hi = n - 1;
    } else {
        const gp<const int> b = G(pbox);
        lo = b[d] - m;
        hi = b[3 + d] + m;
    }
}

__device__ __forceinline__ float dpp_next(float v)
{
    // wave_shl:1: lane l receives lane l + 1 (lane 63 receives 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

}  // namespace

__global__ __launch_bounds__(1024) void k_fused(FusedArgs a)
{
    __shared__ float xe[3][MAX_WAVES][R][2];  // lane 0's new (Ey, Ez) of each wavefront and row
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int i = threadIdx.x;
    const bool xin = i < a.nx;
    const int ic = xin ? i : a.nx - 1;  // inactive lanes load a valid cell and store nothing
    const int u = xcd_tile();
    const int j0 = (u % a.gy) * R, k0 = (u / a.gy) * FUSED_PLANES;
    const int nplanes = min(FUSED_PLANES, a.nz - k0);
    const int nx = a.nx, ny = a.ny, nz = a.nz, N = a.N;
    const float S = a.S;
    const gp<const float> __restrict__ Ein = G(a.Ein);
    const gp<const float> __restrict__ Hin = G(a.Hin);
    const gp<float> __restrict__ Eout = G(a.Eout);
    const gp<float> __restrict__ Hout = G(a.Hout);

    // particle box: J_b of this step, and the time-centred H the next step's
    // push gathers (one step of drift and a possible re-sort later)
    const gp<const DevState> st = G(a.st);
    const int since = st->since_sort;
    const bool hasbox = a.pbox != nullptr;
    const int mj = box_margin(since, S);
    const int mh = mj + (int)ceilf(S) + 1;
    int jlo[3] = {0, 0, 0}, jhi[3] = {-1, -1, -1}, hlo[3] = {0, 0, 0}, hhi[3] = {-1, -1, -1};
    if (hasbox) {
        const int n3[3] = {nx, ny, nz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            box_axis(a.pbox, d, n3[d], a.per[d], mj, jlo[d], jhi[d]);
            box_axis(a.pbox, d, n3[d], a.per[d], mh, hlo[d], hhi[d]);
        }
    }
    const bool jb_x = a.Jb && ic >= jlo[0] && ic <= jhi[0];
    const bool hv_x = a.Havg && ic >= hlo[0] && ic <= hhi[0];

    // per-lane x data
    bool okxm;
    const int oxm = nb_off(ic, -1, nx, a.per[0], 1, okxm);
    const bool wall_x = !a.per[0] && ic == 0;
    const bool sx = a.pon[0] && (ic < a.npml[0] || ic >= nx - a.npml[0]);
    Coef6 cx{};
    if (sx) cx = coef6(a.tab[0], nx, ic);
    const int pxs = slab_p(ic, nx, a.npml[0]);
    const bool mx = ic >= a.mlo[0] && ic < a.mhi[0];
    const int mwx = a.mhi[0] - a.mlo[0], mwy = a.mhi[1] - a.mlo[1];

    // rows 0 .. R (R: the halo row)
    Line row[R + 1];
#pragma unroll
    for (int r = 0; r <= R; ++r) row[r] = line_at(j0 + r, r < R, ny, a.per[1]);

    // H^{n+1/2} of the previous plane, rows 0 .. R (its x, y components feed
    // the new E's z derivatives; all three the H update of that plane)
    float hp[R + 1][3];
    // new E of the previous plane, rows 0 .. R
    float ep[R + 1][3];
    {
        bool ok;
        const int kq = k0 - 1 >= 0 ? k0 - 1 : (a.per[2] ? nz - 1 : 0);
        ok = k0 - 1 >= 0 || a.per[2];
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int id = ic + nx * (row[r].q + ny * kq);
            const bool v = ok && row[r].mode != ZERO;
            hp[r][0] = v ? Hin[id] : 0.f;
            hp[r][1] = v ? Hin[N + id] : 0.f;
            hp[r][2] = 0.f;
            ep[r][0] = ep[r][1] = ep[r][2] = 0.f;
        }
    }

    for (int t = 0; t <= nplanes; ++t) {
        const Line pl = line_at(k0 + t, t < nplanes, nz, a.per[2]);
        const int k = pl.q;
        // ---- E^{n+1} of plane k, rows 0 .. R ----
        float hc[R + 1][3], ec[R + 1][3];
        const bool sz = a.pon[2] && (k < a.npml[2] || k >= nz - a.npml[2]);
        Coef6 cz{};
        if (sz && pl.mode != ZERO) cz = coef6(a.tab[2], nz, k);
        const int pzs = slab_p(k, nz, a.npml[2]);
        const bool mz = k >= a.mlo[2] && k < a.mhi[2];
        const bool jb_z = k >= jlo[2] && k <= jhi[2];
        const bool wall_z = !a.per[2] && k == 0;
        // every main load of the plane first, branch-free (a row or plane
        // outside the grid reads a valid cell and is zeroed), so the
        // wavefront waits for memory once per plane
        float hxm, hzm;  // H of row -1, the -y neighbour of row 0
        {
            const bool ok = pl.mode != ZERO && (j0 > 0 || a.per[1]);
            const int jm = j0 > 0 ? j0 - 1 : ny - 1;
            const int id = ic + nx * (jm + ny * k);
            hxm = Hin[id];
            hzm = Hin[2 * N + id];
            hxm = ok ? hxm : 0.f;
            hzm = ok ? hzm : 0.f;
        }
        float ld[R + 1][8];
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int id = ic + nx * (row[r].q + ny * k);
            ld[r][0] = Hin[id];
            ld[r][1] = Hin[N + id];
            ld[r][2] = Hin[2 * N + id];
            ld[r][3] = Hin[N + id + oxm];
            ld[r][4] = Hin[2 * N + id + oxm];
            ld[r][5] = Ein[id];
            ld[r][6] = Ein[N + id];
            ld[r][7] = Ein[2 * N + id];
        }
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int j = row[r].q;
            const bool live = pl.mode != ZERO && row[r].mode != ZERO;
            const int id = ic + nx * (j + ny * k);
            const float hx = live ? ld[r][0] : 0.f, hy = live ? ld[r][1] : 0.f, hz = live ? ld[r][2] : 0.f;
            float hyx = live ? ld[r][3] : 0.f, hzx = live ? ld[r][4] : 0.f;
            const float ex = live ? ld[r][5] : 0.f, ey = live ? ld[r][6] : 0.f, ez = live ? ld[r][7] : 0.f;
            hc[r][0] = hx;
            hc[r][1] = hy;
            hc[r][2] = hz;
            if (!live) {
                ec[r][0] = ec[r][1] = ec[r][2] = 0.f;
                continue;
            }
            const bool own = pl.mode == OWN && row[r].mode == OWN && xin;
            hyx = okxm ? hyx : 0.f;
            hzx = okxm ? hzx : 0.f;
            const float hxy = r == 0 ? hxm : hc[r - 1][0];
            const float hzy = r == 0 ? hzm : hc[r - 1][2];
            const float hxz = hp[r][0], hyz = hp[r][1];
            float dyHz = hz - hzy, dzHy = hy - hyz;
            float dzHx = hx - hxz, dxHz = hz - hzx;
            float dxHy = hy - hyx, dyHx = hx - hxy;
            // CPML memories: read from the in block, written to the out block for owned cells
            if (sx) {
                const int sid = pxs + 2 * a.npml[0] * (j + ny * k);
                const gp<const float> pi_ = G(a.psiEin[0]);
                float o0, o1;
                dxHz = cpml_step(pi_[sid], dxHz, cx.bE, cx.cE, cx.kE, o0);
                dxHy = cpml_step(pi_[a.slab[0] + sid], dxHy, cx.bE, cx.cE, cx.kE, o1);
                if (own) {
                    G(a.psiEout[0])[sid] = o0;
                    G(a.psiEout[0])[a.slab[0] + sid] = o1;
                }
            }
            const bool sy = a.pon[1] && (j < a.npml[1] || j >= ny - a.npml[1]);
            if (sy) {
                const Coef6 cy = coef6(a.tab[1], ny, j);
                const int sid = ic + nx * (slab_p(j, ny, a.npml[1]) + 2 * a.npml[1] * k);
                const gp<const float> pi_ = G(a.psiEin[1]);
                float o0, o1;
                dyHz = cpml_step(pi_[sid], dyHz, cy.bE, cy.cE, cy.kE, o0);
                dyHx = cpml_step(pi_[a.slab[1] + sid], dyHx, cy.bE, cy.cE, cy.kE, o1);
                if (own) {
                    G(a.psiEout[1])[sid] = o0;
                    G(a.psiEout[1])[a.slab[1] + sid] = o1;
                }
            }
            if (sz) {
                const int sid = ic + nx * (j + ny * pzs);
                const gp<const float> pi_ = G(a.psiEin[2]);
                float o0, o1;
                dzHy = cpml_step(pi_[sid], dzHy, cz.bE, cz.cE, cz.kE, o0);
                dzHx = cpml_step(pi_[a.slab[2] + sid], dzHx, cz.bE, cz.cE, cz.kE, o1);
                if (own) {
                    G(a.psiEout[2])[sid] = o0;
                    G(a.psiEout[2])[a.slab[2] + sid] = o1;
                }
            }
            float nex = ex + S * (dyHz - dzHy);
            float ney = ey + S * (dzHx - dxHz);
            float nez = ez + S * (dxHy - dyHx);
            if (mx && mz && j >= a.mlo[1] && j < a.mhi[1]) {
                const int bi = (ic - a.mlo[0]) + mwx * ((j - a.mlo[1]) + mwy * (k - a.mlo[2]));
                const fvec2 cd = *(gp<const fvec2>)G(a.coef + bi);
                const gp<const float> Jin = G(a.Jpin);
                float jx = Jin[bi], jy = Jin[a.nbox + bi], jz = Jin[2 * a.nbox + bi];
                jx += cd.x * ex - cd.y * jx;
                jy += cd.x * ey - cd.y * jy;
                jz += cd.x * ez - cd.y * jz;
                if (own) {
                    const gp<float> Jo = G(a.Jpout);
                    Jo[bi] = jx;
                    Jo[a.nbox + bi] = jy;
                    Jo[2 * a.nbox + bi] = jz;
                }
                nex -= jx;
                ney -= jy;
                nez -= jz;
            }
            if (jb_x && jb_z && j >= jlo[1] && j <= jhi[1]) {
                const gp<const float> Jb = G(a.Jb);
                nex -= Jb[id];
                ney -= Jb[N + id];
                nez -= Jb[2 * N + id];
            }
            if (own && !(isfinite(nex) && isfinite(ney) && isfinite(nez)))
                __hip_atomic_fetch_or(G(a.nan_flag), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // tangential E on a wall is never written: it keeps its old value
            const bool wy = !a.per[1] && j == 0;
            if (wy || wall_z) nex = ex;
            if (wall_x || wall_z) ney = ey;
            if (wall_x || wy) nez = ez;
            if (own) {
                if (!(wy || wall_z)) __builtin_nontemporal_store(nex, Eout + id);
                if (!(wall_x || wall_z)) __builtin_nontemporal_store(ney, Eout + N + id);
                if (!(wall_x || wy)) __builtin_nontemporal_store(nez, Eout + 2 * N + id);
            }
            ec[r][0] = nex;
            ec[r][1] = ney;
            ec[r][2] = nez;
        }
        // publish lane 0's new (Ey, Ez) for the previous wavefront's last lane
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xe[t % 3][w][r][0] = ec[r][1];
                xe[t % 3][w][r][1] = ec[r][2];
            }
        }
        __syncthreads();
        // ---- H^{n+3/2} of the previous plane, owned rows ----
        if (t >= 1) {
            const int kh = k0 + t - 1;
            const bool szh = a.pon[2] && (kh < a.npml[2] || kh >= nz - a.npml[2]);
            Coef6 czh{};
            if (szh) czh = coef6(a.tab[2], nz, kh);
            const int pzh = slab_p(kh, nz, a.npml[2]);
            const bool hv_z = kh >= hlo[2] && kh <= hhi[2];
            const int b = (t - 1) % 3;
            const int wn = (w + 1 < nwave) ? w + 1 : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // the x neighbours come from the other lanes: every lane takes part
                float eyx = dpp_next(ep[r][1]), ezx = dpp_next(ep[r][2]);
                if (row[r].mode != OWN) continue;
                if (ic == nx - 1) {
                    eyx = a.per[0] ? xe[b][0][r][0] : 0.f;
                    ezx = a.per[0] ? xe[b][0][r][1] : 0.f;
                } else if (lane == 63) {
                    eyx = xe[b][wn][r][0];
                    ezx = xe[b][wn][r][1];
                }
                const int j = row[r].q;
                const int id = ic + nx * (j + ny * kh);
                const float ex = ep[r][0], ey = ep[r][1], ez = ep[r][2];
                const float hx = hp[r][0], hy = hp[r][1], hz = hp[r][2];
                const float exy = ep[r + 1][0], ezy = ep[r + 1][2];
                const float exz = ec[r][0], eyz = ec[r][1];
                float dyEz = ezy - ez, dzEy = eyz - ey;
                float dzEx = exz - ex, dxEz = ezx - ez;
                float dxEy = eyx - ey, dyEx = exy - ex;
                if (sx) {
                    const int sid = pxs + 2 * a.npml[0] * (j + ny * kh);
                    const gp<float> ps = G(a.psiH[0]);
                    float o0, o1;
                    dxEz = cpml_step(ps[sid], dxEz, cx.bH, cx.cH, cx.kH, o0);
                    dxEy = cpml_step(ps[a.slab[0] + sid], dxEy, cx.bH, cx.cH, cx.kH, o1);
                    if (xin) {
                        ps[sid] = o0;
                        ps[a.slab[0] + sid] = o1;
                    }
                }
                const bool sy = a.pon[1] && (j < a.npml[1] || j >= ny - a.npml[1]);
                if (sy) {
                    const Coef6 cy = coef6(a.tab[1], ny, j);
                    const int sid = ic + nx * (slab_p(j, ny, a.npml[1]) + 2 * a.npml[1] * kh);
                    const gp<float> ps = G(a.psiH[1]);
                    float o0, o1;
                    dyEz = cpml_step(ps[sid], dyEz, cy.bH, cy.cH, cy.kH, o0);
                    dyEx = cpml_step(ps[a.slab[1] + sid], dyEx, cy.bH, cy.cH, cy.kH, o1);
                    if (xin) {
                        ps[sid] = o0;
                        ps[a.slab[1] + sid] = o1;
                    }
                }
                if (szh) {
                    const int sid = ic + nx * (j + ny * pzh);
                    const gp<float> ps = G(a.psiH[2]);
                    float o0, o1;
                    dzEy = cpml_step(ps[sid], dzEy, czh.bH, czh.cH, czh.kH, o0);
                    dzEx = cpml_step(ps[a.slab[2] + sid], dzEx, czh.bH, czh.cH, czh.kH, o1);
                    if (xin) {
                        ps[sid] = o0;
                        ps[a.slab[2] + sid] = o1;
                    }
                }
                const float nhx = hx - S * (dyEz - dzEy);
                const float nhy = hy - S * (dzEx - dxEz);
                const float nhz = hz - S * (dxEy - dyEx);
                if (xin) {
                    __builtin_nontemporal_store(nhx, Hout + id);
                    __builtin_nontemporal_store(nhy, Hout + N + id);
                    __builtin_nontemporal_store(nhz, Hout + 2 * N + id);
                    if (hv_x && hv_z && j >= hlo[1] && j <= hhi[1]) {
                        const gp<float> Ha = G(a.Havg);
                        Ha[id] = 0.5f * (hx + nhx);
                        Ha[N + id] = 0.5f * (hy + nhy);
                        Ha[2 * N + id] = 0.5f * (hz + nhz);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r <= R; ++r) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                hp[r][d] = hc[r][d];
                ep[r][d] = ec[r][d];
            }
        }
    }
}

// Clear the bunch current on the particle box (+ margin) the E update read.
__global__ __launch_bounds__(256) void k_jb_clear(float *Jb, int N, int nx, int ny, int nz, int px, int py, int pz,
                                                  const int *pbox, float S, const DevState *st)
{
    const int m = box_margin(G(st)->since_sort, S);
    const int n3[3] = {nx, ny, nz}, per[3] = {px, py, pz};
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        box_axis(pbox, d, n3[d], per[d], m, lo[d], hi[d]);
        lo[d] = max(lo[d], 0);
        hi[d] = min(hi[d], n3[d] - 1);
    }
    if (hi[0] < lo[0] || hi[1] < lo[1] || hi[2] < lo[2]) return;
    const long long ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1;
    const long long total = ex * ey * (hi[2] - lo[2] + 1);
    const gp<float> J = G(Jb);
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = lo[0] + (int)(q % ex), j = lo[1] + (int)((q / ex) % ey), k = lo[2] + (int)(q / (ex * ey));
        const int id = i + nx * (j + ny * k);
        J[id] = 0.f;
        J[N + id] = 0.f;
        J[2 * N + id] = 0.f;
    }
}

void launch_fused(const FusedArgs &a, hipStream_t s)
{
    const int waves = (a.nx + 63) / 64;
    const int blocks = a.gy * ((a.nz + FUSED_PLANES - 1) / FUSED_PLANES);
    hipLaunchKernelGGL(k_fused, dim3(blocks), dim3(64 * waves), 0, s, a);
}

void launch_jb_clear(float *Jb, int N, int nx, int ny, int nz, const int *per, const int *pbox, float S,
                     const DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_jb_clear, dim3(512), dim3(256), 0, s, Jb, N, nx, ny, nz, per[0], per[1], per[2], pbox, S,
                       st);
}

}  // namespace pic
