// Yee curl updates for gfx950: H update (vacuum form) and the fused Drude
// polarization-current + E update.
//
// One thread per cell, one workgroup per (x, y) tile of one z plane (64 x 4
// cells by default; the autotuner picks another shape from a fixed table per
// grid), x fastest so a wavefront reads contiguous rows.  Each
// cell reads its own three old values and the three neighbour values its
// curl needs (+x/+y/+z for H, -x/-y/-z for E); the neighbours are the own
// values of adjacent lanes, rows and planes and are served by L1/L2, so the
// HBM traffic stays close to one read and one write of every array.
// Neighbour loads are branch-free (index clamped to the cell itself, value
// selected to 0 or wrapped) so every load of a thread issues back to back.
// Measured on MI355X this barrier-free form streams faster than an
// LDS-staged z-march of the same stencil (no block-wide stall per plane).
//
// Workgroups are remapped so that the tiles one XCD executes form a
// contiguous range in (x, y, z): neighbours in y and z then share that XCD's
// L2.  The batched entry points run the same per-cell code for many
// simulations in one launch: the remapped work-unit index is looked up in a
// table of (simulation, group of consecutive tiles).
#include "pic_internal.hpp"

namespace pic {

__device__ __forceinline__ int lin(const FieldArgs &a, int i, int j, int k)
{
    return i + a.nx * (j + a.ny * k);
}

// Values a cell reads or writes once, that no neighbour touches in the same
// launch, are streamed past the caches so they keep the stencil's shared
// neighbour data.
__device__ __forceinline__ float ld_once(const float *p) { return __builtin_nontemporal_load(G(p)); }
__device__ __forceinline__ void st_once(float *p, float v) { __builtin_nontemporal_store(v, G(p)); }

// One CPML axis of one cell: its slab index, coefficients and two memories,
// loaded with the cell's field values (all issued before any is used, so a
// slab cell waits for memory once, not twice); update() then applies the
// recursion psi' = b psi + c d, d' = d / kappa + psi' and stores psi'.
struct SlabMem {
    bool in;
    int sid;
    float b, c, ik, p0, p1;
};

__device__ __forceinline__ SlabMem slab_load(float *const *psi, const float *tb, const float *tc, const float *tk,
                                             int pos, bool in, int sid)
{
    SlabMem m{in, sid, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (in) {
        m.b = G(tb)[pos];
        m.c = G(tc)[pos];
        m.ik = G(tk)[pos];
        m.p0 = G(psi[0])[sid];
        m.p1 = G(psi[1])[sid];
    }
    return m;
}

__device__ __forceinline__ float cpml_update(float *__restrict__ psi, const SlabMem &m, float p, float d)
{
    const float s = m.b * p + m.c * d;
    G(psi)[m.sid] = s;
    return d * m.ik + s;
}

// The three slab memberships of cell (i, j, k) with their memories (E = 1:
// the E update's tables and memories, else the H update's).
template <int E>
__device__ __forceinline__ void slab_all(const FieldArgs &a, int i, int j, int k, SlabMem &mx, SlabMem &my,
                                         SlabMem &mz)
{
    const PmlAxis &X = a.pml[0], &Y = a.pml[1], &Z = a.pml[2];
    mx = slab_load(E ? X.psiE : X.psiH, E ? X.bE : X.bH, E ? X.cE : X.cH, E ? X.kE : X.kH, i,
                   X.on && (i < X.npml || i >= a.nx - X.npml), slab_p(i, a.nx, X.npml) + 2 * X.npml * (j + a.ny * k));
    my = slab_load(E ? Y.psiE : Y.psiH, E ? Y.bE : Y.bH, E ? Y.cE : Y.cH, E ? Y.kE : Y.kH, j,
                   Y.on && (j < Y.npml || j >= a.ny - Y.npml), i + a.nx * (slab_p(j, a.ny, Y.npml) + 2 * Y.npml * k));
    mz = slab_load(E ? Z.psiE : Z.psiH, E ? Z.bE : Z.bH, E ? Z.cE : Z.cH, E ? Z.kE : Z.kH, k,
                   Z.on && (k < Z.npml || k >= a.nz - Z.npml), i + a.nx * (j + a.ny * slab_p(k, a.nz, Z.npml)));
}


// Inside the live-particle cell box of the last sort widened by the margin
// (every cell a particle can gather from or deposit to this step); a
// periodic axis counts whole because deposits and gathers wrap there.
__device__ __forceinline__ bool in_particle_box(const FieldArgs &a, int margin, int i, int j, int k)
{
    const int n3[3] = {a.nx, a.ny, a.nz};
    const int id3[3] = {i, j, k};
    const gp<const int> box = G(a.pbox);
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int lo = a.per[d] ? 0 : box[d] - margin;
        const int hi = a.per[d] ? n3[d] - 1 : box[3 + d] + margin;
        in = in && id3[d] >= lo && id3[d] <= hi;
    }
    return in;
}

// H^{n+1/2} = H^{n-1/2} - S curl E^n  (vacuum form for every cell).
__device__ __forceinline__ void h_cell(const FieldArgs &a, int par, int margin, int i, int j, int k)
{
    const int id = lin(a, i, j, k);
    const int sx = 1, sy = a.nx, sz = a.nx * a.ny;
    bool okx, oky, okz;
    const int ox = nb_off(i, 1, a.nx, a.per[0], sx, okx);
    const int oy = nb_off(j, 1, a.ny, a.per[1], sy, oky);
    const int oz = nb_off(k, 1, a.nz, a.per[2], sz, okz);
    const gp<const float> __restrict__ Ex = G(a.E[0]);
    const gp<const float> __restrict__ Ey = G(a.E[1]);
    const gp<const float> __restrict__ Ez = G(a.E[2]);
    const float *__restrict__ H0 = par ? a.H[1][0] : a.H[0][0];
    const float *__restrict__ H1 = par ? a.H[1][1] : a.H[0][1];
    const float *__restrict__ H2 = par ? a.H[1][2] : a.H[0][2];
    float *__restrict__ O0 = par ? a.H[0][0] : a.H[1][0];
    float *__restrict__ O1 = par ? a.H[0][1] : a.H[1][1];
    float *__restrict__ O2 = par ? a.H[0][2] : a.H[1][2];
    const float ex = Ex[id], ey = Ey[id], ez = Ez[id];
    float eyx = Ey[id + ox], ezx = Ez[id + ox];
    float exy = Ex[id + oy], ezy = Ez[id + oy];
    float exz = Ex[id + oz], eyz = Ey[id + oz];
    const float hx = ld_once(H0 + id), hy = ld_once(H1 + id), hz = ld_once(H2 + id);
    SlabMem mx, my, mz;
    slab_all<0>(a, i, j, k, mx, my, mz);
    // tested with the cell's loads: after the first store its box loads
    // would be one more trip to memory
    const bool avg = a.Havg[0] && in_particle_box(a, margin, i, j, k);
    eyx = okx ? eyx : 0.f;
    ezx = okx ? ezx : 0.f;
    exy = oky ? exy : 0.f;
    ezy = oky ? ezy : 0.f;
    exz = okz ? exz : 0.f;
    eyz = okz ? eyz : 0.f;
    float dyEz = ezy - ez, dzEy = eyz - ey;
    float dzEx = exz - ex, dxEz = ezx - ez;
    float dxEy = eyx - ey, dyEx = exy - ex;
    if (mx.in) {
        dxEz = cpml_update(a.pml[0].psiH[0], mx, mx.p0, dxEz);
        dxEy = cpml_update(a.pml[0].psiH[1], mx, mx.p1, dxEy);
    }
    if (my.in) {
        dyEz = cpml_update(a.pml[1].psiH[0], my, my.p0, dyEz);
        dyEx = cpml_update(a.pml[1].psiH[1], my, my.p1, dyEx);
    }
    if (mz.in) {
        dzEy = cpml_update(a.pml[2].psiH[0], mz, mz.p0, dzEy);
        dzEx = cpml_update(a.pml[2].psiH[1], mz, mz.p1, dzEx);
    }
    const float S = a.S;
    const float nhx = hx - S * (dyEz - dzEy);
    const float nhy = hy - S * (dzEx - dxEz);
    const float nhz = hz - S * (dxEy - dyEx);
    st_once(O0 + id, nhx);
    st_once(O1 + id, nhy);
    st_once(O2 + id, nhz);
    if (avg) {
        // B^n of the push, (Ht^{n-1/2} + Ht^{n+1/2})/2, where particles can gather it
        G(a.Havg[0])[id] = 0.5f * (hx + nhx);
        G(a.Havg[1])[id] = 0.5f * (hy + nhy);
        G(a.Havg[2])[id] = 0.5f * (hz + nhz);
    }
}

// Fused step: J_pol^{n+1/2} = J_pol^{n-1/2} + cbt E^n - d J_pol^{n-1/2} on
// metal edges, then E^{n+1} = E^n + S curl H^{n+1/2} - J_pol^{n+1/2} -
// J_b^{n+1/2}; J_b is cleared after use.  Tangential E on PEC walls is
// never written.
__device__ __forceinline__ void e_cell(const FieldArgs &a, int par, int margin, int i, int j, int k)
{
    const int id = lin(a, i, j, k);
    const int sx = 1, sy = a.nx, sz = a.nx * a.ny;
    bool okx, oky, okz;
    const int ox = nb_off(i, -1, a.nx, a.per[0], sx, okx);
    const int oy = nb_off(j, -1, a.ny, a.per[1], sy, oky);
    const int oz = nb_off(k, -1, a.nz, a.per[2], sz, okz);
    // H^{n+1/2}: written by this step's H update into H[par ^ 1]
    const gp<const float> __restrict__ Hx = G(par ? a.H[0][0] : a.H[1][0]);
    const gp<const float> __restrict__ Hy = G(par ? a.H[0][1] : a.H[1][1]);
    const gp<const float> __restrict__ Hz = G(par ? a.H[0][2] : a.H[1][2]);
    const float hx = Hx[id], hy = Hy[id], hz = Hz[id];
    float hyx = Hy[id + ox], hzx = Hz[id + ox];
    float hxy = Hx[id + oy], hzy = Hz[id + oy];
    float hxz = Hx[id + oz], hyz = Hy[id + oz];
    const float ex = ld_once(a.E[0] + id), ey = ld_once(a.E[1] + id), ez = ld_once(a.E[2] + id);
    SlabMem mx, my, mz;
    slab_all<1>(a, i, j, k, mx, my, mz);
    hyx = okx ? hyx : 0.f;
    hzx = okx ? hzx : 0.f;
    hxy = oky ? hxy : 0.f;
    hzy = oky ? hzy : 0.f;
    hxz = okz ? hxz : 0.f;
    hyz = okz ? hyz : 0.f;
    float dyHz = hz - hzy, dzHy = hy - hyz;
    float dzHx = hx - hxz, dxHz = hz - hzx;
    float dxHy = hy - hyx, dyHx = hx - hxy;
    if (mx.in) {
        dxHz = cpml_update(a.pml[0].psiE[0], mx, mx.p0, dxHz);
        dxHy = cpml_update(a.pml[0].psiE[1], mx, mx.p1, dxHy);
    }
    if (my.in) {
        dyHz = cpml_update(a.pml[1].psiE[0], my, my.p0, dyHz);
        dyHx = cpml_update(a.pml[1].psiE[1], my, my.p1, dyHx);
    }
    if (mz.in) {
        dzHy = cpml_update(a.pml[2].psiE[0], mz, mz.p0, dzHy);
        dzHx = cpml_update(a.pml[2].psiE[1], mz, mz.p1, dzHx);
    }
    const float S = a.S;
    float nex = ex + S * (dyHz - dzHy);
    float ney = ey + S * (dzHx - dxHz);
    float nez = ez + S * (dxHy - dyHx);
    if (i >= a.mlo[0] && i < a.mhi[0] && j >= a.mlo[1] && j < a.mhi[1] && k >= a.mlo[2] &&
        k < a.mhi[2]) {
        const int wx = a.mhi[0] - a.mlo[0], wy = a.mhi[1] - a.mlo[1];
        const int bi = (i - a.mlo[0]) + wx * ((j - a.mlo[1]) + wy * (k - a.mlo[2]));
        const fvec2 cd = *(gp<const fvec2>)G(a.coef + bi);
        const gp<float> J0 = G(a.Jp[0]), J1 = G(a.Jp[1]), J2 = G(a.Jp[2]);
        float jx = J0[bi], jy = J1[bi], jz = J2[bi];
        if (a.snap) {
            // the reverse pass's snapshot: E^n and J_pol^{n-1/2} of this cell
            const int nb = wx * wy * (a.mhi[2] - a.mlo[2]);
            const gp<float> sn = G(a.snap);
            sn[bi] = ex;
            sn[nb + bi] = ey;
            sn[2 * nb + bi] = ez;
            sn[3 * nb + bi] = jx;
            sn[4 * nb + bi] = jy;
            sn[5 * nb + bi] = jz;
        }
        jx += cd.x * ex - cd.y * jx;
        jy += cd.x * ey - cd.y * jy;
        jz += cd.x * ez - cd.y * jz;
        J0[bi] = jx;
        J1[bi] = jy;
        J2[bi] = jz;
        nex -= jx;
        ney -= jy;
        nez -= jz;
    }
    if (a.pbox && in_particle_box(a, margin, i, j, k)) {
        if (a.Jq[0]) {
            // fixed-point bunch current (deterministic deposit), FP64 to V/m
            const gp<unsigned long long> q0 = G(a.Jq[0]), q1 = G(a.Jq[1]), q2 = G(a.Jq[2]);
            nex -= (float)((double)(long long)q0[id] * a.qinv);
            ney -= (float)((double)(long long)q1[id] * a.qinv);
            nez -= (float)((double)(long long)q2[id] * a.qinv);
            q0[id] = 0ull;
            q1[id] = 0ull;
            q2[id] = 0ull;
        } else {
            const gp<float> b0 = G(a.Jb[0]), b1 = G(a.Jb[1]), b2 = G(a.Jb[2]);
            nex -= b0[id];
            ney -= b1[id];
            nez -= b2[id];
            b0[id] = 0.f;
            b1[id] = 0.f;
            b2[id] = 0.f;
        }
    }
    const bool wx = !a.per[0] && i == 0, wy = !a.per[1] && j == 0, wz = !a.per[2] && k == 0;
    if (!(wy || wz)) st_once(a.E[0] + id, nex);
    if (!(wx || wz)) st_once(a.E[1] + id, ney);
    if (!(wx || wy)) st_once(a.E[2] + id, nez);
    if (!(isfinite(nex) && isfinite(ney) && isfinite(nez)))
        __hip_atomic_fetch_or(G(a.nan_flag), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decompose a tile index of one simulation into (i, j, k); false when the
// thread lies past the grid's x / y extent.
template <int TXW, int TYW, int ZO>
__device__ __forceinline__ bool tile_cell(const FieldArgs &a, int t, int &i, int &j, int &k)
{
    const int bx = t % a.gx;
    int by;
    if (ZO) {
        k = (t / a.gx) % a.nz;
        by = t / (a.gx * a.nz);
    } else {
        by = (t / a.gx) % a.gy;
        k = t / (a.gx * a.gy);
    }
    i = bx * TXW + threadIdx.x;
    j = by * TYW + threadIdx.y;
    return i < a.nx && j < a.ny && k < a.nz;
}

template <int TXW, int TYW, int ZO>
__global__ __launch_bounds__(TXW *TYW) void k_h_update(FieldArgs a)
{
    int i, j, k;
    if (!tile_cell<TXW, TYW, ZO>(a, xcd_tile(), i, j, k)) return;
    const gp<const DevState> st = G(a.st);
    h_cell(a, st->parity, box_margin(st->since_sort, a.S), i, j, k);
}

template <int TXW, int TYW, int ZO>
__global__ __launch_bounds__(TXW *TYW) void k_e_update(FieldArgs a)
{
    int i, j, k;
    if (!tile_cell<TXW, TYW, ZO>(a, xcd_tile_rev(), i, j, k)) return;
    const gp<const DevState> st = G(a.st);
    e_cell(a, st->parity, box_margin(st->since_sort, a.S), i, j, k);
}

// Work unit u of a batched launch belongs to simulation own[u] >> 24 as its
// own unit own[u] & 0xffffff (a table the host builds: one load per
// workgroup, whatever the number of simulations), which covers that
// simulation's tiles BATCH_TILES * unit onwards, x-neighbours first.
template <int TXW, int TYW, int ZO>
__global__ __launch_bounds__(TXW *TYW) void k_h_update_batch(const FieldArgs *__restrict__ args,
                                                             const int *__restrict__ own)
{
    const int o = own[xcd_tile()];
    const FieldArgs &a = args[o >> 24];
    const gp<const DevState> st = G(a.st);
    const int parity = st->parity, margin = box_margin(st->since_sort, a.S);
    const int t0 = (o & 0xffffff) * BATCH_TILES, nt = a.gx * a.gy * a.nz;
    for (int q = 0; q < BATCH_TILES && t0 + q < nt; ++q) {
        int i, j, k;
        if (tile_cell<TXW, TYW, ZO>(a, t0 + q, i, j, k)) h_cell(a, parity, margin, i, j, k);
    }
}

template <int TXW, int TYW, int ZO>
__global__ __launch_bounds__(TXW *TYW) void k_e_update_batch(const FieldArgs *__restrict__ args,
                                                             const int *__restrict__ own)
{
    const int o = own[xcd_tile_rev()];
    const FieldArgs &a = args[o >> 24];
    const gp<const DevState> st = G(a.st);
    const int parity = st->parity, margin = box_margin(st->since_sort, a.S);
    const int t0 = (o & 0xffffff) * BATCH_TILES, nt = a.gx * a.gy * a.nz;
    for (int q = 0; q < BATCH_TILES && t0 + q < nt; ++q) {
        int i, j, k;
        if (tile_cell<TXW, TYW, ZO>(a, t0 + q, i, j, k)) e_cell(a, parity, margin, i, j, k);
    }
}

// One launch of a tile-shape instantiation: the shape index selects the
// template arguments (the table in pic_internal.hpp).
template <template <int, int, int> class K, typename... Args>
void launch_shape(int shape, int blocks, hipStream_t s, Args... args)
{
    switch (shape) {
#define PIC_SHAPE(v)                                                                                          \
    case v:                                                                                                   \
        K<TILE_FX[v], TILE_FY[v], TILE_ZO[v]>::launch(blocks, s, args...);                                    \
        break;
        PIC_SHAPE(1) PIC_SHAPE(2) PIC_SHAPE(3) PIC_SHAPE(4) PIC_SHAPE(5) PIC_SHAPE(6) PIC_SHAPE(7)
        PIC_SHAPE(8) PIC_SHAPE(9) PIC_SHAPE(10) PIC_SHAPE(11) PIC_SHAPE(12) PIC_SHAPE(13) PIC_SHAPE(14)
        PIC_SHAPE(15)
#undef PIC_SHAPE
    default: K<TILE_FX[0], TILE_FY[0], TILE_ZO[0]>::launch(blocks, s, args...); break;
    }
}

template <int TXW, int TYW, int ZO>
struct HLaunch {
    static void launch(int blocks, hipStream_t s, FieldArgs a)
    {
        hipLaunchKernelGGL((k_h_update<TXW, TYW, ZO>), dim3(blocks), dim3(TXW, TYW), 0, s, a);
    }
};
template <int TXW, int TYW, int ZO>
struct ELaunch {
    static void launch(int blocks, hipStream_t s, FieldArgs a)
    {
        hipLaunchKernelGGL((k_e_update<TXW, TYW, ZO>), dim3(blocks), dim3(TXW, TYW), 0, s, a);
    }
};
template <int TXW, int TYW, int ZO>
struct HBatchLaunch {
    static void launch(int blocks, hipStream_t s, const FieldArgs *args, const int *own)
    {
        hipLaunchKernelGGL((k_h_update_batch<TXW, TYW, ZO>), dim3(blocks), dim3(TXW, TYW), 0, s, args, own);
    }
};
template <int TXW, int TYW, int ZO>
struct EBatchLaunch {
    static void launch(int blocks, hipStream_t s, const FieldArgs *args, const int *own)
    {
        hipLaunchKernelGGL((k_e_update_batch<TXW, TYW, ZO>), dim3(blocks), dim3(TXW, TYW), 0, s, args, own);
    }
};

void launch_h_update(const FieldArgs &a, hipStream_t s)
{
    launch_shape<HLaunch>(a.tile, field_tiles(a.nx, a.ny, a.nz, a.tile), s, a);
}

void launch_e_update(const FieldArgs &a, hipStream_t s)
{
    launch_shape<ELaunch>(a.tile, field_tiles(a.nx, a.ny, a.nz, a.tile), s, a);
}

void launch_h_update_batch(const FieldArgs *args, const int *own, int total, int shape, hipStream_t s)
{
    launch_shape<HBatchLaunch>(shape, total, s, args, own);
}

void launch_e_update_batch(const FieldArgs *args, const int *own, int total, int shape, hipStream_t s)
{
    launch_shape<EBatchLaunch>(shape, total, s, args, own);
}

}  // namespace pic
