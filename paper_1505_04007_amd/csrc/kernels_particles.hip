// Particle kernels for gfx950: staggered trilinear gather, relativistic
// Boris push, move, and charge-conserving (Esirkepov, first-order shape)
// current deposition; counting sort of the particles by cell.
//
// Deposit.  A move x0 -> x1 shorter than one cell touches at most three
// nodes per axis, [b, b+2] with b = min(floor x0, floor x1).  Its current is
// 18 Jx + 18 Jy + 18 Jz edge values on that window.  Particles are kept
// sorted by cell, so the lanes of a wavefront mostly share a window: lanes
// with equal windows are summed across the wavefront by recursive halving
// (64 slots -> one slot per lane after 6 exchange rounds of shrinking width),
// and each lane then issues at most one global float atomic.  Windows that
// are still unresolved after a few rounds fall back to per-lane atomics.
#include "pic_internal.hpp"

namespace pic {

// Index on a periodic axis (window indices reach n + 1, which is 2 periods
// away when n = 1).
__device__ __forceinline__ int wrapn(int i, int n)
{
    if (i >= 0 && i < n) return i;
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Fold a finite coordinate that moved less than one period back into [0, n).
__device__ __forceinline__ float fold(float v, int n)
{
    const float L = (float)n;
    if (v >= L) v -= L;
    if (v < 0.f) v += L;
    return v >= L ? 0.f : v;  // v + L may round up to L
}

// Stored value at integer lattice index; 0 outside the box on a wall axis.
__device__ __forceinline__ float fetch(const float *__restrict__ f, const PartArgs &a, int i, int j,
                                       int k)
{
    if (a.per[0]) i = wrapn(i, a.nx);
    else if (i < 0 || i >= a.nx) return 0.f;
    if (a.per[1]) j = wrapn(j, a.ny);
    else if (j < 0 || j >= a.ny) return 0.f;
    if (a.per[2]) k = wrapn(k, a.nz);
    else if (k < 0 || k >= a.nz) return 0.f;
    return f[i + a.nx * (j + a.ny * k)];
}

// Trilinear interpolation of one component whose lattice is shifted by half a
// cell along the axes flagged in (hx, hy, hz).  f2 (optional) is added
// corner by corner (the two time levels of H).
__device__ __forceinline__ float gather(const float *__restrict__ f, const float *__restrict__ f2,
                                        const PartArgs &a, float x, float y, float z, int hx, int hy,
                                        int hz)
{
    const float xs = hx ? x - 0.5f : x, ys = hy ? y - 0.5f : y, zs = hz ? z - 0.5f : z;
    const float fi = floorf(xs), fj = floorf(ys), fk = floorf(zs);
    const int i = (int)fi, j = (int)fj, k = (int)fk;
    const float wx1 = xs - fi, wy1 = ys - fj, wz1 = zs - fk;
    const float wx0 = 1.f - wx1, wy0 = 1.f - wy1, wz0 = 1.f - wz1;
    float v = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                float s = fetch(f, a, i + q, j + b, k + c);
                if (f2) s += fetch(f2, a, i + q, j + b, k + c);
                v += (q ? wx1 : wx0) * (b ? wy1 : wy0) * (c ? wz1 : wz0) * s;
            }
    return v;
}

// First-order shape on the 3-node window starting at node `base`.
__device__ __forceinline__ void shapes(float x0, float x1, int base, float S0[3], float dS[3])
{
    const float r0 = x0 - (float)base, r1 = x1 - (float)base;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float s0 = fmaxf(0.f, 1.f - fabsf(r0 - (float)m));
        const float s1 = fmaxf(0.f, 1.f - fabsf(r1 - (float)m));
        S0[m] = s0;
        dS[m] = s1 - s0;
    }
}

// Slot s (0..53) of the deposit window: component and offsets from the base node.
//   Jx: s = a*9 + b*3 + c        (edge a in 0..1, nodes b, c in 0..2)
//   Jy: s = 18 + a*6 + m*3 + c   (node a, edge m, node c)
//   Jz: s = 36 + a*6 + b*2 + m   (nodes a, b, edge m)
__device__ __forceinline__ void slot_geom(int s, int &comp, int &oi, int &oj, int &ok)
{
    if (s < 18) {
        comp = 0;
        oi = s / 9;
        oj = (s / 3) % 3;
        ok = s % 3;
    } else if (s < 36) {
        const int t = s - 18;
        comp = 1;
        oi = t / 6;
        oj = (t / 3) % 2;
        ok = t % 3;
    } else {
        const int t = s - 36;
        comp = 2;
        oi = t / 6;
        oj = (t / 2) % 3;
        ok = t % 2;
    }
}

// Current of slot s from the per-axis shapes (qd folded in by the caller).
struct Dep {
    float S0[3][3], dS[3][3];
};

__device__ __forceinline__ float slot_value(const Dep &d, int s)
{
    int comp, oi, oj, ok;
    slot_geom(s, comp, oi, oj, ok);
    // prefix of dS along the current's own axis, transverse weight of the
    // other two: S0 S0 + (dS S0 + S0 dS)/2 + dS dS/3
    const int ax = comp, a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
    int e, n1, n2;
    if (comp == 0) {
        e = oi;
        n1 = oj;
        n2 = ok;
    } else if (comp == 1) {
        e = oj;
        n1 = ok;  // a1 = z
        n2 = oi;  // a2 = x
    } else {
        e = ok;
        n1 = oi;  // a1 = x
        n2 = oj;  // a2 = y
    }
    const float pre = e == 0 ? d.dS[ax][0] : d.dS[ax][0] + d.dS[ax][1];
    const float s1 = d.S0[a1][n1], t1 = d.dS[a1][n1];
    const float s2 = d.S0[a2][n2], t2 = d.dS[a2][n2];
    return pre * (s1 * s2 + 0.5f * (t1 * s2 + s1 * t2) + (1.f / 3.f) * t1 * t2);
}

__device__ __forceinline__ float *slot_addr(const PartArgs &a, int s, int bx, int by, int bz)
{
    int comp, oi, oj, ok;
    slot_geom(s, comp, oi, oj, ok);
    int i = bx + oi, j = by + oj, k = bz + ok;
    if (a.per[0]) i = wrapn(i, a.nx);
    else if (i < 0 || i >= a.nx) return nullptr;
    if (a.per[1]) j = wrapn(j, a.ny);
    else if (j < 0 || j >= a.ny) return nullptr;
    if (a.per[2]) k = wrapn(k, a.nz);
    else if (k < 0 || k >= a.nz) return nullptr;
    return a.Jb[comp] + (i + a.nx * (j + a.ny * k));
}

template <int OFF>
__device__ __forceinline__ void halve(float *v, int lane)
{
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int e = 0; e < OFF; ++e) {
        const float send = up ? v[e] : v[e + OFF];
        const float keep = up ? v[e + OFF] : v[e];
        v[e] = keep + __shfl_xor(send, OFF, 64);
    }
}

// After the six rounds lane l holds the wavefront sum of slot l.
__device__ __forceinline__ float wave_reduce64(float *v, int lane)
{
    halve<32>(v, lane);
    halve<16>(v, lane);
    halve<8>(v, lane);
    halve<4>(v, lane);
    halve<2>(v, lane);
    halve<1>(v, lane);
    return v[0];
}

constexpr int MAX_ROUNDS = 4;

template <int MODE>
__global__ __launch_bounds__(PBLOCK) void k_push_deposit(PartArgs a)
{
    const int p = blockIdx.x * PBLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool dep = false;
    Dep d;
    int base[3] = {0, 0, 0};
    if (p < a.n) {
        const float x = a.x[p], y = a.y[p], z = a.z[p];
        if (live_pos(x, y, z, a.nx, a.ny, a.nz)) {
            float u0 = a.ux[p], u1 = a.uy[p], u2 = a.uz[p];
            // E^n and Ht^n = (Ht^{n-1/2} + Ht^{n+1/2})/2 at x^n
            const float e0 = gather(a.E[0], nullptr, a, x, y, z, 1, 0, 0);
            const float e1 = gather(a.E[1], nullptr, a, x, y, z, 0, 1, 0);
            const float e2 = gather(a.E[2], nullptr, a, x, y, z, 0, 0, 1);
            const float h0 = 0.5f * gather(a.Hold[0], a.Hnew[0], a, x, y, z, 0, 1, 1);
            const float h1 = 0.5f * gather(a.Hold[1], a.Hnew[1], a, x, y, z, 1, 0, 1);
            const float h2 = 0.5f * gather(a.Hold[2], a.Hnew[2], a, x, y, z, 1, 1, 0);
            // relativistic Boris: half kick, rotation, half kick (u in units of c)
            const float ah = a.ah;
            const float m0 = u0 + ah * e0, m1 = u1 + ah * e1, m2 = u2 + ah * e2;
            const float gi = rsqrtf(1.f + m0 * m0 + m1 * m1 + m2 * m2);
            const float t0 = ah * h0 * gi, t1 = ah * h1 * gi, t2 = ah * h2 * gi;
            const float f = 2.f / (1.f + t0 * t0 + t1 * t1 + t2 * t2);
            const float s0 = f * t0, s1 = f * t1, s2 = f * t2;
            const float p0 = m0 + (m1 * t2 - m2 * t1);
            const float p1 = m1 + (m2 * t0 - m0 * t2);
            const float p2 = m2 + (m0 * t1 - m1 * t0);
            u0 = m0 + (p1 * s2 - p2 * s1) + ah * e0;
            u1 = m1 + (p2 * s0 - p0 * s2) + ah * e1;
            u2 = m2 + (p0 * s1 - p1 * s0) + ah * e2;
            const float g = rsqrtf(1.f + u0 * u0 + u1 * u1 + u2 * u2);
            float x1 = x + a.S * u0 * g, y1 = y + a.S * u1 * g, z1 = z + a.S * u2 * g;
            // leaving through a wall, or a non-finite move, deactivates the particle
            const bool out = !(isfinite(x1) && isfinite(y1) && isfinite(z1)) ||
                             (!a.per[0] && !(x1 >= 0.f && x1 < (float)a.nx)) ||
                             (!a.per[1] && !(y1 >= 0.f && y1 < (float)a.ny)) ||
                             (!a.per[2] && !(z1 >= 0.f && z1 < (float)a.nz));
            a.ux[p] = u0;
            a.uy[p] = u1;
            a.uz[p] = u2;
            if (out) {
                a.x[p] = -1.f;  // left the box: deactivated, last move not deposited
            } else {
                const float X0[3] = {x, y, z}, X1[3] = {x1, y1, z1};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const int i0 = (int)floorf(X0[ax]), i1 = (int)floorf(X1[ax]);
                    base[ax] = min(i0, i1);
                    shapes(X0[ax], X1[ax], base[ax], d.S0[ax], d.dS[ax]);
                }
                dep = true;
                if (a.per[0]) x1 = fold(x1, a.nx);
                if (a.per[1]) y1 = fold(y1, a.ny);
                if (a.per[2]) z1 = fold(z1, a.nz);
                a.x[p] = x1;
                a.y[p] = y1;
                a.z[p] = z1;
            }
        }
    }
    const float qd = a.qd;
    const unsigned long long live = __ballot(dep);
    if (lane == 0 && live) atomicAdd(a.pushes, (unsigned long long)__popcll(live));
    if (MODE == 1) {
        if (dep) {
            for (int s = 0; s < 54; ++s) {
                const float v = qd * slot_value(d, s);
                if (v != 0.f) {
                    float *ad = slot_addr(a, s, base[0], base[1], base[2]);
                    if (ad) atomicAdd(ad, v);
                }
            }
        }
        return;
    }
    const int key = (base[0] + 1) + (a.nx + 2) * ((base[1] + 1) + (a.ny + 2) * (base[2] + 1));
    unsigned long long rem = live;
    int round = 0;
    while (rem && round < MAX_ROUNDS) {
        const int leader = __ffsll((long long)rem) - 1;
        const int k0 = __builtin_amdgcn_readlane(key, leader);
        const bool mine = ((rem >> lane) & 1ull) && key == k0;
        const unsigned long long m = __ballot(mine);
        float v[64];
#pragma unroll
        for (int s = 0; s < 54; ++s) v[s] = mine ? slot_value(d, s) : 0.f;
#pragma unroll
        for (int s = 54; s < 64; ++s) v[s] = 0.f;
        const float tot = wave_reduce64(v, lane);
        const int bx = __builtin_amdgcn_readlane(base[0], leader);
        const int by = __builtin_amdgcn_readlane(base[1], leader);
        const int bz = __builtin_amdgcn_readlane(base[2], leader);
        if (lane < 54 && tot != 0.f) {
            float *ad = slot_addr(a, lane, bx, by, bz);
            if (ad) atomicAdd(ad, qd * tot);
        }
        rem &= ~m;
        ++round;
    }
    if ((rem >> lane) & 1ull) {
        for (int s = 0; s < 54; ++s) {
            const float v = qd * slot_value(d, s);
            if (v != 0.f) {
                float *ad = slot_addr(a, s, base[0], base[1], base[2]);
                if (ad) atomicAdd(ad, v);
            }
        }
    }
}

void launch_push_deposit(const PartArgs &a, int mode, hipStream_t s)
{
    if (a.n <= 0) return;
    const int nb = (a.n + PBLOCK - 1) / PBLOCK;
    if (mode == 1) hipLaunchKernelGGL(k_push_deposit<1>, dim3(nb), dim3(PBLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_push_deposit<0>, dim3(nb), dim3(PBLOCK), 0, s, a);
}

// ---------------------------------------------------------------------------
// Counting sort by cell: count (with in-cell rank), exclusive scan, scatter.
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int *p, int v, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long q = t; q < n; q += st) p[q] = v;
}

void launch_fill_i32(int *p, int v, long long n, hipStream_t s)
{
    if (n <= 0) return;
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(256), 0, s, p, v, n);
}

__global__ __launch_bounds__(PBLOCK) void k_sort_count(SortArgs a)
{
    __shared__ int bb[6];
    if (threadIdx.x < 6) bb[threadIdx.x] = threadIdx.x < 3 ? INT_MAX : INT_MIN;
    __syncthreads();
    const int p = blockIdx.x * PBLOCK + threadIdx.x;
    if (p < a.n) {
        const float x = a.src[0][p], y = a.src[1][p], z = a.src[2][p];
        int key = a.ncell;
        if (live_pos(x, y, z, a.nx, a.ny, a.nz)) {
            const int i = min((int)x, a.nx - 1);
            const int j = min((int)y, a.ny - 1);
            const int k = min((int)z, a.nz - 1);
            key = i + a.nx * (j + a.ny * k);
            atomicMin(&bb[0], i);
            atomicMin(&bb[1], j);
            atomicMin(&bb[2], k);
            atomicMax(&bb[3], i);
            atomicMax(&bb[4], j);
            atomicMax(&bb[5], k);
        }
        a.key[p] = key;
        a.rank[p] = atomicAdd(&a.counts[key], 1);
    }
    __syncthreads();
    if (threadIdx.x < 3 && bb[threadIdx.x] != INT_MAX) atomicMin(&a.box[threadIdx.x], bb[threadIdx.x]);
    if (threadIdx.x >= 3 && threadIdx.x < 6 && bb[threadIdx.x] != INT_MIN)
        atomicMax(&a.box[threadIdx.x], bb[threadIdx.x]);
}

// Three-phase exclusive scan over SCAN_ITEMS * SCAN_THREADS elements per block.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sm, int &total)
{
    // Hillis-Steele in LDS over 256 thread totals
    const int t = threadIdx.x;
    sm[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const int add = t >= off ? sm[t - off] : 0;
        __syncthreads();
        sm[t] += add;
        __syncthreads();
    }
    total = sm[SCAN_THREADS - 1];
    const int incl = sm[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const int *in, int n, int *tile_sums)
{
    __shared__ int sm[SCAN_THREADS];
    const long long b0 = (long long)blockIdx.x * SCAN_TILE;
    int s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const long long idx = b0 + (long long)q * SCAN_THREADS + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    int total;
    block_exclusive_scan(s, sm, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(int *tile_sums, int ntiles)
{
    __shared__ int sm[SCAN_THREADS];
    int carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += SCAN_THREADS) {
        const int idx = b0 + threadIdx.x;
        const int v = idx < ntiles ? tile_sums[idx] : 0;
        int total;
        const int ex = block_exclusive_scan(v, sm, total);
        if (idx < ntiles) tile_sums[idx] = ex + carry;
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int *data, int n, const int *tile_sums)
{
    __shared__ int sm[SCAN_THREADS];
    // each thread owns SCAN_ITEMS consecutive elements of the tile
    const long long b0 = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    int vals[SCAN_ITEMS];
    int s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const long long idx = b0 + q;
        vals[q] = idx < n ? data[idx] : 0;
        s += vals[q];
    }
    int total;
    int run = block_exclusive_scan(s, sm, total) + tile_sums[blockIdx.x];
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const long long idx = b0 + q;
        if (idx < n) data[idx] = run;
        run += vals[q];
    }
}

__global__ __launch_bounds__(PBLOCK) void k_sort_scatter(SortArgs a)
{
    const int p = blockIdx.x * PBLOCK + threadIdx.x;
    if (p >= a.n) return;
    const int dst = a.counts[a.key[p]] + a.rank[p];
    for (int c = 0; c < 6; ++c) a.dst[c][dst] = a.src[c][p];
    a.id_dst[dst] = a.id_src[p];
}

int scan_tmp_size(int n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_sort(const SortArgs &a, int *scan_tmp, int scan_tmp_len, hipStream_t s)
{
    (void)scan_tmp_len;
    const int ncount = a.ncell + 1;
    launch_fill_i32(a.counts, 0, ncount, s);
    launch_fill_i32(a.box, INT_MAX, 3, s);
    launch_fill_i32(a.box + 3, INT_MIN, 3, s);
    if (a.n > 0) {
        const int nb = (a.n + PBLOCK - 1) / PBLOCK;
        hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(PBLOCK), 0, s, a);
    }
    const int ntiles = (ncount + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_THREADS), 0, s, a.counts, ncount, scan_tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, s, scan_tmp, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(SCAN_THREADS), 0, s, a.counts, ncount, scan_tmp);
    if (a.n > 0) {
        const int nb = (a.n + PBLOCK - 1) / PBLOCK;
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(PBLOCK), 0, s, a);
    }
}

}  // namespace pic
