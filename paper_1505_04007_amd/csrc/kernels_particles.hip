// Particle kernels for gfx950: staggered trilinear gather, relativistic
// Boris push, move, and charge-conserving (Esirkepov, first-order shape)
// current deposition; counting sort of the particles by cell.
//
// Gather.  E^n and B^n = mu0 (H^{n-1/2} + H^{n+1/2})/2 are interpolated on
// each component's own staggered lattice.  The H update also writes the
// average of its two time levels inside the particle box, so B costs one
// array per component.  Along x the two corners of a trilinear stencil are
// adjacent in memory and are fetched with one 8-byte load (4 per component
// instead of 8); a periodic x axis, where the pair can wrap, uses 4-byte loads.
//
// Deposit.  A move x0 -> x1 shorter than one cell touches at most three
// nodes per axis, [b, b+2] with b = min(floor x0, floor x1).  Its current is
// 18 Jx + 18 Jy + 18 Jz edge values on that window.  Particles are kept
// sorted by cell, so the lanes of a wavefront mostly share a window: lanes
// with equal windows are summed across the wavefront by recursive halving
// (64 slots -> one slot per lane).  The two widest exchange rounds use the
// gfx950 half-wave swaps (v_permlane32_swap, v_permlane16_swap), the four
// narrow ones DPP lane moves, so no round goes through LDS.  Each lane then
// issues at most one global float atomic.  Windows still unresolved after a
// few rounds fall back to per-lane atomics.
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

// Per-axis corner data of the trilinear gather on the two lattices an axis
// can carry: nodes (h = 0) and half nodes (h = 1).  o0/o1 are the linear
// offsets of the two corners (clamped into the box), m0/m1 their weights
// with the wall mask folded in (0 for a corner beyond a wall).
struct Axis2 {
    int o0[2], o1[2];
    float m0[2], m1[2];
};

__device__ __forceinline__ void axis_corners(float x, int n, int per, int stride, Axis2 &A)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float s = h ? x - 0.5f : x;
        const float f = floorf(s);
        const int i = (int)f;
        const float w1 = s - f, w0 = 1.f - w1;
        int i0 = i, i1 = i + 1;
        bool ok0 = i0 >= 0 && i0 < n, ok1 = i1 >= 0 && i1 < n;
        if (per) {
            i0 = i0 < 0 ? i0 + n : (i0 >= n ? i0 - n : i0);
            i1 = i1 < 0 ? i1 + n : (i1 >= n ? i1 - n : i1);
            ok0 = ok1 = true;
        }
        i0 = min(max(i0, 0), n - 1);
        i1 = min(max(i1, 0), n - 1);
        A.o0[h] = i0 * stride;
        A.o1[h] = i1 * stride;
        A.m0[h] = ok0 ? w0 : 0.f;
        A.m1[h] = ok1 ? w1 : 0.f;
    }
}

// x corners as one adjacent pair (st, st+1), st in [0, nx-2] (nx >= 2 on a
// wall axis), with the weights of the two loaded values; a corner beyond a
// wall gets weight 0.
struct XPair {
    int o[2];
    float wa[2], wb[2];
};

__device__ __forceinline__ void x_pairs(float x, int nx, XPair &P)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float s = h ? x - 0.5f : x;
        const float f = floorf(s);
        const int i = (int)f;
        const float w1 = s - f, w0 = 1.f - w1;
        const int st = min(max(i, 0), nx - 2);
        // i == st: both corners in the pair; i < st (i = -1): corner 0 = st
        // carries w1; i > st (i = nx-1): corner nx-1 = st+1 carries w0
        P.o[h] = st;
        P.wa[h] = i == st ? w0 : (i < st ? w1 : 0.f);
        P.wb[h] = i == st ? w1 : (i < st ? 0.f : w0);
    }
}

// dword-aligned 8-byte global load
typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ float2 ld2(const float *p)
{
    const float2_a4 v = *(gp<const float2_a4>)G(p);
    return make_float2(v.x, v.y);
}

// Trilinear value of a component that sits at half nodes along the axes
// flagged (HX, HY, HZ).
template <int HX, int HY, int HZ>
__device__ __forceinline__ float gather_pair(const float *__restrict__ f, const XPair &X,
                                             const Axis2 &Y, const Axis2 &Z)
{
    float v = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int o = X.o[HX] + (b ? Y.o1[HY] : Y.o0[HY]) + (c ? Z.o1[HZ] : Z.o0[HZ]);
            const float w = (b ? Y.m1[HY] : Y.m0[HY]) * (c ? Z.m1[HZ] : Z.m0[HZ]);
            const float2 p = ld2(f + o);
            v += w * (X.wa[HX] * p.x + X.wb[HX] * p.y);
        }
    return v;
}

template <int HX, int HY, int HZ>
__device__ __forceinline__ float gather_scalar(const float *__restrict__ f, const Axis2 &X,
                                               const Axis2 &Y, const Axis2 &Z)
{
    float v = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int o = (q ? X.o1[HX] : X.o0[HX]) + (b ? Y.o1[HY] : Y.o0[HY]) +
                              (c ? Z.o1[HZ] : Z.o0[HZ]);
                const float w = (q ? X.m1[HX] : X.m0[HX]) * (b ? Y.m1[HY] : Y.m0[HY]) *
                                (c ? Z.m1[HZ] : Z.m0[HZ]);
                v += w * G(f)[o];
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

// Esirkepov factors of one move: the running sum of dS along each current's
// own axis (pre[axis][edge]) and the transverse weight
//   T = S0 S0' + (dS S0' + S0 dS')/2 + dS dS'/3 = A A' + dS dS'/12,  A = S0 + dS/2,
// of the other two axes.  Slot s has current pre * T.  Every index used
// below is a compile-time constant after unrolling, so nothing leaves
// registers.
struct Dep {
    float pre[3][2];
    float Tyz[3][3], Txz[3][3], Txy[3][3];
};

__device__ __forceinline__ void make_dep(const float S0[3][3], const float dS[3][3], Dep &d)
{
    float A[3][3], D[3][3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        d.pre[ax][0] = dS[ax][0];
        d.pre[ax][1] = dS[ax][0] + dS[ax][1];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            A[ax][m] = S0[ax][m] + 0.5f * dS[ax][m];
            D[ax][m] = (1.f / 12.f) * dS[ax][m];
        }
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            d.Tyz[p][q] = A[1][p] * A[2][q] + D[1][p] * dS[2][q];
            d.Txz[p][q] = A[0][p] * A[2][q] + D[0][p] * dS[2][q];
            d.Txy[p][q] = A[0][p] * A[1][q] + D[0][p] * dS[1][q];
        }
}

// Current of slot s, scaled by f.
__device__ __forceinline__ float slot_value(const Dep &d, int s, float f)
{
    int comp, oi, oj, ok;
    slot_geom(s, comp, oi, oj, ok);
    if (comp == 0) return f * d.pre[0][oi] * d.Tyz[oj][ok];
    if (comp == 1) return f * d.pre[1][oj] * d.Txz[oi][ok];
    return f * d.pre[2][ok] * d.Txy[oi][oj];
}

// Cell index of slot s of the window at (bx, by, bz) after wrapping, or -1
// when it falls outside the grid on a non-periodic axis.
__device__ __forceinline__ int slot_index(const PartArgs &a, int s, int bx, int by, int bz, int &comp)
{
    int oi, oj, ok;
    slot_geom(s, comp, oi, oj, ok);
    int i = bx + oi, j = by + oj, k = bz + ok;
    if (a.per[0]) i = wrapn(i, a.nx);
    else if (i < 0 || i >= a.nx) return -1;
    if (a.per[1]) j = wrapn(j, a.ny);
    else if (j < 0 || j >= a.ny) return -1;
    if (a.per[2]) k = wrapn(k, a.nz);
    else if (k < 0 || k >= a.nz) return -1;
    return i + a.nx * (j + a.ny * k);
}

__device__ __forceinline__ float *slot_addr(const PartArgs &a, int s, int bx, int by, int bz)
{
    int comp;
    const int q = slot_index(a, s, bx, by, bz, comp);
    if (q < 0) return nullptr;
    // select, not a[comp]: a runtime index into the argument block would put it in scratch
    float *J = comp == 0 ? a.Jb[0] : (comp == 1 ? a.Jb[1] : a.Jb[2]);
    return J + q;
}

// Fixed-point deposit: each particle's slot currents are rounded to integer
// units (qscale per V/m, at most 2^24 per slot) before anything is summed, so
// the wavefront sums (at most 2^30) and the 64-bit atomics are exact and the
// result does not depend on which lanes share a round or on atomic order.
__device__ __forceinline__ void add_fixed(const PartArgs &a, int comp, int q, int units)
{
    unsigned long long *J = comp == 0 ? a.Jq[0] : (comp == 1 ? a.Jq[1] : a.Jq[2]);
    gatomic_add(G(J) + q, (unsigned long long)(long long)units);
}

// Sum of two slot values: FP32, or the int32 fixed-point units held in the
// same registers.
template <int INT>
__device__ __forceinline__ float add2(float x, float y)
{
    return INT ? __int_as_float(__float_as_int(x) + __float_as_int(y)) : x + y;
}

// Lane l receives x from lane l ^ OFF (OFF = 8, 4, 2, 1), by DPP row moves.
template <int OFF>
__device__ __forceinline__ float xor_lane(float x)
{
    const int v = __float_as_int(x);
    int r;
    if (OFF == 8) {
        r = __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);  // row_ror:8
    } else if (OFF == 4) {
        // lanes with bit 2 clear (banks 0, 2) read l + 4, the others l - 4
        const int t = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xf, 0x5, false);  // row_shl:4
        r = __builtin_amdgcn_update_dpp(t, v, 0x114, 0xf, 0xa, false);            // row_shr:4
    } else if (OFF == 2) {
        r = __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    } else {
        r = __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    }
    return __int_as_float(r);
}

template <int OFF, int INT>
__device__ __forceinline__ void halve_dpp(float *v, int lane)
{
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int e = 0; e < OFF; ++e) {
        const float send = up ? v[e] : v[e + OFF];
        const float keep = up ? v[e + OFF] : v[e];
        v[e] = add2<INT>(keep, xor_lane<OFF>(send));
    }
}

// Rounds of width 32 and 16: the lower half-wave keeps slot e, the upper
// keeps slot e + OFF; a half-wave swap of the two registers puts each half's
// partner values next to its own, and the sum finishes the round.  The first
// round reads the 54 slot currents of a lane, or zeros for a lane outside
// the round's window.
template <int INT>
__device__ __forceinline__ void halve32(const float *val, bool mine, float *v)
{
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const float lo = mine ? val[e] : 0.f;
        const float hi = (e + 32 < 54 && mine) ? val[e + 32 < 54 ? e + 32 : 0] : 0.f;
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
        v[e] = add2<INT>(__uint_as_float(r[0]), __uint_as_float(r[1]));
    }
}

template <int INT>
__device__ __forceinline__ void halve16(float *v)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[e]), __float_as_uint(v[e + 16]),
                                                        false, false);
        v[e] = add2<INT>(__uint_as_float(r[0]), __uint_as_float(r[1]));
    }
}

// After the six rounds lane l holds the sum of slot l over the lanes with
// `mine` set.
template <int INT>
__device__ __forceinline__ float wave_reduce64(const float *val, bool mine, int lane)
{
    float v[32];
    halve32<INT>(val, mine, v);
    halve16<INT>(v);
    halve_dpp<8, INT>(v, lane);
    halve_dpp<4, INT>(v, lane);
    halve_dpp<2, INT>(v, lane);
    halve_dpp<1, INT>(v, lane);
    return v[0];
}

// A window shared by at least ROUND_LANES lanes is summed by a wavefront
// round (about 220 VALU instructions, then one atomic per slot); the lanes of
// smaller windows add their slots with per-lane atomics, all such lanes of the
// wavefront together (54 atomic instructions however many lanes).
constexpr int ROUND_LANES = 3;

// ---- row-union deposit ----
// A wavefront whose windows share their y and z base and differ only in x
// (consecutive sorted particles in one grid row, the usual case away from the
// bunch core) spans a union of windows along x.  Inclusive prefix sums of the
// 54 slot currents are taken over the wavefront's lanes (six DPP adds per
// slot), so a run of lanes with the same window sums to P(its last lane) -
// P(the last lane of the run before it).  When every window has one run (the
// lanes are sorted), the last lane of each run stores its P as the block of
// its window in tile `plus` and as the block of the next run's window in tile
// `minus`: plain LDS stores of whole blocks, no LDS atomics (which issue
// slowly even when their addresses differ).  Each entry of the union then
// sums, over the up to three windows covering it, plus - minus of the slot it
// is in those windows, and goes to J_b in a few coalesced atomic
// instructions, however many windows the wavefront has.  Lanes that do not
// deposit carry zeros and a key of -1: their runs store nothing in `plus` and
// pass the running sum on to `minus`.
constexpr int UNION_KEYS = 14;           // window bases a union may span
constexpr int UNION_XW = UNION_KEYS + 2;  // x nodes of the widest union
// floats per window: 54 slots, 16-byte aligned, and an odd number of 16-byte
// groups so the readback's lanes (one window apart) fall in different banks
constexpr int UNION_BLOCK = 60;
// two zero blocks on each side: the readback's window index t - a runs over
// -2 .. UNION_XW - 1 without a test
constexpr int UNION_PAD = 2;
constexpr int UNION_TILE = (UNION_KEYS + 2 * UNION_PAD) * UNION_BLOCK;

// Reductions over the wavefront in the usual GFX9 pattern: prefix within
// 16-lane rows, then the row broadcasts; the result is valid at lane 63.
__device__ __forceinline__ int wave_min_dpp(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ unsigned wave_or_dpp(unsigned v)
{
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);
    return __builtin_amdgcn_readlane(v, 63);
}

// Inclusive prefix sum over the wavefront's lanes: prefix sums within the
// 16-lane rows (DPP row shifts, each fused into its add), then the row
// totals carried across rows.  The two cross-row steps add lane 15 of rows 0
// and 2 to rows 1 and 3, then lane 31 to rows 2 and 3; each is one DPP add
// that leaves the other rows untouched, written out because the compiler
// splits a row-masked DPP add into three instructions.  A DPP read of a VGPR
// that a VALU instruction has just written needs two wait states: the s_nops.
__device__ __forceinline__ float wave_prefix(float v)
{
#define PIC_PREFIX_STEP(ctrl)                                                                                 \
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, true))
    PIC_PREFIX_STEP(0x111);  // row_shr:1
    PIC_PREFIX_STEP(0x112);  // row_shr:2
    PIC_PREFIX_STEP(0x114);  // row_shr:4
    PIC_PREFIX_STEP(0x118);  // row_shr:8
#undef PIC_PREFIX_STEP
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(v));
    return v;
}

// Store the 54 values as the block of window k (relative to the union's
// first base) of a tile.
__device__ __forceinline__ void union_store(float *tile, int k, const float *val)
{
    float4 *d = reinterpret_cast<float4 *>(tile + (k + UNION_PAD) * UNION_BLOCK);
#pragma unroll
    for (int q = 0; q < 13; ++q) d[q] = make_float4(val[4 * q], val[4 * q + 1], val[4 * q + 2], val[4 * q + 3]);
    reinterpret_cast<float2 *>(tile + (k + UNION_PAD) * UNION_BLOCK)[26] = make_float2(val[52], val[53]);
}

// Union entries of one current component: x position t (0 .. UNION_XW - 1
// from the first base) and R transverse offsets (r = 0 .. R-1, y-major with NZ
// z offsets per y offset); the window at base t - a holds the entry as slot
// S0 + a * SA + r.  All LDS reads are issued first (windows outside the union
// read the zero padding), then the sums, then one atomic add per nonzero sum;
// the component is a template argument so that J stays a plain pointer.
template <int S0, int SA, int NA, int R, int NZ>
__device__ __forceinline__ void union_flush(float *J, const float *plus, const float *minus, int lane, int base,
                                            int sy, int sz)
{
    constexpr int N = R * UNION_XW;
    constexpr int IT = (N + 63) / 64;
    float pv[IT][NA], mv[IT][NA];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = min(it * 64 + lane, N - 1);
        const int t = e % UNION_XW, r = e / UNION_XW;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int q = (t - a + UNION_PAD) * UNION_BLOCK + S0 + a * SA + r;
            pv[it][a] = plus[q];
            mv[it][a] = minus[q];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = it * 64 + lane;
        const int t = e % UNION_XW, r = e / UNION_XW;
        float v = 0.f;
#pragma unroll
        for (int a = 0; a < NA; ++a) v += pv[it][a] - mv[it][a];
        if (e < N && v != 0.f) gatomic_add(G(J) + base + t + sy * (r / NZ) + sz * (r % NZ), v);
    }
}

// Deposit of a wavefront whose depositing lanes all have window base
// (bx, by, bz) with the same by, bz, bxmin <= bx < bxmin + UNION_KEYS, the
// union inside the grid, and one run of lanes per window.  val: the lane's 54
// slot currents (0 where it does not deposit); key: bx - bxmin, or -1 for a
// lane that does not deposit; knext: the key of lane + 1 (-1 past lane 63);
// last: the lane ends its run.
__device__ __forceinline__ void deposit_union(const PartArgs &a, float *val, int lane, int key, int knext,
                                              bool last, int bxmin, int by, int bz, float *plus, float *minus,
                                              bool ycross, bool zcross)
{
    // one wavefront per workgroup: its LDS operations execute in program
    // order, and the wave barriers keep the compiler from moving the tiles'
    // accesses of one phase into another
    constexpr int N4 = UNION_TILE / 4;
    for (int e = lane; e < N4; e += 64) {
        reinterpret_cast<float4 *>(plus)[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        reinterpret_cast<float4 *>(minus)[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // a slot at node offset 2 along y (z) is exactly 0 for a move that stays
    // in one y (z) cell: when no lane crosses, its prefix sums are 0 as well
#pragma unroll
    for (int s = 0; s < 54; ++s) {
        int comp, oi, oj, ok;
        slot_geom(s, comp, oi, oj, ok);
        const bool y2 = comp != 1 && oj == 2, z2 = comp != 2 && ok == 2;
        if ((y2 && !ycross) || (z2 && !zcross)) continue;
        val[s] = wave_prefix(val[s]);
    }
    __builtin_amdgcn_wave_barrier();
    if (last && key >= 0) union_store(plus, key, val);
    if (last && knext >= 0) union_store(minus, knext, val);
    __builtin_amdgcn_wave_barrier();
    const int base = bxmin + a.nx * (by + a.ny * bz);
    const int sy = a.nx, sz = a.nx * a.ny;
    // the current arrays' addresses held in scalar registers through the
    // flush (otherwise each conditional atomic reloads its pointer from the
    // argument block and waits for it)
    float *J0 = a.Jb[0], *J1 = a.Jb[1], *J2 = a.Jb[2];
    asm volatile("" : "+s"(J0), "+s"(J1), "+s"(J2));
    // slots: Jx a*9 + b*3 + c (a edge, b, c nodes); Jy 18 + a*6 + m*3 + c;
    // Jz 36 + a*6 + b*2 + m (a x node, m edge)
    union_flush<0, 9, 2, 9, 3>(J0, plus, minus, lane, base, sy, sz);
    union_flush<18, 6, 3, 6, 3>(J1, plus, minus, lane, base, sy, sz);
    union_flush<36, 6, 3, 6, 2>(J2, plus, minus, lane, base, sy, sz);
}

template <int MODE, int PX, int FIX>
__device__ __forceinline__ void push_body(const PartArgs &a, int blk)
{
    const int p = blk * PUSH_BLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // the current set's arrays straight from the device state (one scalar
    // load after the state's address, not the set index and then its arrays)
    const gp<const DevState> st = G(a.st);
    const gp<float> __restrict__ X = G(st->P[0]);
    const gp<float> __restrict__ Y = G(st->P[1]);
    const gp<float> __restrict__ Z = G(st->P[2]);
    const gp<float> __restrict__ UX = G(st->P[3]);
    const gp<float> __restrict__ UY = G(st->P[4]);
    const gp<float> __restrict__ UZ = G(st->P[5]);
    bool dep = false;
    // zeroed: a lane that does not deposit is silenced by a factor 0 in the
    // wavefront sum, and 0 x (uninitialised register) could be NaN
    Dep d = {};
    int base[3] = {0, 0, 0};
    bool ycross = false, zcross = false;  // the move leaves its y (z) cell
    if (p < a.n) {
        // The gather and Boris run for every lane, with no branch on liveness
        // before them, so that all six particle loads go out together (a
        // branch lets the compiler sink loads below it, each sunk group one
        // more round trip to memory).  A lost particle gathers at the box
        // corner, a valid position, and nothing of it is written.  The
        // particle state streams with the non-temporal hint: it is touched
        // once per step, and the fields around it should stay cached.
        const float x = __builtin_nontemporal_load(X + p), y = __builtin_nontemporal_load(Y + p),
                    z = __builtin_nontemporal_load(Z + p);
        float u0 = __builtin_nontemporal_load(UX + p), u1 = __builtin_nontemporal_load(UY + p),
              u2 = __builtin_nontemporal_load(UZ + p);
        const bool live = live_pos(x, y, z, a.nx, a.ny, a.nz);
        const float xg = live ? x : 0.f, yg = live ? y : 0.f, zg = live ? z : 0.f;
        {
            Axis2 AY, AZ;
            axis_corners(yg, a.ny, a.per[1], a.nx, AY);
            axis_corners(zg, a.nz, a.per[2], a.nx * a.ny, AZ);
            // E^n and Ht^n = (Ht^{n-1/2} + Ht^{n+1/2})/2 at x^n
            float e0, e1, e2, h0, h1, h2;
            if (PX) {
                Axis2 AX;
                axis_corners(xg, a.nx, a.per[0], 1, AX);
                e0 = gather_scalar<1, 0, 0>(a.E[0], AX, AY, AZ);
                e1 = gather_scalar<0, 1, 0>(a.E[1], AX, AY, AZ);
                e2 = gather_scalar<0, 0, 1>(a.E[2], AX, AY, AZ);
                h0 = gather_scalar<0, 1, 1>(a.B[0], AX, AY, AZ);
                h1 = gather_scalar<1, 0, 1>(a.B[1], AX, AY, AZ);
                h2 = gather_scalar<1, 1, 0>(a.B[2], AX, AY, AZ);
            } else {
                XPair XP;
                x_pairs(xg, a.nx, XP);
                e0 = gather_pair<1, 0, 0>(a.E[0], XP, AY, AZ);
                e1 = gather_pair<0, 1, 0>(a.E[1], XP, AY, AZ);
                e2 = gather_pair<0, 0, 1>(a.E[2], XP, AY, AZ);
                h0 = gather_pair<0, 1, 1>(a.B[0], XP, AY, AZ);
                h1 = gather_pair<1, 0, 1>(a.B[1], XP, AY, AZ);
                h2 = gather_pair<1, 1, 0>(a.B[2], XP, AY, AZ);
            }
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
        }
        if (live) {
            const float g = rsqrtf(1.f + u0 * u0 + u1 * u1 + u2 * u2);
            float x1 = x + a.S * u0 * g, y1 = y + a.S * u1 * g, z1 = z + a.S * u2 * g;
            // leaving through a wall, or a non-finite move, deactivates the particle
            const bool out = !(isfinite(x1) && isfinite(y1) && isfinite(z1)) ||
                             (!a.per[0] && !(x1 >= 0.f && x1 < (float)a.nx)) ||
                             (!a.per[1] && !(y1 >= 0.f && y1 < (float)a.ny)) ||
                             (!a.per[2] && !(z1 >= 0.f && z1 < (float)a.nz));
            __builtin_nontemporal_store(u0, UX + p);
            __builtin_nontemporal_store(u1, UY + p);
            __builtin_nontemporal_store(u2, UZ + p);
            if (out) {
                __builtin_nontemporal_store(-1.f, X + p);  // left the box: deactivated, last move not deposited
            } else {
                // written out per axis: constant indices keep S0/dS in registers
                float S0[3][3], dS[3][3];
                base[0] = min((int)floorf(x), (int)floorf(x1));
                base[1] = min((int)floorf(y), (int)floorf(y1));
                base[2] = min((int)floorf(z), (int)floorf(z1));
                ycross = (int)floorf(y) != (int)floorf(y1);
                zcross = (int)floorf(z) != (int)floorf(z1);
                shapes(x, x1, base[0], S0[0], dS[0]);
                shapes(y, y1, base[1], S0[1], dS[1]);
                shapes(z, z1, base[2], S0[2], dS[2]);
                make_dep(S0, dS, d);
                dep = true;
                if (a.per[0]) x1 = fold(x1, a.nx);
                if (a.per[1]) y1 = fold(y1, a.ny);
                if (a.per[2]) z1 = fold(z1, a.nz);
                __builtin_nontemporal_store(x1, X + p);
                __builtin_nontemporal_store(y1, Y + p);
                __builtin_nontemporal_store(z1, Z + p);
            }
        }
    }
    // the 54 slot currents of this particle's move (0 for a lane that does not deposit)
    const float qd = a.qd;
    float val[54];
#pragma unroll
    for (int s = 0; s < 54; ++s) val[s] = slot_value(d, s, qd);
    if (FIX) {
        // integer units per slot, kept in the same registers
        const float qs = a.qscale;
#pragma unroll
        for (int s = 0; s < 54; ++s) val[s] = __int_as_float(__float2int_rn(val[s] * qs));
    }
    const unsigned long long live = __ballot(dep);
    // per-wavefront push counter (one slot per wavefront of the launch)
    // (an atomic whose result is unused: the wavefront does not wait for the
    // counter's old value as a load-add-store would)
    if (lane == 0 && live) gatomic_add(G(a.pushes) + (p >> 6), (unsigned long long)__popcll(live));
    unsigned long long rem = live;
    if (MODE == 0 && !FIX && live) {
        // one grid row of windows spanning at least two x bases: the row-union tiles
        __shared__ float4 tplus4[UNION_TILE / 4], tminus4[UNION_TILE / 4];
        const int leader = __ffsll((long long)live) - 1;
        const int by0 = __builtin_amdgcn_readlane(base[1], leader);
        const int bz0 = __builtin_amdgcn_readlane(base[2], leader);
        if (__ballot(dep && (base[1] != by0 || base[2] != bz0)) == 0ull) {
            const int bxmin = wave_min_dpp(dep ? base[0] : INT_MAX);
            const int bxmax = -wave_min_dpp(dep ? -base[0] : INT_MAX);
            const bool inside = bxmin >= 0 && bxmax + 2 < a.nx && by0 >= 0 && by0 + 2 < a.ny && bz0 >= 0 &&
                                bz0 + 2 < a.nz;
            if (inside && bxmax > bxmin && bxmax - bxmin < UNION_KEYS) {
                const int key = dep ? base[0] - bxmin : -1;
                const int knext = __builtin_amdgcn_update_dpp(-1, key, 0x130, 0xf, 0xf, false);  // wave_shl:1
                const bool last = lane == 63 || knext != key;
                // one run per window: as many runs as windows
                const unsigned keys = wave_or_dpp(last && key >= 0 ? 1u << key : 0u);
                if (__popc(keys) == __popcll(__ballot(last && key >= 0))) {
                    deposit_union(a, val, lane, key, knext, last, bxmin, by0, bz0, (float *)tplus4,
                                  (float *)tminus4, __ballot(dep && ycross) != 0ull,
                                  __ballot(dep && zcross) != 0ull);
                    rem = 0;
                }
            }
        }
    }
    if (MODE != 1 && rem) {
        // lane l < 54 owns slot l of every round's window: its component and
        // offset from the window's base node, computed once
        int lc, li, lj, lk;
        slot_geom(lane < 54 ? lane : 0, lc, li, lj, lk);
        const int lrel = li + a.nx * (lj + a.ny * lk);
        float *Jl = lc == 0 ? a.Jb[0] : (lc == 1 ? a.Jb[1] : a.Jb[2]);
        const int key = (base[0] + 1) + (a.nx + 2) * ((base[1] + 1) + (a.ny + 2) * (base[2] + 1));
        unsigned long long small = 0;
        while (rem) {
            const int leader = __ffsll((long long)rem) - 1;
            const int k0 = __builtin_amdgcn_readlane(key, leader);
            const bool mine = ((rem >> lane) & 1ull) && key == k0;
            const unsigned long long m = __ballot(mine);
            rem &= ~m;
            if (__popcll(m) < ROUND_LANES) {
                small |= m;
                continue;
            }
            const float tot = wave_reduce64<FIX>(val, mine, lane);
            const int bx = __builtin_amdgcn_readlane(base[0], leader);
            const int by = __builtin_amdgcn_readlane(base[1], leader);
            const int bz = __builtin_amdgcn_readlane(base[2], leader);
            if (lane < 54 && (FIX ? __float_as_int(tot) != 0 : tot != 0.f)) {
                const bool inside = bx >= 0 && bx + 2 < a.nx && by >= 0 && by + 2 < a.ny && bz >= 0 &&
                                    bz + 2 < a.nz;
                if (FIX) {
                    int comp = lc;
                    const int q = inside ? (bx + a.nx * (by + a.ny * bz)) + lrel
                                         : slot_index(a, lane, bx, by, bz, comp);
                    if (q >= 0) add_fixed(a, comp, q, __float_as_int(tot));
                } else {
                    float *ad = inside ? Jl + (bx + a.nx * (by + a.ny * bz)) + lrel : slot_addr(a, lane, bx, by, bz);
                    if (ad) gatomic_add(G(ad), tot);
                }
            }
        }
        rem = small;
    }
    if ((rem >> lane) & 1ull) {
        const bool inside = base[0] >= 0 && base[0] + 2 < a.nx && base[1] >= 0 && base[1] + 2 < a.ny &&
                            base[2] >= 0 && base[2] + 2 < a.nz;
        if (inside) {
            // slot offsets from the window's base node are uniform: one add per slot
            const int lin = base[0] + a.nx * (base[1] + a.ny * base[2]);
            const int sy = a.nx, sz = a.nx * a.ny;
#pragma unroll
            for (int s = 0; s < 54; ++s) {
                int comp, oi, oj, ok;
                slot_geom(s, comp, oi, oj, ok);
                const float v = val[s];
                if (FIX) {
                    const int u = __float_as_int(v);
                    if (u != 0) add_fixed(a, comp, lin + (oi + sy * oj + sz * ok), u);
                } else {
                    float *J = comp == 0 ? a.Jb[0] : (comp == 1 ? a.Jb[1] : a.Jb[2]);
                    if (v != 0.f) gatomic_add(G(J) + lin + (oi + sy * oj + sz * ok), v);
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < 54; ++s) {
                const float v = val[s];
                if (FIX) {
                    const int u = __float_as_int(v);
                    int comp;
                    const int q = u != 0 ? slot_index(a, s, base[0], base[1], base[2], comp) : -1;
                    if (q >= 0) add_fixed(a, comp, q, u);
                } else if (v != 0.f) {
                    float *ad = slot_addr(a, s, base[0], base[1], base[2]);
                    if (ad) gatomic_add(G(ad), v);
                }
            }
        }
    }
}

template <int MODE, int PX, int FIX>
__global__ __launch_bounds__(PUSH_BLOCK) void k_push_deposit(PartArgs a)
{
    push_body<MODE, PX, FIX>(a, blockIdx.x);
}

// Many simulations in one launch: workgroup b is push block own[b] & 0xffffff
// of simulation own[b] >> 24 (a table the host builds).
template <int MODE, int PX>
__global__ __launch_bounds__(PUSH_BLOCK) void k_push_deposit_batch(const PartArgs *__restrict__ args,
                                                                   const int *__restrict__ own)
{
    const int o = own[blockIdx.x];
    push_body<MODE, PX, 0>(args[o >> 24], o & 0xffffff);
}

void launch_push_deposit(const PartArgs &a, int mode, hipStream_t s)
{
    if (a.n <= 0) return;
    const int nb = (int)(((long long)a.n + PUSH_BLOCK - 1) / PUSH_BLOCK);
    // mode 2: wavefront-reduced deposit into the fixed-point current
    const bool fix = mode == 2 && a.Jq[0];
    if (a.per[0]) {
        if (fix) hipLaunchKernelGGL((k_push_deposit<0, 1, 1>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
        else if (mode == 1) hipLaunchKernelGGL((k_push_deposit<1, 1, 0>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_push_deposit<0, 1, 0>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
    } else {
        if (fix) hipLaunchKernelGGL((k_push_deposit<0, 0, 1>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
        else if (mode == 1) hipLaunchKernelGGL((k_push_deposit<1, 0, 0>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_push_deposit<0, 0, 0>), dim3(nb), dim3(PUSH_BLOCK), 0, s, a);
    }
}

// `mode` bit 0: per-lane atomics; bit 1: some simulation has a periodic x axis.
void launch_push_deposit_batch(const PartArgs *args, const int *own, int total, int mode, hipStream_t s)
{
    if (total <= 0) return;
    switch (mode & 3) {
    case 0: hipLaunchKernelGGL((k_push_deposit_batch<0, 0>), dim3(total), dim3(PUSH_BLOCK), 0, s, args, own); break;
    case 1: hipLaunchKernelGGL((k_push_deposit_batch<1, 0>), dim3(total), dim3(PUSH_BLOCK), 0, s, args, own); break;
    case 2: hipLaunchKernelGGL((k_push_deposit_batch<0, 1>), dim3(total), dim3(PUSH_BLOCK), 0, s, args, own); break;
    default: hipLaunchKernelGGL((k_push_deposit_batch<1, 1>), dim3(total), dim3(PUSH_BLOCK), 0, s, args, own); break;
    }
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

template <bool MAX>
__device__ __forceinline__ int wave_minmax(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = MAX ? max(v, o) : min(v, o);
    }
    return v;
}

// Cell key of a particle position (the lost-particle bucket ncell when it is
// not live).
// live_pos evaluated without short-circuit: every coordinate is read before
// the test, so the compiler cannot sink the loads of y and z below a branch
// on x (each sunk group would be one more round trip to memory).
__device__ __forceinline__ bool live_all(float x, float y, float z, int nx, int ny, int nz)
{
    return (x >= 0.f) & (x < (float)nx) & (y >= 0.f) & (y < (float)ny) & (z >= 0.f) & (z < (float)nz);
}

__device__ __forceinline__ int cell_key(float x, float y, float z, int nx, int ny, int nz)
{
    if (!live_all(x, y, z, nx, ny, nz)) return nx * ny * nz;
    return min((int)x, nx - 1) + nx * (min((int)y, ny - 1) + ny * min((int)z, nz - 1));
}

// Count particles per cell.  Lanes of a wavefront with the same cell (most
// of them: the particles are nearly sorted from the last sort) reserve their
// ranks with one atomic and take consecutive ones in lane order, so the
// scatter writes them to consecutive places.  The groups are found first and
// their leaders then issue all their atomics at once, so a wavefront spread
// over many cells waits for one atomic return, not one per cell.
// Each run of equal keys in the array's order also counts itself in
// runs[key] and records its start in first[key]: the scatter keeps the order
// of a key that forms a single run.  The bunch is loaded ordered by x inside
// each cell and drifts almost uniformly, so that order survives the sorts
// and the particles of a wavefront stay ordered by their deposit windows.
__device__ __forceinline__ void count_body(const SortArgs &a, int blk)
{
    __shared__ int bb[6];
    if (threadIdx.x < 6) bb[threadIdx.x] = threadIdx.x < 3 ? INT_MAX : INT_MIN;
    __syncthreads();
    const int p = blk * PBLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int pc = a.st->pcur;
    int key = a.ncell;
    int cell[3] = {INT_MAX, INT_MAX, INT_MAX};
    bool in = false;
    // lane 0 also needs the cell of particle p - 1 (the run test below):
    // its position is loaded here, with the lane's own
    float xq = -1.f, yq = -1.f, zq = -1.f;
    if (lane == 0 && p > 0 && p <= a.n) {
        xq = a.P[pc][0][p - 1];
        yq = a.P[pc][1][p - 1];
        zq = a.P[pc][2][p - 1];
    }
    if (p < a.n) {
        const float x = a.P[pc][0][p], y = a.P[pc][1][p], z = a.P[pc][2][p];
        if (live_all(x, y, z, a.nx, a.ny, a.nz)) {
            cell[0] = min((int)x, a.nx - 1);
            cell[1] = min((int)y, a.ny - 1);
            cell[2] = min((int)z, a.nz - 1);
            key = cell[0] + a.nx * (cell[1] + a.ny * cell[2]);
            in = true;
        }
    }
    unsigned long long rem = __ballot(p < a.n);
    unsigned long long group = 0;  // lanes sharing this lane's cell
    int leader = lane;
    while (rem) {
        const int l0 = __ffsll((long long)rem) - 1;
        const int k0 = __builtin_amdgcn_readlane(key, l0);
        const unsigned long long m = __ballot(((rem >> lane) & 1ull) && key == k0);
        if ((m >> lane) & 1ull) {
            group = m;
            leader = l0;
        }
        rem &= ~m;
    }
    int b = 0;
    if (p < a.n && lane == leader) b = atomicAdd(&a.counts[key], __popcll(group));
    b = __shfl(b, leader, 64);
    const int rank = b + __popcll(group & ((1ull << lane) - 1ull));
    if (p < a.n) {
        a.key[p] = key;
        a.rank[p] = rank;
    }
    // key of particle p - 1: the lane below, or for lane 0 from its position
    int kprev = __builtin_amdgcn_update_dpp(-1, key, 0x138, 0xf, 0xf, false);  // wave_shr:1
    if (lane == 0 && p > 0 && p <= a.n) kprev = cell_key(xq, yq, zq, a.nx, a.ny, a.nz);
    if (p < a.n && (p == 0 || kprev != key)) {
        atomicAdd(&a.runs[key], 1);
        a.first[key] = p;
    }
    // box of the live cells: wavefront min / max, then the workgroup's in LDS
    const bool any = __ballot(in) != 0ull;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int lo = wave_minmax<false>(in ? cell[q] : INT_MAX);
        const int hi = wave_minmax<true>(in ? cell[q] : INT_MIN);
        if (lane == 0 && any) {
            atomicMin(&bb[q], lo);
            atomicMax(&bb[3 + q], hi);
        }
    }
    __syncthreads();
    // one partial box per workgroup (global atomics from every workgroup on
    // the same six words would serialise); k_box_reduce combines them
    if (threadIdx.x < 6) a.boxpart[blk * 6 + threadIdx.x] = bb[threadIdx.x];
}

__global__ __launch_bounds__(PBLOCK) void k_sort_count(SortArgs a) { count_body(a, blockIdx.x); }

// The live-cell box from the count workgroups' partial boxes (one workgroup).
constexpr int BOX_THREADS = 1024;
__device__ __forceinline__ void box_reduce_body(const SortArgs &a, int nparts)
{
    __shared__ int red[6][BOX_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int v[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
    for (int w = threadIdx.x; w < nparts; w += BOX_THREADS) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] = min(v[q], a.boxpart[w * 6 + q]);
            v[3 + q] = max(v[3 + q], a.boxpart[w * 6 + 3 + q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        v[q] = q < 3 ? wave_minmax<false>(v[q]) : wave_minmax<true>(v[q]);
        if (lane == 0) red[q][wave] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        int r = red[q][0];
        for (int w = 1; w < BOX_THREADS / 64; ++w) r = q < 3 ? min(r, red[q][w]) : max(r, red[q][w]);
        a.box[q] = r;
    }
}

__global__ __launch_bounds__(BOX_THREADS) void k_box_reduce(SortArgs a, int nparts) { box_reduce_body(a, nparts); }

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

// The keys a sort gives out: the cells of its live-cell box (the count
// kernel's), in global key order, then the lost-particle bucket (key ncell).
// Element e of that list.  The scans run over it alone: a key outside the box
// has no particle, so its offset is never read, and the offsets inside are
// those of a scan over every cell.
struct KeyDomain {
    int lo[3], w[3];
    long long cells;  // box cells; the list has cells + 1 entries
};

__device__ __forceinline__ KeyDomain key_domain(const SortArgs &a)
{
    KeyDomain D;
    D.cells = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int lo = a.box[d], hi = a.box[3 + d];
        D.lo[d] = lo;
        D.w[d] = hi >= lo ? hi - lo + 1 : 0;
        D.cells *= D.w[d];
    }
    return D;
}

// Element e of the list in 32-bit unsigned arithmetic: e < cells <= ncell
// and every key below ncell fit, since ncell < 2^31 (a box exists, so its
// widths are at least 1).
__device__ __forceinline__ long long domain_key(const SortArgs &a, const KeyDomain &D, long long e)
{
    if (e >= D.cells) return a.ncell;
    const unsigned ue = (unsigned)e, w0 = (unsigned)D.w[0], w1 = (unsigned)D.w[1];
    const unsigned r = ue / w0;
    const unsigned x = ue - r * w0;
    const unsigned z = r / w1;
    const unsigned y = r - z * w1;
    return (long long)(((unsigned)D.lo[0] + x) +
                       (unsigned)a.nx * (((unsigned)D.lo[1] + y) + (unsigned)a.ny * ((unsigned)D.lo[2] + z)));
}

// Workgroups of the scan launches: a fixed grid walking the list's tiles (the
// list's length is known on the device only).
constexpr int SCAN_BLOCKS = 1024;

// Workgroup blk of nblk walking the tiles.
__device__ __forceinline__ void scan_tiles_body(const SortArgs &a, int *tile_sums, int blk, int nblk)
{
    __shared__ int sm[SCAN_THREADS];
    const KeyDomain D = key_domain(a);
    const long long n = D.cells + 1;
    for (long long b0 = (long long)blk * SCAN_TILE; b0 < n; b0 += (long long)nblk * SCAN_TILE) {
        int s = 0;
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            const long long e = b0 + (long long)q * SCAN_THREADS + threadIdx.x;
            if (e < n) s += a.counts[domain_key(a, D, e)];
        }
        int total;
        block_exclusive_scan(s, sm, total);
        if (threadIdx.x == 0) tile_sums[b0 / SCAN_TILE] = total;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(SortArgs a, int *tile_sums)
{
    scan_tiles_body(a, tile_sums, blockIdx.x, gridDim.x);
}

// One workgroup; each thread scans SCAN_ITEMS consecutive tile sums of a
// chunk serially around one block scan of the thread totals.
__device__ __forceinline__ void scan_sums_body(const SortArgs &a, int *tile_sums)
{
    __shared__ int sm[SCAN_THREADS];
    const int ntiles = (int)((key_domain(a).cells + 1 + SCAN_TILE - 1) / SCAN_TILE);
    int carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += SCAN_TILE) {
        const int first = b0 + threadIdx.x * SCAN_ITEMS;
        int v[SCAN_ITEMS];
        int s = 0;
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            v[q] = first + q < ntiles ? tile_sums[first + q] : 0;
            s += v[q];
        }
        int total;
        int run = carry + block_exclusive_scan(s, sm, total);
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            if (first + q < ntiles) tile_sums[first + q] = run;
            run += v[q];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(SortArgs a, int *tile_sums) { scan_sums_body(a, tile_sums); }

__device__ __forceinline__ void scan_apply_body(const SortArgs &a, const int *tile_sums, int blk, int nblk)
{
    __shared__ int sm[SCAN_THREADS];
    const KeyDomain D = key_domain(a);
    const long long n = D.cells + 1;
    for (long long t0 = (long long)blk * SCAN_TILE; t0 < n; t0 += (long long)nblk * SCAN_TILE) {
        // each thread owns SCAN_ITEMS consecutive entries of the tile
        const long long b0 = t0 + (long long)threadIdx.x * SCAN_ITEMS;
        long long g[SCAN_ITEMS];
        int vals[SCAN_ITEMS];
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            g[q] = b0 + q < n ? domain_key(a, D, b0 + q) : -1;
            vals[q] = g[q] >= 0 ? a.counts[g[q]] : 0;
        }
        int s = 0;
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) s += vals[q];
        int total;
        int run = block_exclusive_scan(s, sm, total) + tile_sums[t0 / SCAN_TILE];
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            if (g[q] >= 0) a.counts[g[q]] = run;
            run += vals[q];
        }
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(SortArgs a, const int *tile_sums)
{
    scan_apply_body(a, tile_sums, blockIdx.x, gridDim.x);
}

// After the scatter: the counts and run counts of the list's keys back to 0,
// so that both arrays are 0 at every key between sorts (they start so).
__device__ __forceinline__ void sort_clear_body(const SortArgs &a, int blk, int nblk)
{
    const KeyDomain D = key_domain(a);
    const long long n = D.cells + 1;
    for (long long e = (long long)blk * blockDim.x + threadIdx.x; e < n; e += (long long)nblk * blockDim.x) {
        const long long g = domain_key(a, D, e);
        a.counts[g] = 0;
        a.runs[g] = 0;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_sort_clear(SortArgs a) { sort_clear_body(a, blockIdx.x, gridDim.x); }

__device__ __forceinline__ void scatter_body(const SortArgs &a, int blk)
{
    const int p = blk * PBLOCK + threadIdx.x;
    if (p >= a.n) return;
    const int pc = a.st->pcur;
    // every load first, in two rounds (the particle, its key and rank; then
    // the key's count and run), then the stores: the stores to the other
    // buffer set may alias the loads as far as the compiler knows, so a load
    // after a store would wait for it
    float v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = a.P[pc][c][p];
    const int id = a.id[pc][p];
    const int k = a.key[p];
    const int rk = a.rank[p];
    const int cnt = a.counts[k], runs = a.runs[k], f = a.first[k];
    const int dst = cnt + (runs == 1 ? p - f : rk);
#pragma unroll
    for (int c = 0; c < 6; ++c) a.P[pc ^ 1][c][dst] = v[c];
    a.id[pc ^ 1][dst] = id;
}

__global__ __launch_bounds__(PBLOCK) void k_sort_scatter(SortArgs a) { scatter_body(a, blockIdx.x); }

// After the scatter: the sorted set becomes current and the sort clock restarts.
__device__ __forceinline__ void done_body(const SortArgs &a)
{
    const int pc = a.st->pcur ^ 1;
    a.st->pcur = pc;
    a.st->since_sort = 0;
    for (int c = 0; c < 6; ++c) a.st->P[c] = a.P[pc][c];
}

__global__ void k_sort_done(SortArgs a)
{
    if (threadIdx.x == 0) done_body(a);
}

// ---- the sorts of many simulations in one launch per kernel ----
// Particle workgroups come from a table (member << 24 | the workgroup's index
// in that member, built by the host); each member's scans and clear get
// SORT_BATCH_BLOCKS workgroups of their own, walking its key list; the
// per-member single-workgroup kernels take one workgroup per member.
constexpr int SORT_BATCH_BLOCKS = 64;

__global__ __launch_bounds__(PBLOCK) void k_sort_count_batch(const SortArgs *__restrict__ args,
                                                             const int *__restrict__ own)
{
    const int o = own[blockIdx.x];
    count_body(args[o >> 24], o & 0xffffff);
}

__global__ __launch_bounds__(BOX_THREADS) void k_box_reduce_batch(const SortArgs *__restrict__ args)
{
    const SortArgs &a = args[blockIdx.x];
    box_reduce_body(a, (int)(((long long)a.n + PBLOCK - 1) / PBLOCK));
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles_batch(const SortArgs *__restrict__ args)
{
    const SortArgs &a = args[blockIdx.x / SORT_BATCH_BLOCKS];
    scan_tiles_body(a, a.scan_tmp, blockIdx.x % SORT_BATCH_BLOCKS, SORT_BATCH_BLOCKS);
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums_batch(const SortArgs *__restrict__ args)
{
    const SortArgs &a = args[blockIdx.x];
    scan_sums_body(a, a.scan_tmp);
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply_batch(const SortArgs *__restrict__ args)
{
    const SortArgs &a = args[blockIdx.x / SORT_BATCH_BLOCKS];
    scan_apply_body(a, a.scan_tmp, blockIdx.x % SORT_BATCH_BLOCKS, SORT_BATCH_BLOCKS);
}

__global__ __launch_bounds__(PBLOCK) void k_sort_scatter_batch(const SortArgs *__restrict__ args,
                                                               const int *__restrict__ own)
{
    const int o = own[blockIdx.x];
    scatter_body(args[o >> 24], o & 0xffffff);
}

__global__ __launch_bounds__(SCAN_THREADS) void k_sort_clear_batch(const SortArgs *__restrict__ args)
{
    sort_clear_body(args[blockIdx.x / SORT_BATCH_BLOCKS], blockIdx.x % SORT_BATCH_BLOCKS, SORT_BATCH_BLOCKS);
}

__global__ void k_sort_done_batch(const SortArgs *__restrict__ args, int nmem)
{
    if (threadIdx.x < nmem) done_body(args[threadIdx.x]);
}

int scan_tmp_size(long long n) { return (int)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

void launch_sort(const SortArgs &a, int *scan_tmp, hipStream_t s)
{
    // counts and runs are 0 at every key here (cleared at allocation and by
    // the previous sort over the keys it used)
    const int nb = (int)(((long long)a.n + PBLOCK - 1) / PBLOCK);
    if (a.n > 0) {
        hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(PBLOCK), 0, s, a);
        hipLaunchKernelGGL(k_box_reduce, dim3(1), dim3(BOX_THREADS), 0, s, a, nb);
    } else {
        launch_fill_i32(a.box, INT_MAX, 3, s);
        launch_fill_i32(a.box + 3, INT_MIN, 3, s);
    }
    // the list of keys has at most ncell + 1 entries
    const long long tiles = ((long long)a.ncell + 1 + SCAN_TILE - 1) / SCAN_TILE;
    const int grid = (int)std::min<long long>(tiles, SCAN_BLOCKS);
    hipLaunchKernelGGL(k_scan_tiles, dim3(grid), dim3(SCAN_THREADS), 0, s, a, scan_tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, s, a, scan_tmp);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid), dim3(SCAN_THREADS), 0, s, a, scan_tmp);
    if (a.n > 0) hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(PBLOCK), 0, s, a);
    hipLaunchKernelGGL(k_sort_clear, dim3(grid), dim3(SCAN_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_sort_done, dim3(1), dim3(64), 0, s, a);
}

void launch_sort_batch(const SortArgs *args, const int *own, int nown, int nmem, hipStream_t s)
{
    // every member has particles, and its counts and runs are 0 at every key
    if (nmem <= 0 || nown <= 0) return;
    const int g = nmem * SORT_BATCH_BLOCKS;
    hipLaunchKernelGGL(k_sort_count_batch, dim3(nown), dim3(PBLOCK), 0, s, args, own);
    hipLaunchKernelGGL(k_box_reduce_batch, dim3(nmem), dim3(BOX_THREADS), 0, s, args);
    hipLaunchKernelGGL(k_scan_tiles_batch, dim3(g), dim3(SCAN_THREADS), 0, s, args);
    hipLaunchKernelGGL(k_scan_sums_batch, dim3(nmem), dim3(SCAN_THREADS), 0, s, args);
    hipLaunchKernelGGL(k_scan_apply_batch, dim3(g), dim3(SCAN_THREADS), 0, s, args);
    hipLaunchKernelGGL(k_sort_scatter_batch, dim3(nown), dim3(PBLOCK), 0, s, args, own);
    hipLaunchKernelGGL(k_sort_clear_batch, dim3(g), dim3(SCAN_THREADS), 0, s, args);
    hipLaunchKernelGGL(k_sort_done_batch, dim3(1), dim3(64), 0, s, args, nmem);
}

}  // namespace pic
