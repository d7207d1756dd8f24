// HIP kernels for gfx950 (CDNA4): the acoustic leapfrog step with fused
// source injection and receiver sampling, the on-the-fly probe contractions
// of Algorithm 1, imaging, residual/objective, probe generation and model
// preparation.  Every kernel is deterministic: fixed summation orders, no
// floating-point atomics.
#include <hip/hip_runtime.h>

#include <cmath>

#include "tpx_internal.h"

namespace tpx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// The step kernels and their helpers pin every rounding: products are fused
// only where an fmaf is written, so one- and two-step launches, fused and
// separate sampling give bitwise identical results.

// (distance into the absorbing layer / nbl)^2 along one axis, padded index I
__device__ __forceinline__ float layer_frac2(int I, int nphys, int nb, float inv_nb) {
#pragma clang fp contract(off)
    int into = 0;
    if (I < nb) into = nb - I;
    else if (I > nb + nphys - 1) into = I - (nb + nphys - 1);
    const float d = (float)into * inv_nb;
    return d * d;
}

// leapfrog update of the damped wave equation for one node:
//   (1 + hd) next = 2 cur - (1 - hd) prev + beta (lap + src),  hd = d dt / 2
__device__ __forceinline__ float leapfrog(float cur, float prev, float beta, float lap, float src, float hd) {
#pragma clang fp contract(off)
    const float num = __builtin_fmaf(beta, lap + src, __builtin_fmaf(-(1.0f - hd), prev, 2.0f * cur));
    return num * __builtin_amdgcn_rcpf(1.0f + hd);   // rcp(1) = 1 exactly in the interior
}

// The same update where hd == 0 (undamped interior): bitwise equal to leapfrog(..., 0).
__device__ __forceinline__ float leapfrog0(float cur, float prev, float beta, float lap, float src) {
#pragma clang fp contract(off)
    return __builtin_fmaf(beta, lap + src, __builtin_fmaf(-1.0f, prev, 2.0f * cur));
}

// Sampling of `field` at this shot's points (receivers in the forward pass,
// the source in the adjoint pass).  Each point is handled by exactly one
// thread of the shot's blocks; the 2^D products are summed in a fixed order.
template <int NC>
__device__ __forceinline__ void sample_points(const Layout &L, const float *field, int k, const SampleTables &smp,
                                              int shot, int64_t block_in_shot, int64_t blocks_per_shot) {
#pragma clang fp contract(off)
    const int64_t G0 = L.G[0], plane = L.G[0] * L.G[1];
    for (int64_t i = block_in_shot * blockDim.x + threadIdx.x; i < smp.nsmp; i += blocks_per_shot * blockDim.x) {
        const int64_t e = (int64_t)shot * smp.nsmp + i;
        const int32_t b = smp.base[e];
        const float *w = smp.w + e * NC;
        float v = w[0] * field[b] + w[1] * field[b + 1] + w[2] * field[b + G0] + w[3] * field[b + G0 + 1];
        if (NC == 8) {
            // second z plane: offsets +plane; the y neighbour lives G0 away
            v += w[4] * field[b + plane] + w[5] * field[b + plane + 1] + w[6] * field[b + plane + G0] +
                 w[7] * field[b + plane + G0 + 1];
        }
        smp.out[shot * smp.out_shot_stride + (int64_t)k * smp.out_k_stride + i] = smp.scale * v;
    }
}

// Source term of one target node: its entries summed in their stored order.
__device__ __forceinline__ float segment_value(const InjectTables &inj, const float *a, float scale, int sg) {
#pragma clang fp contract(off)
    float acc = 0.0f;
    const int e1 = inj.seg_ent[sg + 1];
    for (int e = inj.seg_ent[sg]; e < e1; ++e) acc += inj.ent_w[e] * a[inj.ent_idx[e]];
    return acc * scale;
}

__device__ __forceinline__ int xcd_logical_block(int nlogical) {
    const int per = (int)gridDim.x >> 3;
    const int hw = (int)blockIdx.x;
    const int lid = (hw & 7) * per + (hw >> 3);
    return lid < nlogical ? lid : -1;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// First column past the 128-byte line that holds a row's last padded node.  The
// row's pitch always reaches it (G0 is a multiple of 32 floats and at least
// XO + P0 + R), and the columns between P0 and it are ghost columns, which no
// kernel reads as data (every load there is masked).  The 2D step kernels store
// zeros there: a line written only in part costs the memory a read-modify-write
// (measured: a quarter longer for the whole write stream of a 16-shot 841-node-
// wide tile pass), whole lines are written straight.
__device__ __forceinline__ int row_store_end(int P0) { return ((XO + P0 + 31) & ~31) - XO; }

// Raw buffer access: a descriptor per array (scalar registers), a 32-bit byte
// offset per lane and a wave-uniform byte offset per row (scalar), so row
// addressing costs no vector instructions.  Accesses past `bytes` read zero
// and are not written; the kernels never make them.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
}

// ---------------------------------------------------------------------------
// 2D leapfrog steps, one or two per launch.
//
// A block owns a tile of TZ rows (T2Z; T2Z_MID or T2Z_SMALL when a launch would
// give the CUs fewer than two tiles each) by TX = 64 - 2R columns; lane l of each wave
// holds column x0 - R + l, so a wave row covers the tile plus an R-wide halo on
// both sides.  u^k is staged in LDS with a 2R halo.  Every thread owns NQ
// consecutive rows of one column and keeps that column in registers (z
// neighbours); x neighbours come from LDS.
//
// One step: u^{k+1} on the tile.  Two steps (temporal blocking): u^{k+1} is
// computed on the tile plus its R-wide halo (the extended region, stored in
// LDS), then u^{k+2} on the tile; both are written.  The halo nodes of u^{k+1}
// are recomputed by the neighbouring tiles with the same arithmetic, so the
// result is bitwise that of two one-step launches, while u^{k-1}, u^k and beta
// are read once for two steps.
//
// Tiles whose staged region lies in the padded box and whose extended region
// is undamped take a path with no clamping, masking or damping terms.  Row
// offsets are wave-uniform (scalar registers); lanes add a 32-bit column
// offset.  Blocks are numbered XCD-aware: the hardware hands block b to XCD b
// mod 8, so logical tile (b mod 8) * (nblocks / 8) + b / 8 gives every XCD a
// contiguous run of tiles whose halos then hit in that XCD's L2.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) const float lds_f32;
// An LDS row address the compiler cannot fold into another row's: the reads of
// one row then pair up with small offsets from it, one address add per row
// instead of one per pair of reads.
__device__ __forceinline__ const lds_f32 *lds_row(const float *p) {
    const lds_f32 *q = (const lds_f32 *)p;
    asm volatile("" : "+v"(q));
    return q;
}

template <int R, int NSTEP, bool FAST, int TZ>
__device__ __forceinline__ void step2d_body(const Layout &L, const Physics &ph, const StepArgs &a, int shot, int tile,
                                            int x0, int z0, float (*U)[64 + 2 * R], float (*V)[64 + 2 * R]) {
#pragma clang fp contract(off)
    constexpr int TX = t2x(R);
    constexpr int SH = TZ + 4 * R;            // staged rows of u^k
    constexpr int NQ = TZ / 4;                // rows per thread
    constexpr int NS = (SH + 3) / 4;          // staged rows per thread
    constexpr int NH = NSTEP == 2 ? R / 2 : 0;   // extended-region halo rows per thread (2R rows / 4 waves)
    constexpr int MAPN = 64 * (TZ + 2 * R);   // nodes of one injection map
    const int lx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int G0 = (int)L.G[0], P0 = (int)L.P[0], P2 = (int)L.P[2];
    const uint32_t span = (uint32_t)(L.shot_floats * 4);
    const int64_t so = shot * L.shot_floats + XO;
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.cur + so, span), rp = buf_rsrc(a.prev + so, span);
    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(a.beta + XO, span);
    auto rowoff = [&](int z) { return (uint32_t)(z + R) * (uint32_t)G0 * 4u; };   // byte offset of padded row z (< 2^32)

    // stage u^k, rows z0 - 2R .. z0 + TZ + 2R - 1, columns x0 - 2R .. x0 + TX + 2R - 1
    const int sx = x0 - 2 * R + lx, sx2 = sx + 64;
    const bool sxin = sx >= 0 && sx < P0, sxin2 = lx < 2 * R && sx2 < P0;
    const uint32_t ox1 = 4u * (uint32_t)(FAST ? sx : clampi(sx, 0, P0 - 1));
    const uint32_t ox2 = 4u * (uint32_t)(FAST ? (lx < 2 * R ? sx2 : sx) : clampi(sx2, 0, P0 - 1));
    float t[NS], t2[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = w + 4 * i, gz = z0 - 2 * R + row;
        const bool zin = FAST || (row < SH && gz >= 0 && gz < P2);
        const uint32_t ro = rowoff(FAST ? (row < SH ? gz : z0) : clampi(gz, 0, P2 - 1));
        const float v1 = buf_load(rc, ox1, ro), v2 = buf_load(rc, ox2, ro);
        t[i] = (zin && (FAST || sxin)) ? v1 : 0.0f;
        t2[i] = (zin && (FAST || sxin2)) ? v2 : 0.0f;
    }
    // u^{k-1} and beta at this thread's nodes: column x, rows zb .. zb + NQ - 1
    const int x = x0 - R + lx;
    const bool xin = x >= 0 && x < P0;
    const uint32_t ox = 4u * (uint32_t)(FAST ? x : clampi(x, 0, P0 - 1));
    const int zb = z0 + w * NQ;
    float p[NQ], b[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int z = zb + q;
        const uint32_t ro = rowoff(FAST ? z : clampi(z, 0, P2 - 1));
        const float pv = buf_load(rp, ox, ro), bv = buf_load(rb, ox, ro);
        const bool ok = FAST || (xin && z < P2);
        p[q] = ok ? pv : 0.0f;
        b[q] = ok ? bv : 0.0f;
    }
    // the same at the extended region's halo rows (two steps)
    float hp[NH > 0 ? NH : 1], hb[NH > 0 ? NH : 1];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int hr = w + 4 * i;   // 0 .. 2R-1
        const int z = hr < R ? z0 - R + hr : z0 + TZ + (hr - R);
        const uint32_t ro = rowoff(FAST ? z : clampi(z, 0, P2 - 1));
        const float pv = buf_load(rp, ox, ro), bv = buf_load(rb, ox, ro);
        const bool ok = FAST || (xin && z >= 0 && z < P2);
        hp[i] = ok ? pv : 0.0f;
        hb[i] = ok ? bv : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = w + 4 * i;
        if (row < SH) {
            U[row][lx] = t[i];
            if (lx < 2 * R) U[row][64 + lx] = t2[i];
        }
    }

    // point sources: each node looks up its segment in the tile's dense map
    float s1[NQ], s2[NQ], sh[NH > 0 ? NH : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s1[q] = s2[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < NH; ++i) sh[i] = 0.0f;
    if (a.inject) {
        const int map = a.inj.tile_dense[tile];
        if (map >= 0) {
            const int32_t *dm = a.inj.dense + (int64_t)map * MAPN + lx;
            const float *amp = a.amp.ptr + shot * a.amp.shot_stride;
            const float *amp1 = amp + (int64_t)a.k * a.amp.k_stride;
            const float *amp2 = amp + (int64_t)a.k2 * a.amp.k_stride;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int sg = dm[(w * NQ + q + R) * 64];
                if (sg >= 0) {
                    s1[q] = segment_value(a.inj, amp1, a.amp.scale, sg);
                    if (NSTEP == 2) s2[q] = segment_value(a.inj, amp2, a.amp.scale, sg);
                }
            }
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int hr = w + 4 * i;
                const int sg = dm[(hr < R ? hr : TZ + hr) * 64];
                if (sg >= 0) sh[i] = segment_value(a.inj, amp1, a.amp.scale, sg);
            }
        }
    }
    __syncthreads();

    // first step on this thread's rows
    const float hx = FAST ? 0.0f : layer_frac2(x, (int)L.n[0], L.nb, ph.inv_nb);
    // lanes on tile columns; past the box they store zeros up to the end of the
    // row's last 128-byte line (ghost columns), so the memory sees whole lines
    // instead of a partial one that costs a read-modify-write
    const bool act = lx >= R && lx < R + TX && (FAST || x < row_store_end(P0));
    const uint32_t os = 4u * (uint32_t)x;   // unclamped: x >= 0 on tile lanes
    const __amdgpu_buffer_rsrc_t rn1 = buf_rsrc(a.next + so, span);
    float c[NQ], hd[NQ];
    {
        float col[NQ + 2 * R];
#pragma unroll
        for (int i = 0; i < NQ + 2 * R; ++i) col[i] = U[w * NQ + R + i][lx + R];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int z = zb + q, ur = w * NQ + q + 2 * R;
            const float cv = col[q + R];
            float lap = 2.0f * ph.c[0] * cv;
            const lds_f32 *up = lds_row(&U[ur][lx]);
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap = __builtin_fmaf(ph.c[k], (up[R - k] + up[R + k]) + (col[q + R - k] + col[q + R + k]), lap);
            float v;
            if (FAST) {
                v = leapfrog0(cv, p[q], b[q], lap, s1[q]);
            } else {
                hd[q] = ph.hd_max * (hx + layer_frac2(z, (int)L.n[2], L.nb, ph.inv_nb));
                v = (xin && z < P2) ? leapfrog(cv, p[q], b[q], lap, s1[q], hd[q]) : 0.0f;
            }
            if (NSTEP == 1) {
                if (act && (FAST || z < P2)) buf_store(v, rn1, os, rowoff(z));
            } else {
                V[w * NQ + q + R][lx + R] = v;
            }
            c[q] = cv;
        }
    }
    if (NSTEP == 1) return;

    // first step on the extended region's halo rows
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int hr = w + 4 * i;
        const int z = hr < R ? z0 - R + hr : z0 + TZ + (hr - R);
        const int ur = z - z0 + 2 * R;
        const lds_f32 *up = lds_row(&U[ur][lx]);
        const float cv = up[R];
        float lap = 2.0f * ph.c[0] * cv;
#pragma unroll
        for (int k = 1; k <= R; ++k)
            lap = __builtin_fmaf(ph.c[k], (up[R - k] + up[R + k]) + (U[ur - k][lx + R] + U[ur + k][lx + R]), lap);
        float v;
        if (FAST) {
            v = leapfrog0(cv, hp[i], hb[i], lap, sh[i]);
        } else {
            const float h = ph.hd_max * (hx + layer_frac2(z, (int)L.n[2], L.nb, ph.inv_nb));
            v = (xin && z >= 0 && z < P2) ? leapfrog(cv, hp[i], hb[i], lap, sh[i], h) : 0.0f;
        }
        V[hr < R ? hr : TZ + hr][lx + R] = v;
    }
    __syncthreads();

    // second step on the tile
    const __amdgpu_buffer_rsrc_t rn2 = buf_rsrc(a.next2 + so, span);
    float col[NQ + 2 * R];
#pragma unroll
    for (int i = 0; i < NQ + 2 * R; ++i) col[i] = V[w * NQ + i][lx + R];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int z = zb + q, vr = w * NQ + q + R;
        const float v = col[q + R];
        float lap = 2.0f * ph.c[0] * v;
        // V's rows carry R spare columns on each side, so the idle edge lanes
        // read inside the array (values they never store)
        const lds_f32 *vp = lds_row(&V[vr][lx]);
#pragma unroll
        for (int k = 1; k <= R; ++k)
            lap = __builtin_fmaf(ph.c[k], (vp[R - k] + vp[R + k]) + (col[q + R - k] + col[q + R + k]), lap);
        if (act && (FAST || z < P2)) {
            const uint32_t ro = rowoff(z);
            buf_store(v, rn1, os, ro);
            buf_store(FAST ? leapfrog0(v, c[q], b[q], lap, s2[q]) : (xin ? leapfrog(v, c[q], b[q], lap, s2[q], hd[q]) : 0.0f),
                      rn2, os, ro);
        }
    }
}

template <int R, int NSTEP, int TZ>
__global__ __launch_bounds__(256) void k_step2d(const Layout L, const Physics ph, const StepArgs a) {
    constexpr int TX = t2x(R);
    __shared__ float U[TZ + 4 * R][64 + 2 * R];
    __shared__ float V[NSTEP == 2 ? TZ + 2 * R : 1][64 + 2 * R];
    const int ntx = (int)L.ntiles[0], ntz = (int)L.ntiles[2], nsp = ntx * ntz;
    const int lid = xcd_logical_block(nsp * L.S);
    if (lid < 0) return;
    // Shots are split into eight equal groups when they divide evenly, one
    // group per XCD; inside a group the shots of one spatial tile are adjacent,
    // so the tile's beta is fetched once into that XCD's L2 for all of them.
    const int sg = L.S % 8 == 0 ? L.S / 8 : 1;
    const int grp = lid / (nsp * sg), rem = lid - grp * (nsp * sg);
    const int sp = rem / sg, shot = grp * sg + (rem - sp * sg);
    const int bx = sp % ntx, bz = sp / ntx;
    const int x0 = bx * TX, z0 = bz * TZ, nb = L.nb;
    const bool fast = x0 - 2 * R >= 0 && z0 - 2 * R >= 0 && x0 + TX + 2 * R <= (int)L.P[0] &&
                      z0 + TZ + 2 * R <= (int)L.P[2] && x0 - R >= nb && z0 - R >= nb &&
                      x0 + TX + R <= nb + (int)L.n[0] && z0 + TZ + R <= nb + (int)L.n[2];
    const int tile = (shot * ntz + bz) * ntx + bx;
    if (fast) step2d_body<R, NSTEP, true, TZ>(L, ph, a, shot, tile, x0, z0, U, V);
    else step2d_body<R, NSTEP, false, TZ>(L, ph, a, shot, tile, x0, z0, U, V);

    const int per_shot = ntx * ntz;
    if (a.do_sample) sample_points<4>(L, a.cur + shot * L.shot_floats, a.k, a.smp, shot, bz * ntx + bx, per_shot);
    if (a.sample_prev) sample_points<4>(L, a.prev + shot * L.shot_floats, a.kp, a.smp, shot, bz * ntx + bx, per_shot);
    if (a.sample_prev2) sample_points<4>(L, a.prev2 + shot * L.shot_floats, a.kp2, a.smp, shot, bz * ntx + bx, per_shot);
}

// ---------------------------------------------------------------------------
// 2D leapfrog, three steps per launch (deeper temporal blocking).
//
// A block owns a tile of TZ rows by TX = 64 - 4R columns; lane l of each wave
// holds column x0 - 2R + l.  Step 1 gives u^{k+1} on the tile plus a 2R-wide
// halo (rows z0 - 2R .. z0 + TZ + 2R - 1, all 64 lanes), step 2 gives u^{k+2}
// on the tile plus an R-wide halo, step 3 gives u^{k+3} on the tile.  u^k is
// staged in LDS with a 3R halo (U); u^{k+1} goes to LDS (V); u^{k+2} is written
// over U once step 1 has read it.  Each thread owns NQ consecutive tile rows
// of its column in all three steps (z neighbours from a register copy of the
// column), R/2 rows of step 2's halo for steps 1 and 2, and R/2 rows of step
// 1's own halo.  u^{k-1}, u^k and beta are read once for three steps; the
// three new levels are written on the tile.  Every node is computed with the
// one-step arithmetic, so the result is bitwise that of three one-step
// launches.  Injection maps cover the first step's region (64 x (TZ + 4R)
// nodes from (-2R, -2R)).
// ---------------------------------------------------------------------------
template <int R, bool FAST, int TZ>
__device__ __forceinline__ void step2d3_body(const Layout &L, const Physics &ph, const StepArgs &a, int shot,
                                             int tile, int x0, int z0, float (*U)[64 + 2 * R],
                                             float (*V)[64 + 2 * R]) {
#pragma clang fp contract(off)
    constexpr int TX = t3x(R);
    constexpr int SH = TZ + 6 * R;            // staged rows of u^k (from z0 - 3R)
    constexpr int NQ = TZ / 4;                // tile rows per thread
    constexpr int NS = (SH + 3) / 4;          // staged rows per thread
    constexpr int NH = R / 2;                 // halo rows per thread, per halo band (2R rows / 4 waves)
    constexpr int MAPN = 64 * (TZ + 4 * R);   // nodes of one injection map
    const int lx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int G0 = (int)L.G[0], P0 = (int)L.P[0], P2 = (int)L.P[2];
    const uint32_t span = (uint32_t)(L.shot_floats * 4);
    const int64_t so = shot * L.shot_floats + XO;
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.cur + so, span), rp = buf_rsrc(a.prev + so, span);
    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(a.beta + XO, span);
    auto rowoff = [&](int z) { return (uint32_t)(z + R) * (uint32_t)G0 * 4u; };   // byte offset of padded row z (< 2^32)

    // stage u^k, rows z0 - 3R .. z0 + TZ + 3R - 1, columns x0 - 3R .. x0 + TX + 3R - 1
    const int sx = x0 - 3 * R + lx, sx2 = sx + 64;
    const bool sxin = sx >= 0 && sx < P0, sxin2 = lx < 2 * R && sx2 < P0;
    const uint32_t ox1 = 4u * (uint32_t)(FAST ? sx : clampi(sx, 0, P0 - 1));
    const uint32_t ox2 = 4u * (uint32_t)(FAST ? (lx < 2 * R ? sx2 : sx) : clampi(sx2, 0, P0 - 1));
    float t[NS], t2[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = w + 4 * i, gz = z0 - 3 * R + row;
        const bool zin = FAST || (row < SH && gz >= 0 && gz < P2);
        const uint32_t ro = rowoff(FAST ? (row < SH ? gz : z0) : clampi(gz, 0, P2 - 1));
        const float v1 = buf_load(rc, ox1, ro), v2 = buf_load(rc, ox2, ro);
        t[i] = (zin && (FAST || sxin)) ? v1 : 0.0f;
        t2[i] = (zin && (FAST || sxin2)) ? v2 : 0.0f;
    }
    // u^{k-1} and beta at this thread's nodes: column x; tile rows zb .. zb + NQ - 1,
    // step 2's halo rows (hz2) and step 1's own halo rows (hz1)
    const int x = x0 - 2 * R + lx;
    const bool xin = x >= 0 && x < P0;
    const uint32_t ox = 4u * (uint32_t)(FAST ? x : clampi(x, 0, P0 - 1));
    const int zb = z0 + w * NQ;
    auto hz2 = [&](int i) { const int hr = w + 4 * i; return hr < R ? z0 - R + hr : z0 + TZ + (hr - R); };
    auto hz1 = [&](int i) { const int hr = w + 4 * i; return hr < R ? z0 - 2 * R + hr : z0 + TZ + R + (hr - R); };
    float p[NQ], b[NQ], hp2[NH], hb2[NH], hp1[NH], hb1[NH];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int z = zb + q;
        const uint32_t ro = rowoff(FAST ? z : clampi(z, 0, P2 - 1));
        const float pv = buf_load(rp, ox, ro), bv = buf_load(rb, ox, ro);
        const bool ok = FAST || (xin && z < P2);
        p[q] = ok ? pv : 0.0f;
        b[q] = ok ? bv : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int z2 = hz2(i), z1 = hz1(i);
        const uint32_t ro2 = rowoff(FAST ? z2 : clampi(z2, 0, P2 - 1)), ro1 = rowoff(FAST ? z1 : clampi(z1, 0, P2 - 1));
        const float pv2 = buf_load(rp, ox, ro2), bv2 = buf_load(rb, ox, ro2);
        const float pv1 = buf_load(rp, ox, ro1), bv1 = buf_load(rb, ox, ro1);
        const bool ok2 = FAST || (xin && z2 >= 0 && z2 < P2), ok1 = FAST || (xin && z1 >= 0 && z1 < P2);
        hp2[i] = ok2 ? pv2 : 0.0f;
        hb2[i] = ok2 ? bv2 : 0.0f;
        hp1[i] = ok1 ? pv1 : 0.0f;
        hb1[i] = ok1 ? bv1 : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = w + 4 * i;
        if (row < SH) {
            U[row][lx] = t[i];
            if (lx < 2 * R) U[row][64 + lx] = t2[i];
        }
    }

    // point sources: each node looks up its segment in the tile's dense map
    // (map row = z - (z0 - 2R), map column = lane)
    float s1[NQ], s2[NQ], s3[NQ], sh21[NH], sh22[NH], sh1[NH];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s1[q] = s2[q] = s3[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < NH; ++i) sh21[i] = sh22[i] = sh1[i] = 0.0f;
    if (a.inject) {
        const int map = a.inj.tile_dense[tile];
        if (map >= 0) {
            const int32_t *dm = a.inj.dense + (int64_t)map * MAPN + lx;
            const float *amp = a.amp.ptr + shot * a.amp.shot_stride;
            const float *amp1 = amp + (int64_t)a.k * a.amp.k_stride;
            const float *amp2 = amp + (int64_t)a.k2 * a.amp.k_stride;
            const float *amp3 = amp + (int64_t)a.k3 * a.amp.k_stride;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int sg = dm[(w * NQ + q + 2 * R) * 64];
                if (sg >= 0) {
                    s1[q] = segment_value(a.inj, amp1, a.amp.scale, sg);
                    s2[q] = segment_value(a.inj, amp2, a.amp.scale, sg);
                    s3[q] = segment_value(a.inj, amp3, a.amp.scale, sg);
                }
            }
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int sg2 = dm[(hz2(i) - (z0 - 2 * R)) * 64], sg1 = dm[(hz1(i) - (z0 - 2 * R)) * 64];
                if (sg2 >= 0) {
                    sh21[i] = segment_value(a.inj, amp1, a.amp.scale, sg2);
                    sh22[i] = segment_value(a.inj, amp2, a.amp.scale, sg2);
                }
                if (sg1 >= 0) sh1[i] = segment_value(a.inj, amp1, a.amp.scale, sg1);
            }
        }
    }
    __syncthreads();

    const float hx = FAST ? 0.0f : layer_frac2(x, (int)L.n[0], L.nb, ph.inv_nb);
    auto hdz = [&](int z) { return ph.hd_max * (hx + layer_frac2(z, (int)L.n[2], L.nb, ph.inv_nb)); };
    // one node of any step: centre, x neighbours of its LDS row, z neighbour pairs zs[k]
    auto node = [&](float cv, const lds_f32 *row, const float *zs, float prev, float beta, float src, int z) {
        float lap = 2.0f * ph.c[0] * cv;
#pragma unroll
        for (int k = 1; k <= R; ++k) lap = __builtin_fmaf(ph.c[k], (row[R - k] + row[R + k]) + zs[k], lap);
        if (FAST) return leapfrog0(cv, prev, beta, lap, src);
        return (xin && z >= 0 && z < P2) ? leapfrog(cv, prev, beta, lap, src, hdz(z)) : 0.0f;
    };

    // step 1: u^{k+1} on rows z0 - 2R .. z0 + TZ + 2R - 1 into V (row z - (z0 - 2R))
    float c[NQ], v1[NQ], hc2[NH];
    {
        float col[NQ + 2 * R];
#pragma unroll
        for (int i = 0; i < NQ + 2 * R; ++i) col[i] = U[w * NQ + 2 * R + i][lx + R];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float zs[R + 1];
#pragma unroll
            for (int k = 1; k <= R; ++k) zs[k] = col[q + R - k] + col[q + R + k];
            const float cv = col[q + R];
            const float v = node(cv, lds_row(&U[w * NQ + q + 3 * R][lx]), zs, p[q], b[q], s1[q], zb + q);
            V[w * NQ + q + 2 * R][lx + R] = v;
            c[q] = cv;
            v1[q] = v;
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) {
#pragma unroll
            for (int band = 0; band < 2; ++band) {   // step 2's halo rows, then step 1's own
                const int z = band == 0 ? hz2(i) : hz1(i);
                const int ur = z - (z0 - 3 * R);
                float zs[R + 1];
#pragma unroll
                for (int k = 1; k <= R; ++k) zs[k] = U[ur - k][lx + R] + U[ur + k][lx + R];
                const float cv = U[ur][lx + R];
                const float v = band == 0 ? node(cv, lds_row(&U[ur][lx]), zs, hp2[i], hb2[i], sh21[i], z)
                                          : node(cv, lds_row(&U[ur][lx]), zs, hp1[i], hb1[i], sh1[i], z);
                V[z - (z0 - 2 * R)][lx + R] = v;
                if (band == 0) hc2[i] = cv;
            }
        }
    }
    __syncthreads();

    // step 2: u^{k+2} on rows z0 - R .. z0 + TZ + R - 1, written over U (row z - (z0 - R));
    // lanes outside R .. 63 - R read V's spare columns and are never used
    float v2[NQ];
    {
        float col[NQ + 2 * R];
#pragma unroll
        for (int i = 0; i < NQ + 2 * R; ++i) col[i] = V[w * NQ + R + i][lx + R];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float zs[R + 1];
#pragma unroll
            for (int k = 1; k <= R; ++k) zs[k] = col[q + R - k] + col[q + R + k];
            const float v = node(col[q + R], lds_row(&V[w * NQ + q + 2 * R][lx]), zs, c[q], b[q], s2[q], zb + q);
            U[w * NQ + q + R][lx + R] = v;
            v2[q] = v;
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int z = hz2(i), vr = z - (z0 - 2 * R);
            float zs[R + 1];
#pragma unroll
            for (int k = 1; k <= R; ++k) zs[k] = V[vr - k][lx + R] + V[vr + k][lx + R];
            U[z - (z0 - R)][lx + R] = node(V[vr][lx + R], lds_row(&V[vr][lx]), zs, hc2[i], hb2[i], sh22[i], z);
        }
    }
    __syncthreads();

    // step 3: u^{k+3} on the tile; the three new levels are written there
    // lanes on tile columns, and past the box up to the end of the row's last
    // 128-byte line (zeros into ghost columns, as in the two-step kernel)
    const bool act = lx >= 2 * R && lx < 2 * R + TX && (FAST || x < row_store_end(P0));
    const uint32_t os = 4u * (uint32_t)x;
    const __amdgpu_buffer_rsrc_t rn1 = buf_rsrc(a.next + so, span), rn2 = buf_rsrc(a.next2 + so, span);
    const __amdgpu_buffer_rsrc_t rn3 = buf_rsrc(a.next3 + so, span);
    float col[NQ + 2 * R];
#pragma unroll
    for (int i = 0; i < NQ + 2 * R; ++i) col[i] = U[w * NQ + i][lx + R];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int z = zb + q;
        float zs[R + 1];
#pragma unroll
        for (int k = 1; k <= R; ++k) zs[k] = col[q + R - k] + col[q + R + k];
        const float v3 = node(col[q + R], lds_row(&U[w * NQ + q + R][lx]), zs, v1[q], b[q], s3[q], z);
        if (act && (FAST || z < P2)) {
            const uint32_t ro = rowoff(z);
            buf_store(v1[q], rn1, os, ro);
            buf_store(v2[q], rn2, os, ro);
            buf_store(v3, rn3, os, ro);
        }
    }
}

template <int R, int TZ>
__global__ __launch_bounds__(256) void k_step2d3(const Layout L, const Physics ph, const StepArgs a) {
    constexpr int TX = t3x(R);
    __shared__ float U[TZ + 6 * R][64 + 2 * R];
    __shared__ float V[TZ + 4 * R][64 + 2 * R];
    const int ntx = (int)L.ntiles[0], ntz = (int)L.ntiles[2], nsp = ntx * ntz;
    const int lid = xcd_logical_block(nsp * L.S);
    if (lid < 0) return;
    // shot groups per XCD and shot-adjacent tiles, as in k_step2d
    const int sg = L.S % 8 == 0 ? L.S / 8 : 1;
    const int grp = lid / (nsp * sg), rem = lid - grp * (nsp * sg);
    const int sp = rem / sg, shot = grp * sg + (rem - sp * sg);
    const int bx = sp % ntx, bz = sp / ntx;
    const int x0 = bx * TX, z0 = bz * TZ, nb = L.nb;
    const bool fast = x0 - 3 * R >= 0 && z0 - 3 * R >= 0 && x0 + TX + 3 * R <= (int)L.P[0] &&
                      z0 + TZ + 3 * R <= (int)L.P[2] && x0 - 2 * R >= nb && z0 - 2 * R >= nb &&
                      x0 + TX + 2 * R <= nb + (int)L.n[0] && z0 + TZ + 2 * R <= nb + (int)L.n[2];
    const int tile = (shot * ntz + bz) * ntx + bx;
    if (fast) step2d3_body<R, true, TZ>(L, ph, a, shot, tile, x0, z0, U, V);
    else step2d3_body<R, false, TZ>(L, ph, a, shot, tile, x0, z0, U, V);

    const int per_shot = ntx * ntz, bis = bz * ntx + bx;
    if (a.do_sample) sample_points<4>(L, a.cur + shot * L.shot_floats, a.k, a.smp, shot, bis, per_shot);
    if (a.sample_prev) sample_points<4>(L, a.prev + shot * L.shot_floats, a.kp, a.smp, shot, bis, per_shot);
    if (a.sample_prev2) sample_points<4>(L, a.prev2 + shot * L.shot_floats, a.kp2, a.smp, shot, bis, per_shot);
}

// ---------------------------------------------------------------------------
// 3D leapfrog step.  Block = 64 x 4 threads over a 64 (x) by 8 (y) column of
// outputs (two y rows per thread) that marches T3Z planes in z.  z neighbours
// come from per-thread register queues of 2R+1 values; x/y neighbours from
// the current plane staged in LDS (double-buffered, one barrier per plane).
// The halo of the next plane is prefetched into registers while the current
// plane is computed.  Every lane's byte offsets within a plane are fixed for
// the whole march and the plane offset is wave-uniform, so the raw buffer
// accesses need no vector address arithmetic.  Columns whose halo lies in
// the padded box and whose nodes are undamped take a path without clamping,
// masking or damping terms.  u^{k-1}, beta and u^{k+1} are streamed past the
// caches (nontemporal).  Logical blocks are numbered XCD-aware as in 2D.
// ---------------------------------------------------------------------------
constexpr int kBufNT = 2;   // cache-policy bit of a streamed (nontemporal) buffer access

// Arguments of the 3D step kernels as one kernel parameter, so the step
// arguments sit at a known offset of the kernel-argument segment.
struct Step3DArgs {
    Layout L;
    Physics ph;
    StepArgs a;
};
typedef const __attribute__((address_space(4))) StepArgs *KernargStep;

// The step arguments read straight from the kernel-argument segment through a
// pointer the compiler cannot see through: the source-injection tables are
// rarely needed, and loading them only where they are used keeps them out of
// the scalar registers of the march.
__device__ __forceinline__ KernargStep kernarg_step_args() {
    KernargStep p = (KernargStep)((const __attribute__((address_space(4))) char *)__builtin_amdgcn_kernarg_segment_ptr() +
                                  offsetof(Step3DArgs, a));
    asm volatile("" : "+s"(p));
    return p;
}

// Source term of padded node (x, y, z) inside the box, looked up in the
// injection map of the two-step kernel's tile that owns the node.
template <int R>
__device__ __forceinline__ float source_3d(const Layout &L, KernargStep ka, int shot, int x, int y, int z) {
    constexpr int TX = t2x(R);
    InjectTables inj;
    inj.tile_dense = ka->inj.tile_dense;
    inj.dense = ka->inj.dense;
    inj.seg_ent = ka->inj.seg_ent;
    inj.ent_idx = ka->inj.ent_idx;
    inj.ent_w = ka->inj.ent_w;
    inj.col_z = nullptr;
    const int tx = x / TX, ty = y / T3Y2;
    const int map = inj.tile_dense[(((int64_t)shot * L.ntiles[2] + z) * L.ntiles[1] + ty) * L.ntiles[0] + tx];
    if (map < 0) return 0.0f;
    const int sg = inj.dense[(int64_t)map * (64 * (T3Y2 + 2 * R)) + (y - ty * T3Y2 + R) * 64 + (x - tx * TX + R)];
    const float *amp = ka->amp.ptr + shot * ka->amp.shot_stride + (int64_t)ka->k * ka->amp.k_stride;
    return sg >= 0 ? segment_value(inj, amp, ka->amp.scale, sg) : 0.0f;
}

template <int R, bool FAST>
__device__ __forceinline__ void step3d_body(const Layout &L, const Physics &ph, const StepArgs &a, int shot, int bx,
                                            int by, int zc, float (*plane_t)[T3Y + 2 * R][T3X + 2 * R]) {
#pragma clang fp contract(off)
    constexpr int W = T3X + 2 * R;
    const int lx = threadIdx.x & 63;
    const int ly = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int x0 = bx * T3X, y0 = by * T3Y, zc0 = zc * T3Z;
    const int x = x0 + lx;
    const int ya = y0 + ly, yb = y0 + ly + 4;            // the two y rows of this thread
    const int G0 = (int)L.G[0], PL = (int)(L.G[0] * L.G[1]);
    const int P0 = (int)L.P[0], P1 = (int)L.P[1], P2 = (int)L.P[2], oy = (int)L.oy;
    const uint32_t span = (uint32_t)(L.shot_floats * 4);
    const int64_t so = shot * L.shot_floats + XO;
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.cur + so, span), rp = buf_rsrc(a.prev + so, span);
    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(a.beta + XO, span), rn = buf_rsrc(a.next + so, span);
    auto plane = [&](int z) { return (uint32_t)((FAST ? z : clampi(z, 0, P2 - 1)) + R) * (uint32_t)PL * 4u; };
    auto lane = [&](int y, int xx) {   // byte offset of (y, x) within a plane
        return 4u * (uint32_t)(((FAST ? y : clampi(y, 0, P1 - 1)) + oy) * G0 + (FAST ? xx : clampi(xx, 0, P0 - 1)));
    };

    const bool oa = FAST || (x < P0 && ya < P1), ob = FAST || (x < P0 && yb < P1);   // columns inside the box
    const uint32_t va = lane(ya, x), vb = lane(yb, x);

    // halo of a plane: staged rows ly and T3Y + R + ly (y0 - R + ly, y0 + T3Y + ly) for
    // ly < R, all 64 + 2R columns; the centre rows R + ly and R + 4 + ly only their
    // x-halo columns.
    const int hy0 = y0 - R + ly, hy1 = y0 + T3Y + ly;
    const int hxa = x0 - R + lx;                     // columns 0..63 of the staged row
    const int hxb = x0 - R + 64 + lx;                // columns 64..71 (lanes < 2R)
    const int hxc = lx < R ? x0 - R + lx : x0 + T3X + (lx - R);  // x-halo of the centre rows (lanes < 2R)
    const bool y0ok = FAST || (hy0 >= 0 && hy0 < P1), y1ok = FAST || hy1 < P1;
    const bool xaok = FAST || (hxa >= 0 && hxa < P0);
    const bool xbok = lx < 2 * R && (FAST || hxb < P0), xcok = lx < 2 * R && (FAST || (hxc >= 0 && hxc < P0));
    const uint32_t h0 = lane(hy0, hxa), h1 = lane(hy0, lx < 2 * R ? hxb : hxa), h2 = lane(hy1, hxa);
    const uint32_t h3 = lane(hy1, lx < 2 * R ? hxb : hxa);
    const uint32_t h4 = lane(ya, lx < 2 * R ? hxc : x), h5 = lane(yb, lx < 2 * R ? hxc : x);
    const bool h4ok = xcok && (FAST || ya < P1), h5ok = xcok && (FAST || yb < P1);
    auto load_halo = [&](int z, float h[6]) {
        const uint32_t zo = plane(z);
        const float v0 = buf_load(rc, h0, zo), v1 = buf_load(rc, h1, zo), v2 = buf_load(rc, h2, zo);
        const float v3 = buf_load(rc, h3, zo), v4 = buf_load(rc, h4, zo), v5 = buf_load(rc, h5, zo);
        h[0] = (y0ok && xaok) ? v0 : 0.0f;
        h[1] = (y0ok && xbok) ? v1 : 0.0f;
        h[2] = (y1ok && xaok) ? v2 : 0.0f;
        h[3] = (y1ok && xbok) ? v3 : 0.0f;
        h[4] = h4ok ? v4 : 0.0f;
        h[5] = h5ok ? v5 : 0.0f;
    };

    float qa[2 * R + 1], qb[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) {
        const int z = zc0 - R + i;
        const bool zin = FAST || (z >= 0 && z < P2);
        const uint32_t zo = plane(z);
        const float va_ = buf_load(rc, va, zo), vb_ = buf_load(rc, vb, zo);
        qa[i] = (oa && zin) ? va_ : 0.0f;
        qb[i] = (ob && zin) ? vb_ : 0.0f;
    }
    float h[6];
    load_halo(zc0, h);
    // planes with source nodes in the two-step kernel's tile columns this
    // block overlaps (its 64 columns span at most two, its 8 rows one)
    int zlo = 1, zhi = 0;
    if (a.inject) {
        const int ty = y0 / T3Y2, tx0 = x0 / t2x(R), tx1 = min(x0 + T3X - 1, P0 - 1) / t2x(R);
        const int c0 = (shot * (int)L.ntiles[1] + ty) * (int)L.ntiles[0] + tx0, c1 = c0 + (tx1 - tx0);
        zlo = __builtin_amdgcn_readfirstlane(min(a.inj.col_z[2 * c0], a.inj.col_z[2 * c1]));
        zhi = __builtin_amdgcn_readfirstlane(max(a.inj.col_z[2 * c0 + 1], a.inj.col_z[2 * c1 + 1]));
    }
    const float hx = FAST ? 0.0f : layer_frac2(x, (int)L.n[0], L.nb, ph.inv_nb);
    const float hxy_a = FAST ? 0.0f : hx + layer_frac2(ya, (int)L.n[1], L.nb, ph.inv_nb);
    const float hxy_b = FAST ? 0.0f : hx + layer_frac2(yb, (int)L.n[1], L.nb, ph.inv_nb);

    // the column's own loads of a plane: u^k at z + R, u^{k-1} and beta at z;
    // issued one plane ahead, like the halo, so they overlap a plane of compute
    float nq[2], np[2], nbt[2];
    auto load_column = [&](int z) {
        const uint32_t zo = plane(z), zr_o = plane(z + R);
        nq[0] = buf_load(rc, va, zr_o);
        nq[1] = buf_load(rc, vb, zr_o);
        np[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, (int)va, (int)zo, kBufNT));
        np[1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, (int)vb, (int)zo, kBufNT));
        nbt[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, (int)va, (int)zo, kBufNT));
        nbt[1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, (int)vb, (int)zo, kBufNT));
    };
    load_column(zc0);

    for (int lz = 0; lz < T3Z; ++lz) {
        const int z = zc0 + lz;
        if (!FAST && z >= P2) break;
        const uint32_t zo = plane(z);
        const bool zr = FAST || z + R < P2;
        qa[2 * R] = (oa && zr) ? nq[0] : 0.0f;
        qb[2 * R] = (ob && zr) ? nq[1] : 0.0f;
        const float pa = oa ? np[0] : 0.0f, pb = ob ? np[1] : 0.0f, ba = oa ? nbt[0] : 0.0f, bb = ob ? nbt[1] : 0.0f;

        float(*pt)[W] = plane_t[lz & 1];
        if (R >= 4 || ly < R) {   // the R halo rows on each side: one per wave when R = 4
            pt[ly][lx] = h[0];
            if (lx < 2 * R) pt[ly][64 + lx] = h[1];
            pt[T3Y + R + ly][lx] = h[2];
            if (lx < 2 * R) pt[T3Y + R + ly][64 + lx] = h[3];
        }
        pt[R + ly][R + lx] = qa[R];
        pt[R + 4 + ly][R + lx] = qb[R];
        if (lx < 2 * R) {
            const int hc = lx < R ? lx : T3X + lx;   // column in the staged row
            pt[R + ly][hc] = h[4];
            pt[R + 4 + ly][hc] = h[5];
        }
        float sa = 0.0f, sbv = 0.0f;   // point-source terms of this thread's two nodes
        if (z >= zlo && z <= zhi) {
            const KernargStep ka = kernarg_step_args();
            if (oa) sa = source_3d<R>(L, ka, shot, x, ya, z);
            if (ob) sbv = source_3d<R>(L, ka, shot, x, yb, z);
        }
        __syncthreads();
        if (lz + 1 < T3Z && (FAST || z + 1 < P2)) {   // prefetch, overlaps the compute below
            load_halo(z + 1, h);
            load_column(z + 1);
        }

        float lapa = 3.0f * ph.c[0] * qa[R], lapb = 3.0f * ph.c[0] * qb[R];
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lapa = __builtin_fmaf(ph.c[k], (pt[R + ly][R + lx - k] + pt[R + ly][R + lx + k]) +
                                               (pt[R + ly - k][R + lx] + pt[R + ly + k][R + lx]) + (qa[R - k] + qa[R + k]),
                                  lapa);
            lapb = __builtin_fmaf(ph.c[k], (pt[R + 4 + ly][R + lx - k] + pt[R + 4 + ly][R + lx + k]) +
                                               (pt[R + 4 + ly - k][R + lx] + pt[R + 4 + ly + k][R + lx]) + (qb[R - k] + qb[R + k]),
                                  lapb);
        }
        float na, nb_;
        if (FAST) {
            na = leapfrog0(qa[R], pa, ba, lapa, sa);
            nb_ = leapfrog0(qb[R], pb, bb, lapb, sbv);
        } else {
            const float hz = layer_frac2(z, (int)L.n[2], L.nb, ph.inv_nb);
            na = leapfrog(qa[R], pa, ba, lapa, sa, ph.hd_max * (hxy_a + hz));
            nb_ = leapfrog(qb[R], pb, bb, lapb, sbv, ph.hd_max * (hxy_b + hz));
        }
        if (oa) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, na), rn, (int)va, (int)zo, kBufNT);
        if (ob) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, nb_), rn, (int)vb, (int)zo, kBufNT);
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) {
            qa[i] = qa[i + 1];
            qb[i] = qb[i + 1];
        }
    }
}

template <int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_step3d(const Step3DArgs P) {
    const Layout &L = P.L;
    const Physics &ph = P.ph;
    const StepArgs &a = P.a;
    __shared__ float plane_t[2][T3Y + 2 * R][T3X + 2 * R];
    const int ntx = (int)((L.P[0] + T3X - 1) / T3X), nty = (int)((L.P[1] + T3Y - 1) / T3Y);
    const int nzc = (int)((L.P[2] + T3Z - 1) / T3Z);
    const int lid = xcd_logical_block(ntx * nty * nzc * L.S);
    if (lid < 0) return;
    const int bx = lid % ntx, by = (lid / ntx) % nty, zc = (lid / (ntx * nty)) % nzc, shot = lid / (ntx * nty * nzc);
    const int x0 = bx * T3X, y0 = by * T3Y, zc0 = zc * T3Z, nb = L.nb;
    // interior column: every node undamped and every read inside the padded box
    const bool fast = x0 - R >= nb && x0 + T3X + R <= nb + (int)L.n[0] && y0 - R >= nb &&
                      y0 + T3Y + R <= nb + (int)L.n[1] && zc0 - R >= nb && zc0 + T3Z + R <= nb + (int)L.n[2];
    // sampling first: the launch's inputs are read-only
    const int per_shot = ntx * nty * nzc, bis = (zc * nty + by) * ntx + bx;
    if (a.do_sample) sample_points<8>(L, a.cur + shot * L.shot_floats, a.k, a.smp, shot, bis, per_shot);
    if (a.sample_prev) sample_points<8>(L, a.prev + shot * L.shot_floats, a.kp, a.smp, shot, bis, per_shot);
    if (fast) step3d_body<R, true>(L, ph, a, shot, bx, by, zc, plane_t);
    else step3d_body<R, false>(L, ph, a, shot, bx, by, zc, plane_t);
}

// ---------------------------------------------------------------------------
// 3D leapfrog, two steps per launch (temporal blocking along the z march).
//
// Block = 8 waves over a tile of T3Y2 rows (y) by TX = 64 - 2R columns (x);
// lane l of every wave holds column x0 - R + l, so a wave row covers the tile
// plus an R-wide x halo.  The tile plus an R-wide halo in x and y is the
// extended region.  The block marches a z chunk of tz3 planes: at march
// position p the first step gives u^{k+1} at plane z1 = zc0 - R + p on the
// extended region, and the second step gives u^{k+2} at plane z2 = z1 - R on
// the tile.  The second step lags R planes behind the first, so its z
// neighbours are known when it runs.  Each thread owns two tile rows and (in
// waves < 2R) one halo row of the extended region and keeps, in registers,
//   u^k      a z queue of 2R + 1 planes per owned row,
//   u^{k+1}  a z queue of 2R + 1 planes per owned tile row,
//   beta     the last R + 1 planes per owned tile row (the second step's).
// x/y neighbours come from LDS: u^k at plane z1 staged with a 2R halo around
// the extended region (double-buffered), and the last R + 1 planes of u^{k+1}
// on the extended region (a ring).  One barrier per plane.  u^{k-1}, u^k and
// beta are read once for two steps; u^{k+1} and u^{k+2} are written on the
// tile.  Halo nodes of u^{k+1} are recomputed by the neighbouring tiles and
// chunks with the one-step kernel's arithmetic, so one launch of two steps
// and two launches of one step give the same bits.
// ---------------------------------------------------------------------------
template <int N>
struct Phase {
    static constexpr int value = N;
};

template <int R, bool FAST>
__device__ __forceinline__ void step3d2_body(const Layout &L, const Physics &ph, const StepArgs &a, int shot, int bx,
                                             int by, int zc0, int zend, float (*Us)[T3Y2 + 4 * R][64 + 2 * R],
                                             float (*Vr)[T3Y2 + 2 * R][64 + 2 * R]) {
#pragma clang fp contract(off)
    constexpr int TX = t2x(R);
    constexpr int EY = T3Y2 + 2 * R;   // rows of the extended region
    constexpr int SY = T3Y2 + 4 * R;   // staged rows of u^k
    constexpr int NV = R + 1;          // planes of u^{k+1} held in LDS
    constexpr int NQ = 2 * R + 1;      // planes held by a z queue
    constexpr int MAPN = 64 * EY;      // nodes of one plane's injection map
    const int lx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int x0 = bx * TX, y0 = by * T3Y2;
    const int x = x0 - R + lx;
    const bool hrow = w < 2 * R;   // this wave owns a halo row of the extended region
    // owned rows of the extended region: two tile rows, then the halo row
    const int er[3] = {R + w, R + 8 + w, w < R ? w : T3Y2 + w};
    const int G0 = (int)L.G[0], PL = (int)(L.G[0] * L.G[1]);
    const int P0 = (int)L.P[0], P1 = (int)L.P[1], P2 = (int)L.P[2], oy = (int)L.oy;
    const uint32_t span = (uint32_t)(L.shot_floats * 4);
    const int64_t so = shot * L.shot_floats + XO;
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.cur + so, span), rp = buf_rsrc(a.prev + so, span);
    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(a.beta + XO, span);
    const __amdgpu_buffer_rsrc_t rn1 = buf_rsrc(a.next + so, span), rn2 = buf_rsrc(a.next2 + so, span);
    auto plane = [&](int z) { return (uint32_t)((FAST ? z : clampi(z, 0, P2 - 1)) + R) * (uint32_t)PL * 4u; };
    auto lane = [&](int y, int xx) {   // byte offset of (y, x) within a plane
        return 4u * (uint32_t)(((FAST ? y : clampi(y, 0, P1 - 1)) + oy) * G0 + (FAST ? xx : clampi(xx, 0, P0 - 1)));
    };
    auto zin = [&](int z) { return FAST || (z >= 0 && z < P2); };

    // this lane's node in each owned row
    const bool xin = FAST || (x >= 0 && x < P0);
    const bool act = lx >= R && lx < R + TX;   // tile columns
    uint32_t vo[3];
    bool rin[3];
    float hxy[3];
    const float hx = FAST ? 0.0f : layer_frac2(x, (int)L.n[0], L.nb, ph.inv_nb);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int y = y0 - R + er[i];
        vo[i] = lane(y, x);
        rin[i] = (i < 2 || hrow) && (FAST || (xin && y >= 0 && y < P1));
        hxy[i] = FAST ? 0.0f : hx + layer_frac2(y, (int)L.n[1], L.nb, ph.inv_nb);
    }
    // the staged plane's x halo of each owned row (lanes < 2R): staged column scx
    const bool xl = lx < 2 * R;
    const int scx = lx < R ? lx : 64 + lx;
    const int xc = x0 - 2 * R + scx;
    uint32_t co[3];
    bool cin[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int y = y0 - R + er[i];
        co[i] = lane(y, xl ? xc : x);
        cin[i] = xl && (i < 2 || hrow) && (FAST || (xc >= 0 && xc < P0 && y >= 0 && y < P1));
    }
    // the staged plane's y halo: staged row xr (waves < 2R), columns lx and 64 + lx (lanes < 2R)
    const int xr = w < R ? w : SY - 2 * R + w;
    const int yr = y0 - 2 * R + xr;
    const int xa = x0 - 2 * R + lx, xb = x0 + TX + lx;
    const bool yrin = FAST || (yr >= 0 && yr < P1);
    const bool rain = hrow && yrin && (FAST || (xa >= 0 && xa < P0));
    const bool rbin = hrow && xl && yrin && (FAST || xb < P0);
    const uint32_t ra = lane(yr, xa), rbo = lane(yr, xl ? xb : xa);

    // z queues indexed by plane modulo NQ: the march position p holds the
    // first step at plane z1 = zc0 - R + p, and plane z1 + d sits in slot
    // (p + d) mod NQ.  The march is unrolled NQ times, so every slot index is
    // a constant and no value moves between registers.
    float qk[3][NQ], qv[2][NQ];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {   // u^k at planes z1 - R .. z1 + R - 1 of position 0
        const int z = zc0 - 2 * R + j;
        const uint32_t zo = plane(z);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
            if (i < 2 || hrow) v = buf_load(rc, vo[i], zo);
            qk[i][(j - R + NQ) % NQ] = (rin[i] && zin(z)) ? v : 0.0f;
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int j = 0; j < NQ; ++j) qv[t][j] = 0.0f;
    }

    // loads of one march position, issued one plane ahead: u^k at z1 + R and
    // the staged plane's halo at z1, u^{k-1} and beta at z1, beta at z1 - R
    // for the second step (tile rows; read R planes ago, so a cache hit)
    float nk[3], nc[3], np_[3], nbt[3], nr[2], nb2[2];
    auto load_plane = [&](int z1) {
        const uint32_t zo = plane(z1), zq = plane(z1 + R), zb2 = plane(z1 - R);
        nb2[0] = buf_load(rb, vo[0], zb2);
        nb2[1] = buf_load(rb, vo[1], zb2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < 2 || hrow) {
                nk[i] = buf_load(rc, vo[i], zq);
                nc[i] = buf_load(rc, co[i], zo);
                np_[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, (int)vo[i], (int)zo, kBufNT));
                nbt[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, (int)vo[i], (int)zo, kBufNT));
            } else {
                nk[i] = nc[i] = np_[i] = nbt[i] = 0.0f;
            }
        }
        if (hrow) {
            nr[0] = buf_load(rc, ra, zo);
            nr[1] = buf_load(rc, rbo, zo);
        } else {
            nr[0] = nr[1] = 0.0f;
        }
    };
    load_plane(zc0 - R);

    const int niter = (zend - zc0) + 2 * R;
    // planes of this tile column that hold source nodes (none: zlo > zhi)
    int zlo = 1, zhi = 0;
    if (a.inject) {
        const int col = (shot * (int)L.ntiles[1] + by) * (int)L.ntiles[0] + bx;
        zlo = __builtin_amdgcn_readfirstlane(a.inj.col_z[2 * col]);
        zhi = __builtin_amdgcn_readfirstlane(a.inj.col_z[2 * col + 1]);
    }

    // one march position; PH = p mod NQ
    auto position = [&](auto phase, int p) __attribute__((always_inline)) {
        constexpr int PH = decltype(phase)::value;
        auto sk = [](int d) { return (PH + d + 2 * NQ) % NQ; };   // slot of plane z1 + d
        const int z1 = zc0 - R + p, z2 = z1 - R;
        const bool z1in = zin(z1);
        const bool two = p >= 2 * R;   // the second step runs at z2
        // take the loads of this position
        float pm[3], bt[3], b2[2] = {nb2[0], nb2[1]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            qk[i][sk(R)] = (rin[i] && zin(z1 + R)) ? nk[i] : 0.0f;
            pm[i] = np_[i];
            bt[i] = nbt[i];
        }
        float(*U)[64 + 2 * R] = Us[p & 1];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < 2 || hrow) {
                U[er[i] + R][lx + R] = qk[i][sk(0)];
                if (xl) U[er[i] + R][scx] = (cin[i] && z1in) ? nc[i] : 0.0f;
            }
        }
        if (hrow) {
            U[xr][lx] = (rain && z1in) ? nr[0] : 0.0f;
            if (xl) U[xr][64 + lx] = (rbin && z1in) ? nr[1] : 0.0f;
        }
        // point-source terms: the first step's on the extended region at z1,
        // the second step's on the tile at z2
        float s1[3] = {0.0f, 0.0f, 0.0f}, s2[2] = {0.0f, 0.0f};
        if (zlo <= zhi && ((z1 >= zlo && z1 <= zhi) || (two && z2 >= zlo && z2 <= zhi))) {
            const KernargStep ka = kernarg_step_args();
            InjectTables inj;
            inj.tile_dense = ka->inj.tile_dense;
            inj.dense = ka->inj.dense;
            inj.seg_ent = ka->inj.seg_ent;
            inj.ent_idx = ka->inj.ent_idx;
            inj.ent_w = ka->inj.ent_w;
            inj.col_z = nullptr;
            const float *amp0 = ka->amp.ptr + shot * ka->amp.shot_stride;
            const float scale = ka->amp.scale;
            const int64_t col_planes = (int64_t)shot * L.ntiles[2];
            if (z1 >= zlo && z1 <= zhi) {
                const int map = inj.tile_dense[((col_planes + z1) * L.ntiles[1] + by) * L.ntiles[0] + bx];
                if (map >= 0) {
                    const float *amp1 = amp0 + (int64_t)ka->k * ka->amp.k_stride;
                    const int32_t *dm = inj.dense + (int64_t)map * MAPN + lx;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        if (i < 2 || hrow) {
                            const int sg = dm[er[i] * 64];
                            if (sg >= 0) s1[i] = segment_value(inj, amp1, scale, sg);
                        }
                    }
                }
            }
            if (two && z2 >= zlo && z2 <= zhi) {
                const int map = inj.tile_dense[((col_planes + z2) * L.ntiles[1] + by) * L.ntiles[0] + bx];
                if (map >= 0) {
                    const float *amp2 = amp0 + (int64_t)ka->k2 * ka->amp.k_stride;
                    const int32_t *dm = inj.dense + (int64_t)map * MAPN + lx;
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int sg = dm[er[t] * 64];
                        if (sg >= 0) s2[t] = segment_value(inj, amp2, scale, sg);
                    }
                }
            }
        }
        __syncthreads();
        if (p + 1 < niter) load_plane(z1 + 1);   // overlaps the compute below

        // first step at z1 on the owned rows of the extended region
        const float hz1 = FAST ? 0.0f : layer_frac2(z1, (int)L.n[2], L.nb, ph.inv_nb);
        const bool out1 = z1 >= zc0 && z1 < zend;   // u^{k+1} of this plane belongs to the chunk
        const uint32_t zo1 = plane(z1);
        float(*Vw)[64 + 2 * R] = Vr[p % NV];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < 2 || hrow) {
                const int sr = er[i] + R, sc = lx + R;
                const float cv = qk[i][sk(0)];
                float lap = 3.0f * ph.c[0] * cv;
#pragma unroll
                for (int k = 1; k <= R; ++k)
                    lap = __builtin_fmaf(ph.c[k], (U[sr][sc - k] + U[sr][sc + k]) + (U[sr - k][sc] + U[sr + k][sc]) +
                                                      (qk[i][sk(-k)] + qk[i][sk(k)]),
                                         lap);
                float v;
                if (FAST) {
                    v = leapfrog0(cv, pm[i], bt[i], lap, s1[i]);
                } else {
                    v = (rin[i] && z1in) ? leapfrog(cv, pm[i], bt[i], lap, s1[i], ph.hd_max * (hxy[i] + hz1)) : 0.0f;
                }
                Vw[er[i]][lx + R] = v;
                if (i < 2) {
                    qv[i][sk(0)] = v;
                    if (act && out1 && rin[i]) buf_store(v, rn1, vo[i], zo1);
                }
            }
        }
        // second step at z2 on the owned tile rows; the u^{k+1} plane z2 was
        // written R positions ago, before this position's barrier
        if (two) {
            const float(*V)[64 + 2 * R] = Vr[(p - R) % NV];
            const float hz2 = FAST ? 0.0f : layer_frac2(z2, (int)L.n[2], L.nb, ph.inv_nb);
            const uint32_t zo2 = plane(z2);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int vr = er[t], vc = lx + R;   // idle lanes read the pad columns
                const float cv = qv[t][sk(-R)];
                float lap = 3.0f * ph.c[0] * cv;
#pragma unroll
                for (int k = 1; k <= R; ++k)
                    lap = __builtin_fmaf(ph.c[k], (V[vr][vc - k] + V[vr][vc + k]) + (V[vr - k][vc] + V[vr + k][vc]) +
                                                      (qv[t][sk(-R - k)] + qv[t][sk(-R + k)]),
                                         lap);
                const float u2 = FAST ? leapfrog0(cv, qk[t][sk(-R)], b2[t], lap, s2[t])
                                      : leapfrog(cv, qk[t][sk(-R)], b2[t], lap, s2[t], ph.hd_max * (hxy[t] + hz2));
                if (act && rin[t]) buf_store(u2, rn2, vo[t], zo2);
            }
        }
    };

    for (int p = 0; p < niter; p += NQ) {
        position(Phase<0>{}, p);
        if (p + 1 >= niter) break;
        position(Phase<1>{}, p + 1);
        if (p + 2 >= niter) break;
        position(Phase<2>{}, p + 2);
        if (p + 3 >= niter) break;
        position(Phase<3>{}, p + 3);
        if (p + 4 >= niter) break;
        position(Phase<4>{}, p + 4);
        if constexpr (NQ > 5) {
            if (p + 5 >= niter) break;
            position(Phase<5 % NQ>{}, p + 5);
            if (p + 6 >= niter) break;
            position(Phase<6 % NQ>{}, p + 6);
            if (p + 7 >= niter) break;
            position(Phase<7 % NQ>{}, p + 7);
            if (p + 8 >= niter) break;
            position(Phase<8 % NQ>{}, p + 8);
        }
    }
}

template <int R>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_step3d2(const Step3DArgs P) {
    constexpr int TX = t2x(R);
    const Layout &L = P.L;
    const Physics &ph = P.ph;
    const StepArgs &a = P.a;
    __shared__ float Us[2][T3Y2 + 4 * R][64 + 2 * R];
    __shared__ float Vr[R + 1][T3Y2 + 2 * R][64 + 2 * R];   // R pad columns each side
    const int ntx = (int)L.ntiles[0], nty = (int)L.ntiles[1], tz = L.tz3;
    const int P0 = (int)L.P[0], P1 = (int)L.P[1], P2 = (int)L.P[2];
    const int nzc = (P2 + tz - 1) / tz;
    const int lid = xcd_logical_block(ntx * nty * nzc * L.S);
    if (lid < 0) return;
    const int bx = lid % ntx, by = (lid / ntx) % nty, zc = (lid / (ntx * nty)) % nzc, shot = lid / (ntx * nty * nzc);
    const int x0 = bx * TX, y0 = by * T3Y2, zc0 = zc * tz, nb = L.nb;
    const int zend = zc0 + tz < P2 ? zc0 + tz : P2;
    // interior block: every staged read inside the padded box, every node of
    // the extended region undamped at every plane of the first step
    const bool fast = x0 - 2 * R >= 0 && x0 + TX + 2 * R <= P0 && y0 - 2 * R >= 0 && y0 + T3Y2 + 2 * R <= P1 &&
                      zc0 - 2 * R >= 0 && zc0 + tz + 2 * R <= P2 && x0 - R >= nb && x0 + TX + R <= nb + (int)L.n[0] &&
                      y0 - R >= nb && y0 + T3Y2 + R <= nb + (int)L.n[1] && zc0 - R >= nb &&
                      zc0 + tz + R <= nb + (int)L.n[2];
    // sampling first: the launch's inputs are read-only, and its arguments
    // are dead before the march starts
    const int per_shot = ntx * nty * nzc, bis = (zc * nty + by) * ntx + bx;
    if (a.do_sample) sample_points<8>(L, a.cur + shot * L.shot_floats, a.k, a.smp, shot, bis, per_shot);
    if (a.sample_prev) sample_points<8>(L, a.prev + shot * L.shot_floats, a.kp, a.smp, shot, bis, per_shot);
    if (fast) step3d2_body<R, true>(L, ph, a, shot, bx, by, zc0, zend, Us, Vr);
    else step3d2_body<R, false>(L, ph, a, shot, bx, by, zc0, zend, Us, Vr);
}

template <int NC>
__global__ __launch_bounds__(256) void k_sample(const Layout L, const float *field, int k, const SampleTables smp) {
    const int shot = blockIdx.y;
    sample_points<NC>(L, field + shot * L.shot_floats, k, smp, shot, blockIdx.x, gridDim.x);
}

hipError_t launch_step(const Layout &L, const Physics &ph, const StepArgs &a, hipStream_t stream) {
    if (L.ndim == 2) {
        const int64_t nlog = L.ntiles[0] * L.ntiles[2] * L.S;
        dim3 grid((unsigned)((nlog + 7) / 8 * 8));
        const int tz = (int)L.tile[2];
        if (tz != T2Z && tz != T2Z_MID && tz != T2Z_SMALL) return hipErrorInvalidValue;
#define TPX_STEP2D(RR, NS)                                                                          \
    do {                                                                                            \
        if (tz == T2Z) hipLaunchKernelGGL((k_step2d<RR, NS, T2Z>), grid, dim3(256), 0, stream, L, ph, a); \
        else if (tz == T2Z_MID)                                                                     \
            hipLaunchKernelGGL((k_step2d<RR, NS, T2Z_MID>), grid, dim3(256), 0, stream, L, ph, a);  \
        else hipLaunchKernelGGL((k_step2d<RR, NS, T2Z_SMALL>), grid, dim3(256), 0, stream, L, ph, a); \
    } while (0)
        if (a.nstep == 3) {
            // L is the three-step layout: tiles of t3x(R) columns, rows as the two-step tiles
            if (L.tile[0] != t3x(L.R)) return hipErrorInvalidValue;
#define TPX_STEP2D3(RR, TT) hipLaunchKernelGGL((k_step2d3<RR, TT>), grid, dim3(256), 0, stream, L, ph, a)
            if (tz == T2Z) { if (L.R == 2) TPX_STEP2D3(2, T2Z); else TPX_STEP2D3(4, T2Z); }
            else if (tz == T2Z_MID) { if (L.R == 2) TPX_STEP2D3(2, T2Z_MID); else TPX_STEP2D3(4, T2Z_MID); }
            else { if (L.R == 2) TPX_STEP2D3(2, T2Z_SMALL); else TPX_STEP2D3(4, T2Z_SMALL); }
#undef TPX_STEP2D3
        } else if (a.nstep == 2) {
            if (L.R == 2) TPX_STEP2D(2, 2);
            else TPX_STEP2D(4, 2);
        } else {
            if (L.R == 2) TPX_STEP2D(2, 1);
            else TPX_STEP2D(4, 1);
        }
#undef TPX_STEP2D
    } else if (a.nstep == 2) {
        if (L.tz3 < 1 || L.tile[0] != t2x(L.R) || L.tile[1] != T3Y2) return hipErrorInvalidValue;
        const int64_t zchunks = (L.P[2] + L.tz3 - 1) / L.tz3;
        const int64_t nlog = L.ntiles[0] * L.ntiles[1] * zchunks * L.S;
        dim3 grid((unsigned)((nlog + 7) / 8 * 8));
        const Step3DArgs p3 = {L, ph, a};
        if (L.R == 2) hipLaunchKernelGGL(k_step3d2<2>, grid, dim3(512), 0, stream, p3);
        else hipLaunchKernelGGL(k_step3d2<4>, grid, dim3(512), 0, stream, p3);
    } else {
        if (a.nstep != 1) return hipErrorInvalidValue;
        const int64_t zchunks = (L.P[2] + T3Z - 1) / T3Z;
        const int64_t nlog = ((L.P[0] + T3X - 1) / T3X) * ((L.P[1] + T3Y - 1) / T3Y) * zchunks * L.S;
        dim3 grid((unsigned)((nlog + 7) / 8 * 8));
        const Step3DArgs p3 = {L, ph, a};
        if (L.R == 2) hipLaunchKernelGGL(k_step3d<2>, grid, dim3(256), 0, stream, p3);
        else hipLaunchKernelGGL(k_step3d<4>, grid, dim3(256), 0, stream, p3);
    }
    return hipGetLastError();
}

hipError_t launch_sample_only(const Layout &L, const float *field, int k, const SampleTables &smp,
                              hipStream_t stream) {
    if (smp.nsmp <= 0) return hipSuccess;
    dim3 grid((unsigned)((smp.nsmp + 255) / 256), (unsigned)L.S);
    if (L.ndim == 2) hipLaunchKernelGGL(k_sample<4>, grid, dim3(256), 0, stream, L, field, k, smp);
    else hipLaunchKernelGGL(k_sample<8>, grid, dim3(256), 0, stream, L, field, k, smp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// model preparation: beta = dt^2 / m_pad over the allocated (ghosted) extent
// of one shot field; m_pad is m with its edge values replicated into the
// absorbing layer.  Ghost cells get 0.  flags[0] is set when m is not finite
// and positive somewhere.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_model_prep(const Layout L, const float *__restrict__ m, double dt2,
                                                    float m_min, float *__restrict__ beta, int32_t *flags) {
    const int64_t xg = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = blockIdx.y;  // zg * G1 + yg
    if (xg >= L.G[0]) return;
    const int64_t zg = row / L.G[1], yg = row - zg * L.G[1];
    const int64_t ix = xg - XO, iy = yg - L.oy, iz = zg - L.R;
    float b = 0.0f;
    if (ix >= 0 && ix < L.P[0] && iy >= 0 && iy < L.P[1] && iz >= 0 && iz < L.P[2]) {
        const int64_t oyb = L.ndim == 3 ? L.nb : 0;
        int64_t px = ix - L.nb, py = iy - oyb, pz = iz - L.nb;
        px = px < 0 ? 0 : (px > L.n[0] - 1 ? L.n[0] - 1 : px);
        py = py < 0 ? 0 : (py > L.n[1] - 1 ? L.n[1] - 1 : py);
        pz = pz < 0 ? 0 : (pz > L.n[2] - 1 ? L.n[2] - 1 : pz);
        const float mv = m[(pz * L.n[1] + py) * L.n[0] + px];
        if (!(mv > 0.0f) || !isfinite(mv)) atomicOr(flags, 1);
        else if (mv < m_min) atomicOr(flags, 2);
        b = (float)(dt2 / (double)mv);
    }
    beta[row * L.G[0] + xg] = b;
}

hipError_t launch_model_prep(const Layout &L, const float *m, double dt, float m_min, float *beta, int32_t *flags,
                             hipStream_t stream) {
    dim3 grid((unsigned)((L.G[0] + 255) / 256), (unsigned)(L.G[1] * L.G[2]));
    hipLaunchKernelGGL(k_model_prep, grid, dim3(256), 0, stream, L, m, dt * dt, m_min, beta, flags);
    return hipGetLastError();
}

// Header of a probed forward pass's state: the problem and probes it belongs
// to, written by the forward pass and compared by the backward pass, which
// sets flags bit 2 on a mismatch.
__global__ __launch_bounds__(64) void k_state_header(StateHeader h, int32_t *hdr, int32_t *flags, int check) {
    const int i = threadIdx.x;
    if (i >= StateHeader::kWords) return;
    if (!check) {
        hdr[i] = h.w[i];
    } else if (hdr[i] != h.w[i]) {
        atomicOr(flags, 4);
    }
}

hipError_t launch_state_header(const StateHeader &h, void *hdr, int32_t *flags, int check, hipStream_t stream) {
    hipLaunchKernelGGL(k_state_header, dim3(1), dim3(64), 0, stream, h, (int32_t *)hdr, flags, check);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(float4 *p, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    // every sub-buffer of the workspace is 256-byte aligned and sized in 256-byte units
    const int64_t n4 = (int64_t)(bytes / 16);
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, (float4 *)ptr, n4);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probes: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), integer only,
// so the GPU reproduces the host bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_w0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return c0;
}

__global__ __launch_bounds__(256) void k_probe_gen(int kind, int r, uint64_t seed, int nt, int shot0,
                                                   float *__restrict__ Z) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per_shot = (int64_t)nt * r;
    if (i >= per_shot) return;
    const int shot = shot0 + blockIdx.y;
    const int t = (int)(i / r), j = (int)(i - (int64_t)t * r);
    float z;
    if (kind == 2) {
        z = (t == j) ? 1.0f : 0.0f;
    } else {
        const uint64_t w = philox_w0((uint64_t)t + 1, (uint64_t)j, (uint64_t)shot, 0, seed, 0);
        if (kind == 0) z = (w >> 63) ? -1.0f : 1.0f;
        else z = (float)((int)__popcll(w) - 32) * 0.25f;
    }
    Z[(int64_t)blockIdx.y * per_shot + i] = z;
}

hipError_t launch_probe_gen(int kind, int r, uint64_t seed, int nt, int shot0, int nshots, float *Z,
                            hipStream_t stream) {
    const int64_t per_shot = (int64_t)nt * r;
    dim3 grid((unsigned)((per_shot + 255) / 256), (unsigned)nshots);
    hipLaunchKernelGGL(k_probe_gen, grid, dim3(256), 0, stream, kind, r, seed, nt, shot0, Z);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(const float *__restrict__ a, int64_t n, float *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) b[i] = a[i];
}

hipError_t launch_probe_copy(const float *Zsrc, int64_t n, float *Zdst, hipStream_t stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, stream, Zsrc, n, Zdst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probe contractions over a block of buffered time steps (Algorithm 1's
// forward and back-propagation accumulations, time-blocked): one thread per
// physical point and shot keeps RC accumulators in registers while it streams
// the buffered slots; the probing row Z[s, :] is uniform across the block and
// is read through scalar loads.  Grid (chunks of 256 points, shots).
// ---------------------------------------------------------------------------
struct PointIndex {
    int off;     // offset within a shot field
    int64_t p;   // flat physical index
    bool ok;
};

// Block = 256 consecutive physical points of one shot (so every buffered
// slot is read in runs of about 1 KB); grid (point chunks, shots).
__device__ __forceinline__ PointIndex point_index(const Layout &L) {
    PointIndex pi;
    const int p = (int)blockIdx.x * 256 + (int)threadIdx.x;
    pi.ok = p < L.nphys;
    const int n0 = (int)L.n[0], n1 = (int)L.n[1];
    const int row = p / n0, x = p - row * n0;
    const int z = row / n1, y = row - z * n1;
    const int oyb = L.ndim == 3 ? L.nb : 0;
    pi.off = (int)L.pad_off(x + L.nb, y + oyb, z + L.nb);
    pi.p = p;
    return pi;
}

constexpr int kAccUnroll = 8;   // buffered steps whose loads are issued together

// Buffered slots are read exactly once by a contraction (plain loads: a
// nontemporal hint measured no faster).
__device__ __forceinline__ float ring_load(const float *p) { return *p; }

// Forward contraction of exactly RC probes j0..j0+RC-1 (no per-probe
// predicates: the launcher splits r into power-of-two chunks).
template <int RC>
__global__ __launch_bounds__(256) void k_accum_fwd(const Layout L, const float *__restrict__ ring, int nslots,
                                                   int s_lo, int s_hi, const float *__restrict__ Z, int nt, int r,
                                                   int j0, float *__restrict__ ubar) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.y;
    const float *base = ring + shot * L.shot_floats + pi.off;
    const float *Zs = Z + (int64_t)shot * nt * r + j0;
    float acc[RC];
#pragma unroll
    for (int j = 0; j < RC; ++j) acc[j] = 0.0f;
    int s = s_lo;
    for (; s + kAccUnroll - 1 <= s_hi; s += kAccUnroll) {
        float v[kAccUnroll];
#pragma unroll
        for (int u = 0; u < kAccUnroll; ++u) v[u] = ring_load(&base[(int64_t)((s + u) % nslots) * L.slot_floats]);
#pragma unroll
        for (int u = 0; u < kAccUnroll; ++u) {
            const float *zr = Zs + (int64_t)(s + u) * r;
#pragma unroll
            for (int j = 0; j < RC; ++j) acc[j] = fmaf(zr[j], v[u], acc[j]);
        }
    }
    for (; s <= s_hi; ++s) {
        const float v = ring_load(&base[(int64_t)(s % nslots) * L.slot_floats]);
        const float *zr = Zs + (int64_t)s * r;
#pragma unroll
        for (int j = 0; j < RC; ++j) acc[j] = fmaf(zr[j], v, acc[j]);
    }
    float *ub = ubar + ((int64_t)shot * r + j0) * L.nphys + pi.p;
#pragma unroll
    for (int j = 0; j < RC; ++j) ub[(int64_t)j * L.nphys] += acc[j];
}

// One buffered step: w = f^{s-1} - 2 f^s + f^{s+1} (SD) or w = f^s (lp holds f^s).
template <int RC, int FOLD, int SD>
__device__ __forceinline__ void adj_step(float &lm, float &l0, float lp, const float *zr, const float *u, float *acc,
                                         float &fsum) {
    const float w = SD ? (lm - 2.0f * l0) + lp : lp;
    if (FOLD) {
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < RC; ++j) t = fmaf(zr[j], u[j], t);
        fsum = fmaf(w, t, fsum);
    } else {
#pragma unroll
        for (int j = 0; j < RC; ++j) acc[j] = fmaf(zr[j], w, acc[j]);
    }
    lm = l0;
    l0 = lp;
}

// Contraction of exactly RC probes j0..j0+RC-1 over w^s, s = s_lo..s_hi: either
// vbar_j += sum_s Z[s,j] w^s, or (FOLD) gpart -= c sum_s w^s sum_j Z[s,j] ubar_j.
// SD = 1: w^s = f^{s-1} - 2 f^s + f^{s+1} (second time difference of the
// buffered field f); SD = 0: w^s = f^s.
template <int RC, int FOLD, int SD>
__global__ __launch_bounds__(256) void k_accum_adj(const Layout L, const float *__restrict__ ring, int nslots,
                                                   int s_lo, int s_hi, const float *__restrict__ Z, int nt, int r,
                                                   int j0, const float *__restrict__ ubar, float c,
                                                   float *__restrict__ vbar, float *__restrict__ gpart) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.y;
    const float *base = ring + shot * L.shot_floats + pi.off;
    const float *Zs = Z + (int64_t)shot * nt * r + j0;
    float u[RC];
    float acc[RC];
#pragma unroll
    for (int j = 0; j < RC; ++j) {
        acc[j] = 0.0f;
        u[j] = 0.0f;
    }
    if (FOLD) {
        const float *ub = ubar + ((int64_t)shot * r + j0) * L.nphys + pi.p;
#pragma unroll
        for (int j = 0; j < RC; ++j) u[j] = ub[(int64_t)j * L.nphys];
    }
    // SD: (lm, l0) hold f^{s-1}, f^s and the loads fetch f^{s+1}; otherwise the loads fetch f^s
    const int ahead = SD ? 1 : 0;
    float lm = SD ? ring_load(&base[(int64_t)(((s_lo - 1) % nslots + nslots) % nslots) * L.slot_floats]) : 0.0f;
    float l0 = SD ? ring_load(&base[(int64_t)(s_lo % nslots) * L.slot_floats]) : 0.0f;
    float fsum = 0.0f;
    int s = s_lo;
    for (; s + kAccUnroll - 1 <= s_hi; s += kAccUnroll) {
        float lp[kAccUnroll];
#pragma unroll
        for (int q = 0; q < kAccUnroll; ++q) lp[q] = ring_load(&base[(int64_t)((s + q + ahead) % nslots) * L.slot_floats]);
#pragma unroll
        for (int q = 0; q < kAccUnroll; ++q) adj_step<RC, FOLD, SD>(lm, l0, lp[q], Zs + (int64_t)(s + q) * r, u, acc, fsum);
    }
    for (; s <= s_hi; ++s)
        adj_step<RC, FOLD, SD>(lm, l0, ring_load(&base[(int64_t)((s + ahead) % nslots) * L.slot_floats]),
                               Zs + (int64_t)s * r, u, acc, fsum);
    if (FOLD) {
        gpart[(int64_t)shot * L.nphys + pi.p] -= c * fsum;
    } else {
        float *vb = vbar + ((int64_t)shot * r + j0) * L.nphys + pi.p;
#pragma unroll
        for (int j = 0; j < RC; ++j) vb[(int64_t)j * L.nphys] += acc[j];
    }
}

__global__ __launch_bounds__(256) void k_accum_full(const Layout L, const float *__restrict__ hist,
                                                    const float *__restrict__ ring, int nslots, int s_lo, int s_hi,
                                                    float *__restrict__ gpart) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.y;
    const float *hb = hist + shot * L.shot_floats + pi.off;
    const float *base = ring + shot * L.shot_floats + pi.off;
    float lm = ring_load(&base[(int64_t)((s_lo - 1) % nslots) * L.slot_floats]);
    float l0 = ring_load(&base[(int64_t)(s_lo % nslots) * L.slot_floats]);
    float acc = 0.0f;
    int s = s_lo;
    for (; s + kAccUnroll - 1 <= s_hi; s += kAccUnroll) {
        float lp[kAccUnroll], uh[kAccUnroll];
#pragma unroll
        for (int q = 0; q < kAccUnroll; ++q) {
            lp[q] = ring_load(&base[(int64_t)((s + q + 1) % nslots) * L.slot_floats]);
            uh[q] = ring_load(&hb[(int64_t)(s + q) * L.slot_floats]);
        }
#pragma unroll
        for (int q = 0; q < kAccUnroll; ++q) {
            const float w = (lm - 2.0f * l0) + lp[q];
            acc = fmaf(uh[q], w, acc);
            lm = l0;
            l0 = lp[q];
        }
    }
    for (; s <= s_hi; ++s) {
        const float lp = ring_load(&base[(int64_t)((s + 1) % nslots) * L.slot_floats]);
        const float w = (lm - 2.0f * l0) + lp;
        acc = fmaf(ring_load(&hb[(int64_t)s * L.slot_floats]), w, acc);
        lm = l0;
        l0 = lp;
    }
    gpart[(int64_t)shot * L.nphys + pi.p] -= acc;
}

// ---------------------------------------------------------------------------
// Probe contractions on the matrix cores.  A time block of b buffered levels
// is the dense product acc (r x P) += Z^T (r x b) . F (b x P), F the buffered
// field (or its second time difference) at P physical points.  The probes
// of the counter-hash kinds are exact in bfloat16 (+-1, and multiples of 1/4
// up to 8 in magnitude), and every FP32 field value splits exactly into
// three bfloat16 parts (each keeps the next 8 significant bits), so three
// bf16 products per tile accumulate, in FP32, the same terms as the FP32
// contraction.  v_mfma_f32_16x16x16_bf16: lane l = 16 g + n supplies
// A[m = n][k = 4 g + q] and B[k = 4 g + q][n], q = 0..3, and receives
// D[m = 4 g + i][n], i = 0..3.  A wave covers 64 consecutive physical points
// of one shot as four 16-point tiles; k runs over 16 buffered levels.
// ---------------------------------------------------------------------------
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int phys_offset(const Layout &L, int p) {
    const int n0 = (int)L.n[0], n1 = (int)L.n[1];
    const int row = p / n0, x = p - row * n0;
    const int z = row / n1, y = row - z * n1;
    const int oyb = L.ndim == 3 ? L.nb : 0;
    return (int)L.pad_off(x + L.nb, y + oyb, z + L.nb);
}

// x = h + m + l exactly, each a bfloat16 (the upper 16 bits of a float)
__device__ __forceinline__ void split_bf16x3(const float (&x)[4], shortx4 &h, shortx4 &m, shortx4 &l) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned uh = __float_as_uint(x[q]) & 0xffff0000u;
        const float r1 = x[q] - __uint_as_float(uh);
        const unsigned um = __float_as_uint(r1) & 0xffff0000u;
        const float r2 = r1 - __uint_as_float(um);
        h[q] = (short)(uh >> 16);
        m[q] = (short)(um >> 16);
        l[q] = (short)(__float_as_uint(r2) >> 16);
    }
}

__device__ __forceinline__ floatx4 mfma_bf16x3(shortx4 a, shortx4 bh, shortx4 bm, shortx4 bl, floatx4 d) {
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bl, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bm, d, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bh, d, 0, 0, 0);
}

// Both operands split in three (probes that are not exact in bfloat16): the
// six products down to the order of 2^-14 relative, smallest first; the
// three dropped terms are below 2^-21 of the product.
__device__ __forceinline__ floatx4 mfma_bf16x6(shortx4 ah, shortx4 am, shortx4 al, shortx4 bh, shortx4 bm,
                                               shortx4 bl, floatx4 d) {
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, d, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, d, 0, 0, 0);
}

__device__ __forceinline__ shortx4 unpack_bf16x4(uint2 z) {
    shortx4 a;
    a[0] = (short)(z.x & 0xffffu);
    a[1] = (short)(z.x >> 16);
    a[2] = (short)(z.y & 0xffffu);
    a[3] = (short)(z.y >> 16);
    return a;
}

__device__ __forceinline__ int ring_slot(int s, int nslots) { return ((s % nslots) + nslots) % nslots; }

// The buffered levels behind one 16-level group at this lane's four points:
// f^{sb-1} .. f^{sb+4} (SD = 1) or f^{sb} .. f^{sb+3} (SD = 0), loaded one
// group ahead of their use.  The loads are unconditional (every slot and
// offset lies inside the ring) and the masks are applied at the use, so the
// loads of the next group stay in flight while this group is contracted.
template <int SD>
struct GroupLoads {
    float f[4][SD ? 6 : 4];
};

// sl: ring slot of level sb - SD (the first level loaded), kept incrementally
// so the loop needs no division.
template <int SD>
__device__ __forceinline__ void group_load(const float *base, uint32_t slot_floats, int nslots, int sl,
                                           const int (&off)[4], GroupLoads<SD> &G) {
    constexpr int NE = SD ? 6 : 4;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const float *fs = base + (uint64_t)(uint32_t)sl * slot_floats;
#pragma unroll
        for (int t = 0; t < 4; ++t) G.f[t][e] = fs[off[t]];
        sl = sl + 1 == nslots ? 0 : sl + 1;
    }
}

// The contracted values of levels sb..sb+3: f^s (SD = 0) or
// f^{s-1} - 2 f^s + f^{s+1} (SD = 1) where s_lo <= s <= s_hi, else zero; a
// buffered level outside s_lo - SD .. s_hi + SD, or a point past the end,
// counts as zero (its slot may hold anything).
template <int SD>
__device__ __forceinline__ void group_values(const GroupLoads<SD> &G, int s_lo, int s_hi, int sb,
                                             const bool (&ok)[4], float (&x)[4][4]) {
#pragma clang fp contract(off)
    constexpr int NE = SD ? 6 : 4;
    float f[4][NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int s = sb - SD + e;
        const bool in = s >= s_lo - SD && s <= s_hi + SD;
#pragma unroll
        for (int t = 0; t < 4; ++t) f[t][e] = (in && ok[t]) ? G.f[t][e] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool in = sb + q >= s_lo && sb + q <= s_hi;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            x[t][q] = in ? (SD ? (f[t][q] - 2.0f * f[t][q + 1]) + f[t][q + 2] : f[t][q]) : 0.0f;
    }
}

// Probe rows in the A-operand order: zpk[part][shot][kg][mt][lane] holds
// Z[16 kg + 4 g + q][16 mt + n], q = 0..3, as four bfloat16 (zero past nt);
// with three parts, the exact three-way split of each value.
__global__ __launch_bounds__(256) void k_pack_probes(int S, int nt, int r, int parts, const float *__restrict__ Z,
                                                     uint2 *__restrict__ zpk) {
    const int nkg = (nt + 15) / 16, nm = r / 16;
    const int64_t total = (int64_t)S * nkg * nm * 64;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int lane = (int)(idx & 63);
    int64_t rest = idx >> 6;
    const int mt = (int)(rest % nm);
    rest /= nm;
    const int kg = (int)(rest % nkg);
    const int shot = (int)(rest / nkg);
    const int g = lane >> 4, n = lane & 15;
    float z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int s = 16 * kg + 4 * g + q;
        z[q] = s < nt ? Z[((int64_t)shot * nt + s) * r + 16 * mt + n] : 0.0f;
    }
    shortx4 h, m, l;
    split_bf16x3(z, h, m, l);
    const shortx4 pv[3] = {h, m, l};
    for (int part = 0; part < parts; ++part) {
        const shortx4 v = pv[part];
        zpk[part * total + idx] = make_uint2((unsigned)(unsigned short)v[0] | ((unsigned)(unsigned short)v[1] << 16),
                                             (unsigned)(unsigned short)v[2] | ((unsigned)(unsigned short)v[3] << 16));
    }
}

// acc_j += sum_s Z[s, j] x^s for the RM x 16 probes j0 ..: ubar (forward) or
// vbar (adjoint), x^s as in group_values.
template <int RM, int SD, int ZS>
__global__ __launch_bounds__(256) void k_accum_mfma(const Layout L, const float *__restrict__ ring, int nslots,
                                                    int s_lo, int s_hi, const uint2 *__restrict__ zpk, int nkg,
                                                    int r, int j0, float *__restrict__ out) {
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int shot = blockIdx.y;
    int off[4], pidx[4];
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int p = (int)blockIdx.x * 256 + wave * 64 + 16 * t + n;
        ok[t] = p < L.nphys;
        pidx[t] = ok[t] ? p : 0;
        off[t] = ok[t] ? phys_offset(L, p) : 0;
    }
    const float *base = ring + (int64_t)shot * L.shot_floats;
    const int nm = r / 16;
    const int64_t part_stride = (int64_t)gridDim.y * nkg * nm * 64;   // gridDim.y = shots
    const uint2 *zs = zpk + (int64_t)shot * nkg * nm * 64 + (j0 / 16) * 64 + lane;
    floatx4 acc[RM][4];
#pragma unroll
    for (int mt = 0; mt < RM; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kg_lo = s_lo >> 4, kg_hi = s_hi >> 4;
    const int step16 = 16 % nslots;
    int sl = ring_slot(16 * kg_lo + 4 * g - SD, nslots);
    auto zload = [&](int kg, uint2 (&zz)[RM * ZS]) {
#pragma unroll
        for (int p = 0; p < ZS; ++p)
#pragma unroll
            for (int mt = 0; mt < RM; ++mt) zz[p * RM + mt] = zs[p * part_stride + ((int64_t)kg * nm + mt) * 64];
    };
    auto contract = [&](const GroupLoads<SD> &G, const uint2 (&zz)[RM * ZS], int kg) {
        float x[4][4];
        group_values<SD>(G, s_lo, s_hi, 16 * kg + 4 * g, ok, x);
        shortx4 bh[4], bm[4], bl[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) split_bf16x3(x[t], bh[t], bm[t], bl[t]);
#pragma unroll
        for (int mt = 0; mt < RM; ++mt) {
            const shortx4 a = unpack_bf16x4(zz[mt]);
            if (ZS == 1) {
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[mt][t] = mfma_bf16x3(a, bh[t], bm[t], bl[t], acc[mt][t]);
            } else {
                const shortx4 am = unpack_bf16x4(zz[RM + mt]), al = unpack_bf16x4(zz[2 * RM + mt]);
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[mt][t] = mfma_bf16x6(a, am, al, bh[t], bm[t], bl[t], acc[mt][t]);
            }
        }
    };
    // Software pipeline over two register sets: the loads of group kg + 1 are
    // issued before group kg is contracted (the scheduling barrier keeps them
    // there), so the wait for group kg leaves the next group's loads in
    // flight.  The loop is unrolled twice so no set is copied.
    GroupLoads<SD> ga, gb;
    uint2 za[RM * ZS], zb[RM * ZS];
    auto prefetch = [&](int kg, GroupLoads<SD> &G, uint2 (&zz)[RM * ZS]) {
        sl += step16;
        if (sl >= nslots) sl -= nslots;
        group_load<SD>(base, (uint32_t)L.slot_floats, nslots, sl, off, G);
        zload(kg, zz);
        __builtin_amdgcn_sched_barrier(0);
    };
    group_load<SD>(base, (uint32_t)L.slot_floats, nslots, sl, off, ga);
    zload(kg_lo, za);
    int kg = kg_lo;
    for (; kg + 2 <= kg_hi; kg += 2) {
        prefetch(kg + 1, gb, zb);
        contract(ga, za, kg);
        prefetch(kg + 2, ga, za);
        contract(gb, zb, kg + 1);
    }
    if (kg < kg_hi) {
        prefetch(kg + 1, gb, zb);
        contract(ga, za, kg);
        contract(gb, zb, kg + 1);
    } else {
        contract(ga, za, kg);
    }
#pragma unroll
    for (int mt = 0; mt < RM; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (!ok[t]) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = j0 + 16 * mt + 4 * g + i;
                out[((int64_t)shot * r + j) * L.nphys + pidx[t]] += acc[mt][t][i];
            }
        }
}

// gpart -= c sum_s x^s sum_j Z[s, j] ubar_j for the RK x 16 probes j0 ..:
// per 16 levels, Y (16 levels x 16 points) = Z (levels x probes) . ubar
// (probes x points) on the matrix cores, then the level sum against x^s in
// FP32 and a fixed-order sum over the four lane groups.
template <int RK, int SD, int ZS>
__global__ __launch_bounds__(256) void k_fold_mfma(const Layout L, const float *__restrict__ ring, int nslots,
                                                   int s_lo, int s_hi, const float *__restrict__ Z, int nt, int r,
                                                   int j0, const float *__restrict__ ubar, float c,
                                                   float *__restrict__ gpart) {
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int shot = blockIdx.y;
    int off[4], pidx[4];
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int p = (int)blockIdx.x * 256 + wave * 64 + 16 * t + n;
        ok[t] = p < L.nphys;
        pidx[t] = ok[t] ? p : 0;
        off[t] = ok[t] ? phys_offset(L, p) : 0;
    }
    shortx4 uh[RK][4], um[RK][4], ul[RK][4];
#pragma unroll
    for (int kt = 0; kt < RK; ++kt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + 16 * kt + 4 * g + q;
                x[q] = ok[t] ? ubar[((int64_t)shot * r + j) * L.nphys + pidx[t]] : 0.0f;
            }
            split_bf16x3(x, uh[kt][t], um[kt][t], ul[kt][t]);
        }
    const float *base = ring + (int64_t)shot * L.shot_floats;
    const float *Zs = Z + (int64_t)shot * nt * r + j0 + 4 * g;
    float fsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const int kg_lo = s_lo >> 4, kg_hi = s_hi >> 4;
    const int step16 = 16 % nslots;
    int sl = ring_slot(16 * kg_lo + 4 * g - SD, nslots);
    // probe rows of a group (A operands), loaded with the group's levels
    auto zload = [&](int kg, float4 (&zv)[RK]) {
        const int sa = 16 * kg + n;   // level of this lane's A row
        const float *zr = Zs + (int64_t)(sa < nt ? sa : nt - 1) * r;
#pragma unroll
        for (int kt = 0; kt < RK; ++kt) zv[kt] = *(const float4 *)(zr + 16 * kt);
    };
    auto contract = [&](const GroupLoads<SD> &G, const float4 (&zv)[RK], int kg) {
        const bool zin = 16 * kg + n < nt;
        floatx4 d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) d[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kt = 0; kt < RK; ++kt) {
            const float zf[4] = {zin ? zv[kt].x : 0.0f, zin ? zv[kt].y : 0.0f, zin ? zv[kt].z : 0.0f,
                                 zin ? zv[kt].w : 0.0f};
            shortx4 ah, am, al;
            split_bf16x3(zf, ah, am, al);
            if (ZS == 1) {
#pragma unroll
                for (int t = 0; t < 4; ++t) d[t] = mfma_bf16x3(ah, uh[kt][t], um[kt][t], ul[kt][t], d[t]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) d[t] = mfma_bf16x6(ah, am, al, uh[kt][t], um[kt][t], ul[kt][t], d[t]);
            }
        }
        float x[4][4];
        group_values<SD>(G, s_lo, s_hi, 16 * kg + 4 * g, ok, x);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) fsum[t] = fmaf(x[t][i], d[t][i], fsum[t]);
    };
    // the same two-set software pipeline as the accumulation kernel
    GroupLoads<SD> ga, gb;
    float4 za[RK], zb[RK];
    auto prefetch = [&](int kg, GroupLoads<SD> &G, float4 (&zz)[RK]) {
        sl += step16;
        if (sl >= nslots) sl -= nslots;
        group_load<SD>(base, (uint32_t)L.slot_floats, nslots, sl, off, G);
        zload(kg, zz);
        __builtin_amdgcn_sched_barrier(0);
    };
    group_load<SD>(base, (uint32_t)L.slot_floats, nslots, sl, off, ga);
    zload(kg_lo, za);
    int kg = kg_lo;
    for (; kg + 2 <= kg_hi; kg += 2) {
        prefetch(kg + 1, gb, zb);
        contract(ga, za, kg);
        prefetch(kg + 2, ga, za);
        contract(gb, zb, kg + 1);
    }
    if (kg < kg_hi) {
        prefetch(kg + 1, gb, zb);
        contract(ga, za, kg);
        contract(gb, zb, kg + 1);
    } else {
        contract(ga, za, kg);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float v = fsum[t];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (g == 0 && ok[t]) gpart[(int64_t)shot * L.nphys + pidx[t]] -= c * v;
    }
}

static dim3 point_grid(const Layout &L) {
    return dim3((unsigned)((L.nphys + 255) / 256), (unsigned)L.S);
}

// largest power of two <= min(64, n)
static int chunk_of(int n) {
    int c = 64;
    while (c > n) c >>= 1;
    return c;
}

hipError_t launch_accum_fwd(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int nt, int r, float *ubar, hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    const dim3 g = point_grid(L);
    for (int j0 = 0; j0 < r;) {
        const int rc = chunk_of(r - j0);
#define TPX_FWD(RC) hipLaunchKernelGGL(k_accum_fwd<RC>, g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, j0, ubar)
        switch (rc) {
        case 64: TPX_FWD(64); break;
        case 32: TPX_FWD(32); break;
        case 16: TPX_FWD(16); break;
        case 8: TPX_FWD(8); break;
        case 4: TPX_FWD(4); break;
        case 2: TPX_FWD(2); break;
        default: TPX_FWD(1); break;
        }
#undef TPX_FWD
        j0 += rc;
    }
    return hipGetLastError();
}

template <int FOLD, int SD>
static void launch_adj_chunks(const Layout &L, dim3 g, hipStream_t stream, const float *ring, int nslots, int s_lo,
                              int s_hi, const float *Z, int nt, int r, const float *ubar, float c, float *vbar,
                              float *gpart) {
    for (int j0 = 0; j0 < r;) {
        const int rc = chunk_of(r - j0);
#define TPX_ADJ(RC) hipLaunchKernelGGL((k_accum_adj<RC, FOLD, SD>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, j0, ubar, c, vbar, gpart)
        switch (rc) {
        case 64: TPX_ADJ(64); break;
        case 32: TPX_ADJ(32); break;
        case 16: TPX_ADJ(16); break;
        case 8: TPX_ADJ(8); break;
        case 4: TPX_ADJ(4); break;
        case 2: TPX_ADJ(2); break;
        default: TPX_ADJ(1); break;
        }
#undef TPX_ADJ
        j0 += rc;
    }
}

hipError_t launch_accum_adj(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int nt, int r, int fold, int sd, const float *ubar, float c, float *vbar, float *gpart,
                            hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    const dim3 g = point_grid(L);
    if (fold && sd) launch_adj_chunks<1, 1>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else if (fold) launch_adj_chunks<1, 0>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else if (sd) launch_adj_chunks<0, 1>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else launch_adj_chunks<0, 0>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    return hipGetLastError();
}

size_t pack_probes_bytes(int S, int nt, int r, int parts) {
    return (size_t)parts * S * ((nt + 15) / 16) * (r / 16) * 64 * 8;
}

hipError_t launch_pack_probes(int S, int nt, int r, int parts, const float *Z, void *zpk, hipStream_t stream) {
    const int64_t total = (int64_t)S * ((nt + 15) / 16) * (r / 16) * 64;
    if (total <= 0) return hipSuccess;
    if (parts != 1 && parts != 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_probes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, S, nt, r, parts,
                       Z, (uint2 *)zpk);
    return hipGetLastError();
}

template <int SD, int ZS>
static void launch_accum_mfma_sd(const Layout &L, dim3 g, hipStream_t stream, const float *ring, int nslots,
                                 int s_lo, int s_hi, const uint2 *zpk, int nkg, int r, float *out) {
    for (int j0 = 0; j0 < r;) {
        const int rm = std::min(4, (r - j0) / 16);
#define TPX_MF(RM) hipLaunchKernelGGL((k_accum_mfma<RM, SD, ZS>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, zpk, nkg, r, j0, out)
        switch (rm) {
        case 4: TPX_MF(4); break;
        case 3: TPX_MF(3); break;
        case 2: TPX_MF(2); break;
        default: TPX_MF(1); break;
        }
#undef TPX_MF
        j0 += 16 * rm;
    }
}

hipError_t launch_accum_mfma(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const void *zpk,
                             int parts, int nt, int r, int sd, float *out, hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    if (r % 16 != 0 || s_lo < 0 || (parts != 1 && parts != 3)) return hipErrorInvalidValue;
    const dim3 g = point_grid(L);
    const int nkg = (nt + 15) / 16;
    const uint2 *zp = (const uint2 *)zpk;
    if (parts == 1) {
        if (sd) launch_accum_mfma_sd<1, 1>(L, g, stream, ring, nslots, s_lo, s_hi, zp, nkg, r, out);
        else launch_accum_mfma_sd<0, 1>(L, g, stream, ring, nslots, s_lo, s_hi, zp, nkg, r, out);
    } else {
        if (sd) launch_accum_mfma_sd<1, 3>(L, g, stream, ring, nslots, s_lo, s_hi, zp, nkg, r, out);
        else launch_accum_mfma_sd<0, 3>(L, g, stream, ring, nslots, s_lo, s_hi, zp, nkg, r, out);
    }
    return hipGetLastError();
}

template <int SD, int ZS>
static void launch_fold_mfma_sd(const Layout &L, dim3 g, hipStream_t stream, const float *ring, int nslots, int s_lo,
                                int s_hi, const float *Z, int nt, int r, const float *ubar, float c, float *gpart) {
    for (int j0 = 0; j0 < r;) {
        const int rk = std::min(4, (r - j0) / 16);
#define TPX_FM(RK) hipLaunchKernelGGL((k_fold_mfma<RK, SD, ZS>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, j0, ubar, c, gpart)
        switch (rk) {
        case 4: TPX_FM(4); break;
        case 3: TPX_FM(3); break;
        case 2: TPX_FM(2); break;
        default: TPX_FM(1); break;
        }
#undef TPX_FM
        j0 += 16 * rk;
    }
}

hipError_t launch_fold_mfma(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int parts, int nt, int r, int sd, const float *ubar, float c, float *gpart,
                            hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    if (r % 16 != 0 || s_lo < 0 || (parts != 1 && parts != 3) || ((uintptr_t)Z & 15) != 0)
        return hipErrorInvalidValue;
    const dim3 g = point_grid(L);
    if (parts == 1) {
        if (sd) launch_fold_mfma_sd<1, 1>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, gpart);
        else launch_fold_mfma_sd<0, 1>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, gpart);
    } else {
        if (sd) launch_fold_mfma_sd<1, 3>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, gpart);
        else launch_fold_mfma_sd<0, 3>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, gpart);
    }
    return hipGetLastError();
}

hipError_t launch_accum_full(const Layout &L, const float *hist, const float *ring, int nslots, int s_lo, int s_hi,
                             float *gpart, hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    hipLaunchKernelGGL(k_accum_full, point_grid(L), dim3(256), 0, stream, L, hist, ring, nslots, s_lo, s_hi, gpart);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// imaging: sums over shots (and probes) in a fixed order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_image_sum(int64_t nphys, int S, const float *__restrict__ gpart,
                                                   float *__restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nphys) return;
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += gpart[(int64_t)s * nphys + p];
    g[p] = acc;
}

__global__ __launch_bounds__(256) void k_image_probed(int64_t nphys, int S, int r, float c,
                                                      const float *__restrict__ ubar, const float *__restrict__ vbar,
                                                      float *__restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nphys) return;
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) {
        float tr = 0.0f;
        for (int j = 0; j < r; ++j) {
            const int64_t e = ((int64_t)s * r + j) * nphys + p;
            tr += ubar[e] * vbar[e];
        }
        acc -= c * tr;
    }
    g[p] = acc;
}

// Imaging condition through a space-only linear operator (Eq. 5): the inner
// product of the centred spatial gradients of the probed fields,
// g = -c sum_shots sum_j sum_axes D ubar_j . D vbar_j, D f = (f[+e] - f[-e]) / 2h;
// the outermost physical nodes get 0.
__global__ __launch_bounds__(256) void k_image_graddot(int64_t nphys, int S, int r, float c, int ndim, int n0, int n1,
                                                       int n2, float inv2h, const float *__restrict__ ubar,
                                                       const float *__restrict__ vbar, float *__restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nphys) return;
    const int x = (int)(p % n0), y = (int)((p / n0) % n1), z = (int)(p / ((int64_t)n0 * n1));
    const bool edge = x == 0 || x == n0 - 1 || z == 0 || z == n2 - 1 || (ndim == 3 && (y == 0 || y == n1 - 1));
    float acc = 0.0f;
    if (!edge) {
        const int64_t ex = 1, ey = n0, ez = (int64_t)n0 * n1;
        for (int s = 0; s < S; ++s) {
            float tr = 0.0f;
            for (int j = 0; j < r; ++j) {
                const int64_t e = ((int64_t)s * r + j) * nphys + p;
                tr += ((ubar[e + ex] - ubar[e - ex]) * inv2h) * ((vbar[e + ex] - vbar[e - ex]) * inv2h);
                if (ndim == 3) tr += ((ubar[e + ey] - ubar[e - ey]) * inv2h) * ((vbar[e + ey] - vbar[e - ey]) * inv2h);
                tr += ((ubar[e + ez] - ubar[e - ez]) * inv2h) * ((vbar[e + ez] - vbar[e - ez]) * inv2h);
            }
            acc -= c * tr;
        }
    }
    g[p] = acc;
}

hipError_t launch_image_graddot(const Layout &L, double h, int r, float c, const float *ubar, const float *vbar,
                                float *g, hipStream_t stream) {
    hipLaunchKernelGGL(k_image_graddot, dim3((unsigned)((L.nphys + 255) / 256)), dim3(256), 0, stream, L.nphys, L.S,
                       r, c, L.ndim, (int)L.n[0], (int)L.n[1], (int)L.n[2], (float)(0.5 / h), ubar, vbar, g);
    return hipGetLastError();
}

hipError_t launch_image_sum(const Layout &L, const float *gpart, float *g, hipStream_t stream) {
    hipLaunchKernelGGL(k_image_sum, dim3((unsigned)((L.nphys + 255) / 256)), dim3(256), 0, stream, L.nphys, L.S,
                       gpart, g);
    return hipGetLastError();
}

hipError_t launch_image_probed(const Layout &L, int r, float c, const float *ubar, const float *vbar, float *g,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_image_probed, dim3((unsigned)((L.nphys + 255) / 256)), dim3(256), 0, stream, L.nphys,
                       L.S, r, c, ubar, vbar, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residual dd = d - d_obs and J = 1/2 sum dd^2: per-block FP64 partial sums
// over fixed contiguous chunks, then one block adds the partials in order.
// ---------------------------------------------------------------------------
constexpr int kResidualMaxParts = 512;

int residual_parts(int64_t n) {
    int64_t p = (n + 4095) / 4096;
    if (p < 1) p = 1;
    if (p > kResidualMaxParts) p = kResidualMaxParts;
    return (int)p;
}

__device__ __forceinline__ double block_sum_fixed(double v, double *sh) {
    // fixed tree within the wavefront, then across the 4 wavefronts in order
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    return t;
}

__global__ __launch_bounds__(256) void k_residual(const float *__restrict__ d, const float *__restrict__ dobs,
                                                  float *__restrict__ res, int64_t n, int64_t chunk,
                                                  double *__restrict__ partials) {
    __shared__ double sh[4];
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    int64_t b1 = b0 + chunk;
    if (b1 > n) b1 = n;
    double acc = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        const float rr = d[i] - dobs[i];
        res[i] = rr;
        acc += (double)rr * (double)rr;
    }
    const double t = block_sum_fixed(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_residual_final(const double *__restrict__ partials, int nparts,
                                                        double *__restrict__ J) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += partials[i];
    const double t = block_sum_fixed(acc, sh);
    if (threadIdx.x == 0) *J = 0.5 * t;
}

hipError_t launch_residual(const float *d, const float *dobs, float *res, int64_t n, double *partials, int nparts,
                           double *J, hipStream_t stream) {
    const int64_t chunk = (n + nparts - 1) / nparts;
    hipLaunchKernelGGL(k_residual, dim3((unsigned)nparts), dim3(256), 0, stream, d, dobs, res, n,
                       chunk > 0 ? chunk : 1, partials);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, stream, partials, nparts, J);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probes from the range of the data covariance (Choice of the probing matrix
// Q, Eq. 6): per shot Q = qr(D D^T Z), D = observed traces as nt x nrec, Z the
// shot's Rademacher probes.  FP64 throughout, fixed summation orders.
// ---------------------------------------------------------------------------

// The D^T Z product is split over kRfSeg time segments, so the launch has
// receivers/64 x shots x kRfSeg blocks; the segments are then summed in order.
constexpr int kRfSeg = 16;

// P[s][seg][i][c] = sum over the segment's samples t of D[s][t][i] Z[s][t][j0 + c].
template <int RC>
__global__ __launch_bounds__(64) void k_rf_dtz(int nt, int nrec, int r, int j0, const float *__restrict__ D,
                                               const float *__restrict__ Z, double *__restrict__ P) {
    const int s = blockIdx.y, seg = blockIdx.z;
    const int i = (int)blockIdx.x * 64 + (int)threadIdx.x;
    if (i >= nrec) return;
    const int len = (nt + kRfSeg - 1) / kRfSeg, t0 = seg * len, t1 = min(nt, t0 + len);
    const float *Ds = D + (int64_t)s * nt * nrec + i;
    const float *Zs = Z + (int64_t)s * nt * r + j0;
    double acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = 0.0;
    for (int t = t0; t < t1; ++t) {
        const double d = (double)Ds[(int64_t)t * nrec];
        const float *zr = Zs + (int64_t)t * r;
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = fma(d, (double)zr[c], acc[c]);
    }
    double *pp = P + (((int64_t)s * kRfSeg + seg) * nrec + i) * RC;
#pragma unroll
    for (int c = 0; c < RC; ++c) pp[c] = acc[c];
}

// W[s][i][j0 + c] = sum_seg P[s][seg][i][c], segments in order.
template <int RC>
__global__ __launch_bounds__(256) void k_rf_dtz_sum(int S, int nrec, int r, int j0, const double *__restrict__ P,
                                                    double *__restrict__ W) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)S * nrec) return;
    const int s = (int)(idx / nrec), i = (int)(idx - (int64_t)s * nrec);
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        double acc = 0.0;
        for (int seg = 0; seg < kRfSeg; ++seg) acc += P[(((int64_t)s * kRfSeg + seg) * nrec + i) * RC + c];
        W[((int64_t)s * nrec + i) * r + j0 + c] = acc;
    }
}

// Y[s][t][j0 + c] = sum_i D[s][t][i] W[s][i][j0 + c]: one wave per time
// sample; lanes stride the receivers, then a fixed butterfly sums the lanes.
template <int RC>
__global__ __launch_bounds__(256) void k_rf_dw(int nt, int nrec, int r, int j0, const float *__restrict__ D,
                                               const double *__restrict__ W, double *__restrict__ Y) {
    const int s = blockIdx.y;
    const int t = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= nt) return;   // whole waves leave together
    const float *Dr = D + ((int64_t)s * nt + t) * nrec;
    const double *Ws = W + (int64_t)s * nrec * r + j0;
    double acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = 0.0;
    for (int i = lane; i < nrec; i += 64) {
        const double d = (double)Dr[i];
        const double *wr = Ws + (int64_t)i * r;
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = fma(d, wr[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
    if (lane == 0) {
        double *y = Y + ((int64_t)s * nt + t) * r + j0;
#pragma unroll
        for (int c = 0; c < RC; ++c) y[c] = acc[c];
    }
}

// ---------------------------------------------------------------------------
// Tall-skinny QR of each shot's Y (nt x r, row-major), in FP64 with the
// unblocked Householder algorithms (the reflector of column j is
// I - tau v v^T with v_j = 1, stored below the diagonal):
//   1. the rows are cut into P panels of at least r rows, each factored by
//      its own block: Y_p = Q_p R_p;
//   2. the stacked R_p (P r x r) are factored by one block per shot, and the
//      explicit factor Q2 is formed in place (accumulated backwards);
//   3. each panel's rows of Q are Q_p Q2_p = H_0 ... H_{r-1} [Q2_p; 0], the
//      panel's reflectors applied backwards to its block of Q2.
// Q = diag(Q_p) Q2 is orthonormal and spans Y's columns.  A block is 1024
// threads: 64 columns x 16 row groups, fixed-order sums.
// ---------------------------------------------------------------------------
struct RfShared {
    double red[1024];
    double tau[64];
    double wv[64];
    double scale;
};

__device__ double rf_block_sum(RfShared &sh, double v) {   // fixed-order tree over the block
    const int tid = threadIdx.x;
    sh.red[tid] = v;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) sh.red[tid] += sh.red[tid + st];
        __syncthreads();
    }
    const double out = sh.red[0];
    __syncthreads();
    return out;
}

// wv[k] = X[j][k] + sum_{t > j} V[t][j] X[t][k] for k in (kmin, r): v^T X with v_j = 1
__device__ void rf_dots(RfShared &sh, const double *V, const double *X, int nrows, int r, int j, int kmin) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double part = 0.0;
    if (tx > kmin && tx < r)
        for (int t = j + 1 + ty; t < nrows; t += 16) part = fma(V[(int64_t)t * r + j], X[(int64_t)t * r + tx], part);
    sh.red[ty * 64 + tx] = part;
    __syncthreads();
    if (ty == 0 && tx > kmin && tx < r) {
        double w = X[(int64_t)j * r + tx];
        for (int g = 0; g < 16; ++g) w += sh.red[g * 64 + tx];
        sh.wv[tx] = w;
    }
    __syncthreads();
}

// X[t][k] -= tau v_t wv[k] for t >= j, k in (kmin, r); column j of V is not written
__device__ void rf_update(RfShared &sh, const double *V, double *X, int nrows, int r, int j, int kmin, double tj) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (tx > kmin && tx < r) {
        const double wk = sh.wv[tx];
        for (int t = j + ty; t < nrows; t += 16) {
            const double vt = t == j ? 1.0 : V[(int64_t)t * r + j];
            X[(int64_t)t * r + tx] -= tj * vt * wk;
        }
    }
    __syncthreads();
}

// In-place Householder factorisation of A (nrows x r, nrows >= r); sh.tau holds the coefficients.
__device__ void rf_householder(RfShared &sh, double *A, int nrows, int r) {
    const int tid = threadIdx.x;
    for (int j = 0; j < r; ++j) {
        double part = 0.0;
        for (int t = j + 1 + tid; t < nrows; t += 1024) {
            const double x = A[(int64_t)t * r + j];
            part = fma(x, x, part);
        }
        const double sigma = rf_block_sum(sh, part);
        if (tid == 0) {
            const double alpha = A[(int64_t)j * r + j];
            if (sigma == 0.0) {          // already upper triangular here: H_j = I
                sh.tau[j] = 0.0;
                sh.scale = 0.0;
            } else {
                const double norm = sqrt(fma(alpha, alpha, sigma));
                const double beta = alpha >= 0.0 ? -norm : norm;
                sh.tau[j] = (beta - alpha) / beta;
                sh.scale = 1.0 / (alpha - beta);
                A[(int64_t)j * r + j] = beta;
            }
        }
        __syncthreads();
        const double tj = sh.tau[j];
        if (tj != 0.0) {
            for (int t = j + 1 + tid; t < nrows; t += 1024) A[(int64_t)t * r + j] *= sh.scale;
            __syncthreads();
            rf_dots(sh, A, A, nrows, r, j, j);
            rf_update(sh, A, A, nrows, r, j, j, tj);
        }
    }
}

__device__ __forceinline__ void rf_panel_rows(int nt, int P, int p, int *row0, int *rows) {
    const int m = nt / P;
    *row0 = p * m;
    *rows = p < P - 1 ? m : nt - (P - 1) * m;
}

__global__ __launch_bounds__(1024) void k_rf_panel_qr(int nt, int r, int P, double *__restrict__ Y,
                                                      double *__restrict__ taus, double *__restrict__ Rs) {
    __shared__ RfShared sh;
    const int s = blockIdx.y, p = blockIdx.x, tid = threadIdx.x;
    int row0, rows;
    rf_panel_rows(nt, P, p, &row0, &rows);
    double *A = Y + ((int64_t)s * nt + row0) * r;
    rf_householder(sh, A, rows, r);
    if (tid < r) taus[((int64_t)s * P + p) * r + tid] = sh.tau[tid];
    double *Rp = Rs + ((int64_t)s * P + p) * r * r;
    for (int idx = tid; idx < r * r; idx += 1024) {
        const int i = idx / r, k = idx - i * r;
        Rp[idx] = k >= i ? A[(int64_t)i * r + k] : 0.0;
    }
}

// the stacked R factors of one shot -> Q2 in place (explicit, accumulated backwards)
__global__ __launch_bounds__(1024) void k_rf_stack_qr(int r, int P, double *__restrict__ Rs) {
    __shared__ RfShared sh;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nrows = P * r;
    double *A = Rs + (int64_t)s * nrows * r;
    rf_householder(sh, A, nrows, r);
    for (int j = r - 1; j >= 0; --j) {
        const double tj = sh.tau[j];
        if (j < r - 1 && tj != 0.0) {
            rf_dots(sh, A, A, nrows, r, j, j);
            rf_update(sh, A, A, nrows, r, j, j, tj);
        }
        for (int t = tid; t < nrows; t += 1024) {
            double *a = &A[(int64_t)t * r + j];
            if (t < j) *a = 0.0;
            else if (t == j) *a = 1.0 - tj;
            else *a = -tj * *a;
        }
        __syncthreads();
    }
}

// rows of panel p of Q = H_0 ... H_{r-1} [Q2_p; 0], written as float
__global__ __launch_bounds__(1024) void k_rf_panel_q(int nt, int r, int P, const double *__restrict__ Y,
                                                     const double *__restrict__ taus, const double *__restrict__ Rs,
                                                     double *__restrict__ B, float *__restrict__ Q) {
    __shared__ RfShared sh;
    const int s = blockIdx.y, p = blockIdx.x, tid = threadIdx.x;
    int row0, rows;
    rf_panel_rows(nt, P, p, &row0, &rows);
    const double *V = Y + ((int64_t)s * nt + row0) * r;
    double *X = B + ((int64_t)s * nt + row0) * r;
    const double *Q2p = Rs + ((int64_t)s * P + p) * r * r;   // rows p r .. p r + r - 1 of Q2
    for (int idx = tid; idx < rows * r; idx += 1024) X[idx] = idx < r * r ? Q2p[idx] : 0.0;
    if (tid < r) sh.tau[tid] = taus[((int64_t)s * P + p) * r + tid];
    __syncthreads();
    for (int j = r - 1; j >= 0; --j) {
        const double tj = sh.tau[j];
        if (tj != 0.0) {
            rf_dots(sh, V, X, rows, r, j, -1);
            rf_update(sh, V, X, rows, r, j, -1, tj);
        }
    }
    float *Qp = Q + ((int64_t)s * nt + row0) * r;
    for (int idx = tid; idx < rows * r; idx += 1024) Qp[idx] = (float)X[idx];
}

// Panels per shot: about sqrt(nt / r) (balancing the panel and the stack
// heights), at most 16, each panel at least r rows.
int rf_panels(int nt, int r) {
    int P = (int)std::lround(std::sqrt((double)nt / (double)r));
    if (P > 16) P = 16;
    while (P > 1 && nt / P < r) --P;
    return P < 1 ? 1 : P;
}

size_t rf_scratch_doubles(int S, int nt, int nrec, int r) {
    const int P = rf_panels(nt, r);
    return (size_t)S * kRfSeg * nrec * 16      // segment partials of D^T Z
           + (size_t)S * P * r                 // panel reflector coefficients
           + (size_t)S * P * r * r             // stacked R factors, then Q2
           + (size_t)S * nt * r;               // rows of Q in FP64
}

hipError_t launch_range_finder(int S, int nt, int nrec, int r, const float *d_obs, float *Z, double *W, double *Y,
                               double *X, hipStream_t stream) {
    if (S < 1 || r < 1 || r > 64 || nrec < 1 || nt < r) return hipErrorInvalidValue;
    const int P = rf_panels(nt, r);
    double *part = X;
    double *taus = part + (size_t)S * kRfSeg * nrec * 16;
    double *Rs = taus + (size_t)S * P * r;
    double *Bq = Rs + (size_t)S * P * r * r;
    const dim3 g1((unsigned)((nrec + 63) / 64), (unsigned)S, (unsigned)kRfSeg);
    const dim3 g1s((unsigned)(((int64_t)S * nrec + 255) / 256));
    const dim3 g2((unsigned)((nt + 3) / 4), (unsigned)S);
    for (int j0 = 0; j0 < r;) {
        int q = 16;
        while (q > r - j0) q >>= 1;   // power-of-two chunks of the probe columns
#define TPX_RF(RC)                                                                                                \
    hipLaunchKernelGGL(k_rf_dtz<RC>, g1, dim3(64), 0, stream, nt, nrec, r, j0, d_obs, (const float *)Z, part);    \
    hipLaunchKernelGGL(k_rf_dtz_sum<RC>, g1s, dim3(256), 0, stream, S, nrec, r, j0, (const double *)part, W);     \
    hipLaunchKernelGGL(k_rf_dw<RC>, g2, dim3(256), 0, stream, nt, nrec, r, j0, d_obs, (const double *)W, Y)
        switch (q) {
        case 16: TPX_RF(16); break;
        case 8: TPX_RF(8); break;
        case 4: TPX_RF(4); break;
        case 2: TPX_RF(2); break;
        default: TPX_RF(1); break;
        }
#undef TPX_RF
        j0 += q;
    }
    // Z is read by the products above before Q overwrites it
    hipLaunchKernelGGL(k_rf_panel_qr, dim3((unsigned)P, (unsigned)S), dim3(1024), 0, stream, nt, r, P, Y, taus, Rs);
    hipLaunchKernelGGL(k_rf_stack_qr, dim3((unsigned)S), dim3(1024), 0, stream, r, P, Rs);
    hipLaunchKernelGGL(k_rf_panel_q, dim3((unsigned)P, (unsigned)S), dim3(1024), 0, stream, nt, r, P,
                       (const double *)Y, (const double *)taus, (const double *)Rs, Bq, Z);
    return hipGetLastError();
}

}  // namespace tpx
