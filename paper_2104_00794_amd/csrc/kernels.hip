// HIP kernels for gfx950 (CDNA4): the acoustic leapfrog step with fused
// source injection and receiver sampling, the on-the-fly probe contractions
// of Algorithm 1, imaging, residual/objective, probe generation and model
// preparation.  Every kernel is deterministic: fixed summation orders, no
// floating-point atomics.
#include <hip/hip_runtime.h>

#include "tpx_internal.h"

namespace tpx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// (distance into the absorbing layer / nbl)^2 along one axis, padded index I
__device__ __forceinline__ float layer_frac2(int64_t I, int64_t nphys, int nb, float inv_nb) {
    int64_t into = 0;
    if (I < nb) into = nb - I;
    else if (I > nb + nphys - 1) into = I - (nb + nphys - 1);
    const float d = (float)into * inv_nb;
    return d * d;
}

// leapfrog update of the damped wave equation for one node:
//   (1 + hd) next = 2 cur - (1 - hd) prev + beta (lap + src),  hd = d dt / 2
__device__ __forceinline__ float leapfrog(float cur, float prev, float beta, float lap, float src, float hd) {
    const float num = 2.0f * cur - (1.0f - hd) * prev + beta * (lap + src);
    return hd == 0.0f ? num : num / (1.0f + hd);
}

// Sampling of `field` at this shot's points (receivers in the forward pass,
// the source in the adjoint pass).  Each point is handled by exactly one
// thread of the shot's blocks; the 2^D products are summed in a fixed order.
template <int NC>
__device__ __forceinline__ void sample_points(const Layout &L, const float *field, int k, const SampleTables &smp,
                                              int shot, int64_t block_in_shot, int64_t blocks_per_shot) {
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

// Gather of the point-source term of one injection tile into LDS: one thread
// per target point, entries summed in their stored order.
__device__ __forceinline__ void gather_sources(const InjectTables &inj, const Amplitude &amp, int shot, int k,
                                               int sb, int se, float *srcs) {
    const float *a = amp.ptr + shot * amp.shot_stride + (int64_t)k * amp.k_stride;
    for (int s = sb + (int)threadIdx.x; s < se; s += blockDim.x) {
        float acc = 0.0f;
        const int e1 = inj.seg_ent[s + 1];
        for (int e = inj.seg_ent[s]; e < e1; ++e) acc += inj.ent_w[e] * a[inj.ent_idx[e]];
        srcs[inj.seg_local[s]] = acc * amp.scale;
    }
}

// ---------------------------------------------------------------------------
// 2D leapfrog step.  Block = 64 x 4 threads over a 64 (x) by 16 (z) tile of
// outputs; u^k is staged with its R-wide halo in LDS, every thread produces
// four outputs of one column.  Grid (x tiles, z tiles, shots).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_step2d(const Layout L, const Physics ph, const StepArgs a) {
    constexpr int W = T2X + 2 * R;
    constexpr int H = T2Z + 2 * R;
    __shared__ float tile[H][W];
    __shared__ float srcs[T2Z * T2X];

    const int tid = threadIdx.x;
    const int lx = tid & 63, ly = tid >> 6;
    const int shot = blockIdx.z;
    const int64_t x0 = (int64_t)blockIdx.x * T2X, z0 = (int64_t)blockIdx.y * T2Z;
    const int64_t G0 = L.G[0];
    const float *cur = a.cur + shot * L.shot_floats;

    for (int row = ly; row < H; row += 4) {
        const int64_t gz = z0 - R + row;
        const float *rowp = cur + (gz + R) * G0 + XO;
        const bool zin = gz < L.P[2] + R;
        for (int col = lx; col < W; col += 64) {
            const int64_t gx = x0 - R + col;
            tile[row][col] = (zin && gx < L.P[0] + R) ? rowp[gx] : 0.0f;
        }
    }

    const int64_t tile_id = ((int64_t)shot * L.ntiles[2] + blockIdx.y) * L.ntiles[0] + blockIdx.x;
    int sb = 0, se = 0;
    if (a.inject) {
        sb = a.inj.tile_ptr[tile_id];
        se = a.inj.tile_ptr[tile_id + 1];
    }
    const bool has_src = sb < se;
    if (has_src)
        for (int i = tid; i < T2Z * T2X; i += 256) srcs[i] = 0.0f;
    __syncthreads();
    if (has_src) {
        gather_sources(a.inj, a.amp, shot, a.k, sb, se, srcs);
        __syncthreads();
    }

    float *next = a.next + shot * L.shot_floats;
    const float *prev = a.prev + shot * L.shot_floats;
#pragma unroll
    for (int q = 0; q < T2Z / 4; ++q) {
        const int lz = ly + 4 * q;
        const int64_t z = z0 + lz, x = x0 + lx;
        if (z >= L.P[2] || x >= L.P[0]) continue;
        const float c = tile[lz + R][lx + R];
        float lap = 2.0f * ph.c[0] * c;
#pragma unroll
        for (int k = 1; k <= R; ++k)
            lap += ph.c[k] * ((tile[lz + R][lx + R - k] + tile[lz + R][lx + R + k]) +
                              (tile[lz + R - k][lx + R] + tile[lz + R + k][lx + R]));
        const int64_t off = (z + R) * G0 + XO + x;
        const float hd = ph.hd_max * (layer_frac2(x, L.n[0], L.nb, ph.inv_nb) + layer_frac2(z, L.n[2], L.nb, ph.inv_nb));
        const float s = has_src ? srcs[lz * T2X + lx] : 0.0f;
        next[off] = leapfrog(c, prev[off], a.beta[off], lap, s, hd);
    }

    if (a.do_sample)
        sample_points<4>(L, cur, a.k, a.smp, shot, (int64_t)blockIdx.y * gridDim.x + blockIdx.x,
                         (int64_t)gridDim.x * gridDim.y);
}

// ---------------------------------------------------------------------------
// 3D leapfrog step.  Block = 64 x 4 threads over a 64 (x) by 4 (y) column
// that marches T3Z planes in z.  z neighbours come from a register queue of
// 2R+1 values per thread; x/y neighbours from the current plane staged in LDS
// with its halo.  Grid (x tiles, y tiles, z chunks * shots).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_step3d(const Layout L, const Physics ph, const StepArgs a, int zchunks) {
    constexpr int W = T3X + 2 * R;
    constexpr int H = T3Y + 2 * R;
    __shared__ float plane_t[H][W];
    __shared__ float srcs[T3Y * T3X];

    const int tid = threadIdx.x;
    const int lx = tid & 63, ly = tid >> 6;
    const int shot = blockIdx.z / zchunks;
    const int zc = blockIdx.z % zchunks;
    const int64_t x0 = (int64_t)blockIdx.x * T3X, y0 = (int64_t)blockIdx.y * T3Y;
    const int64_t zc0 = (int64_t)zc * T3Z;
    const int64_t x = x0 + lx, y = y0 + ly;
    const int64_t G0 = L.G[0], PL = L.G[0] * L.G[1];
    const float *cur = a.cur + shot * L.shot_floats;
    const float *prev = a.prev + shot * L.shot_floats;
    float *next = a.next + shot * L.shot_floats;

    const bool col_ok = x < L.P[0] + R && y < L.P[1] + R;  // readable column (ghosts included)
    const bool out_ok = x < L.P[0] && y < L.P[1];
    // pointer to (x, y, padded z = 0) of this column
    const float *colp = cur + R * PL + (y + L.oy) * G0 + XO + x;

    float q[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) {
        const int64_t z = zc0 - R + i;
        q[i] = (col_ok && z < L.P[2] + R) ? colp[z * PL] : 0.0f;
    }
    const float hdxy = layer_frac2(x, L.n[0], L.nb, ph.inv_nb) + layer_frac2(y, L.n[1], L.nb, ph.inv_nb);

    for (int lz = 0; lz < T3Z; ++lz) {
        const int64_t z = zc0 + lz;
        if (z >= L.P[2]) break;
        q[2 * R] = (col_ok && z + R < L.P[2] + R) ? colp[(z + R) * PL] : 0.0f;

        __syncthreads();  // the previous plane is no longer read
        const float *pz = cur + (z + R) * PL + XO;
        for (int i = tid; i < H * W; i += 256) {
            const int r = i / W, c = i - r * W;
            const int64_t gy = y0 - R + r, gx = x0 - R + c;
            plane_t[r][c] = (gy < L.P[1] + R && gx < L.P[0] + R) ? pz[(gy + L.oy) * G0 + gx] : 0.0f;
        }
        int sb = 0, se = 0;
        if (a.inject) {
            const int64_t tile_id = (((int64_t)shot * L.ntiles[2] + z) * L.ntiles[1] + blockIdx.y) * L.ntiles[0] +
                                    blockIdx.x;
            sb = a.inj.tile_ptr[tile_id];
            se = a.inj.tile_ptr[tile_id + 1];
        }
        const bool has_src = sb < se;
        if (has_src) srcs[tid] = 0.0f;
        __syncthreads();
        if (has_src) {
            gather_sources(a.inj, a.amp, shot, a.k, sb, se, srcs);
            __syncthreads();
        }
        if (out_ok) {
            const float c = q[R];
            float lap = 3.0f * ph.c[0] * c;
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap += ph.c[k] * ((plane_t[ly + R][lx + R - k] + plane_t[ly + R][lx + R + k]) +
                                  (plane_t[ly + R - k][lx + R] + plane_t[ly + R + k][lx + R]) +
                                  (q[R - k] + q[R + k]));
            const int64_t off = (z + R) * PL + (y + L.oy) * G0 + XO + x;
            const float hd = ph.hd_max * (hdxy + layer_frac2(z, L.n[2], L.nb, ph.inv_nb));
            const float s = has_src ? srcs[ly * T3X + lx] : 0.0f;
            next[off] = leapfrog(c, prev[off], a.beta[off], lap, s, hd);
        }
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) q[i] = q[i + 1];
    }

    if (a.do_sample) {
        const int64_t bis = ((int64_t)zc * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        sample_points<8>(L, cur, a.k, a.smp, shot, bis, (int64_t)gridDim.x * gridDim.y * zchunks);
    }
}

template <int NC>
__global__ __launch_bounds__(256) void k_sample(const Layout L, const float *field, int k, const SampleTables smp) {
    const int shot = blockIdx.y;
    sample_points<NC>(L, field + shot * L.shot_floats, k, smp, shot, blockIdx.x, gridDim.x);
}

hipError_t launch_step(const Layout &L, const Physics &ph, const StepArgs &a, hipStream_t stream) {
    if (L.ndim == 2) {
        dim3 grid((unsigned)L.ntiles[0], (unsigned)L.ntiles[2], (unsigned)L.S);
        if (L.R == 2) hipLaunchKernelGGL(k_step2d<2>, grid, dim3(256), 0, stream, L, ph, a);
        else hipLaunchKernelGGL(k_step2d<4>, grid, dim3(256), 0, stream, L, ph, a);
    } else {
        const int zchunks = (int)((L.P[2] + T3Z - 1) / T3Z);
        dim3 grid((unsigned)L.ntiles[0], (unsigned)L.ntiles[1], (unsigned)(zchunks * L.S));
        if (L.R == 2) hipLaunchKernelGGL(k_step3d<2>, grid, dim3(256), 0, stream, L, ph, a, zchunks);
        else hipLaunchKernelGGL(k_step3d<4>, grid, dim3(256), 0, stream, L, ph, a, zchunks);
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
        else z = (float)(__popcll(w) - 32) * 0.25f;
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
// Probe contractions over a block of buffered time steps (Algorithm 1, lines
// 2 and 6, time-blocked): one thread per physical point and shot keeps RC
// accumulators in registers while it streams the buffered slots; the probing
// row Z[s, :] is uniform across the block and is read through scalar loads.
// Grid (x chunks of 256, ny * nz rows, shots).
// ---------------------------------------------------------------------------
struct PointIndex {
    int64_t off;  // offset within a shot field
    int64_t p;    // flat physical index
    bool ok;
};

__device__ __forceinline__ PointIndex point_index(const Layout &L) {
    PointIndex pi;
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = blockIdx.y;
    const int64_t z = row / L.n[1], y = row - z * L.n[1];
    pi.ok = x < L.n[0];
    const int64_t oyb = L.ndim == 3 ? L.nb : 0;
    pi.off = L.pad_off(x + L.nb, y + oyb, z + L.nb);
    pi.p = row * L.n[0] + x;
    return pi;
}

template <int RC>
__global__ __launch_bounds__(256) void k_accum_fwd(const Layout L, const float *__restrict__ ring, int nslots,
                                                   int s_lo, int s_hi, const float *__restrict__ Z, int nt, int r,
                                                   float *__restrict__ ubar) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.z;
    const float *base = ring + shot * L.shot_floats + pi.off;
    for (int j0 = 0; j0 < r; j0 += RC) {
        const int rc = (r - j0) < RC ? (r - j0) : RC;
        float acc[RC];
#pragma unroll
        for (int j = 0; j < RC; ++j) acc[j] = 0.0f;
        for (int s = s_lo; s <= s_hi; ++s) {
            const float v = base[(int64_t)(s % nslots) * L.slot_floats];
            const float *zr = Z + ((int64_t)shot * nt + s) * r + j0;
#pragma unroll
            for (int j = 0; j < RC; ++j)
                if (j < rc) acc[j] += zr[j] * v;
        }
        float *ub = ubar + ((int64_t)shot * r + j0) * L.nphys + pi.p;
#pragma unroll
        for (int j = 0; j < RC; ++j)
            if (j < rc) ub[(int64_t)j * L.nphys] += acc[j];
    }
}

template <int RC, int FOLD>
__global__ __launch_bounds__(256) void k_accum_adj(const Layout L, const float *__restrict__ ring, int nslots,
                                                   int s_lo, int s_hi, const float *__restrict__ Z, int nt, int r,
                                                   const float *__restrict__ ubar, float c,
                                                   float *__restrict__ vbar, float *__restrict__ gpart) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.z;
    const float *base = ring + shot * L.shot_floats + pi.off;
    float gacc = 0.0f;
    for (int j0 = 0; j0 < r; j0 += RC) {
        const int rc = (r - j0) < RC ? (r - j0) : RC;
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
            for (int j = 0; j < RC; ++j)
                if (j < rc) u[j] = ub[(int64_t)j * L.nphys];
        }
        float lm = base[(int64_t)((s_lo - 1) % nslots) * L.slot_floats];
        float l0 = base[(int64_t)(s_lo % nslots) * L.slot_floats];
        float fsum = 0.0f;
        for (int s = s_lo; s <= s_hi; ++s) {
            const float lp = base[(int64_t)((s + 1) % nslots) * L.slot_floats];
            const float w = (lm - 2.0f * l0) + lp;
            const float *zr = Z + ((int64_t)shot * nt + s) * r + j0;
            if (FOLD) {
                float t = 0.0f;
#pragma unroll
                for (int j = 0; j < RC; ++j)
                    if (j < rc) t += zr[j] * u[j];
                fsum += w * t;
            } else {
#pragma unroll
                for (int j = 0; j < RC; ++j)
                    if (j < rc) acc[j] += zr[j] * w;
            }
            lm = l0;
            l0 = lp;
        }
        if (FOLD) {
            gacc += fsum;
        } else {
            float *vb = vbar + ((int64_t)shot * r + j0) * L.nphys + pi.p;
#pragma unroll
            for (int j = 0; j < RC; ++j)
                if (j < rc) vb[(int64_t)j * L.nphys] += acc[j];
        }
    }
    if (FOLD) gpart[(int64_t)shot * L.nphys + pi.p] -= c * gacc;
}

__global__ __launch_bounds__(256) void k_accum_full(const Layout L, const float *__restrict__ hist,
                                                    const float *__restrict__ ring, int nslots, int s_lo, int s_hi,
                                                    float *__restrict__ gpart) {
    const PointIndex pi = point_index(L);
    if (!pi.ok) return;
    const int shot = blockIdx.z;
    const float *hb = hist + shot * L.shot_floats + pi.off;
    const float *base = ring + shot * L.shot_floats + pi.off;
    float lm = base[(int64_t)((s_lo - 1) % nslots) * L.slot_floats];
    float l0 = base[(int64_t)(s_lo % nslots) * L.slot_floats];
    float acc = 0.0f;
    for (int s = s_lo; s <= s_hi; ++s) {
        const float lp = base[(int64_t)((s + 1) % nslots) * L.slot_floats];
        const float w = (lm - 2.0f * l0) + lp;
        acc += hb[(int64_t)s * L.slot_floats] * w;
        lm = l0;
        l0 = lp;
    }
    gpart[(int64_t)shot * L.nphys + pi.p] -= acc;
}

static dim3 point_grid(const Layout &L) {
    return dim3((unsigned)((L.n[0] + 255) / 256), (unsigned)(L.n[1] * L.n[2]), (unsigned)L.S);
}

hipError_t launch_accum_fwd(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int nt, int r, float *ubar, hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    const dim3 g = point_grid(L);
    if (r <= 8) hipLaunchKernelGGL(k_accum_fwd<8>, g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar);
    else if (r <= 16) hipLaunchKernelGGL(k_accum_fwd<16>, g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar);
    else if (r <= 32) hipLaunchKernelGGL(k_accum_fwd<32>, g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar);
    else hipLaunchKernelGGL(k_accum_fwd<64>, g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar);
    return hipGetLastError();
}

template <int FOLD>
static void launch_adj_rc(const Layout &L, dim3 g, hipStream_t stream, const float *ring, int nslots, int s_lo,
                          int s_hi, const float *Z, int nt, int r, const float *ubar, float c, float *vbar,
                          float *gpart) {
    if (r <= 8) hipLaunchKernelGGL((k_accum_adj<8, FOLD>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else if (r <= 16) hipLaunchKernelGGL((k_accum_adj<16, FOLD>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else if (r <= 32) hipLaunchKernelGGL((k_accum_adj<32, FOLD>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else hipLaunchKernelGGL((k_accum_adj<64, FOLD>), g, dim3(256), 0, stream, L, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
}

hipError_t launch_accum_adj(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int nt, int r, int fold, const float *ubar, float c, float *vbar, float *gpart,
                            hipStream_t stream) {
    if (s_hi < s_lo) return hipSuccess;
    const dim3 g = point_grid(L);
    if (fold) launch_adj_rc<1>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
    else launch_adj_rc<0>(L, g, stream, ring, nslots, s_lo, s_hi, Z, nt, r, ubar, c, vbar, gpart);
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

}  // namespace tpx
