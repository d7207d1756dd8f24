// Internal declarations shared by the host runtime (runtime.cpp) and the
// kernels (kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

#include "tpx.h"

namespace tpx {

// ---------------------------------------------------------------------------
// Field layout in HBM.
//
// One wavefield "slot" holds all S shots: [shot][zg][yg][xg] with
//   xg in [0, G0): the padded box starts at XO (a 128-byte aligned offset that
//                  also serves as the left ghost border), pitch G0 is a
//                  multiple of 32 floats;
//   yg in [0, G1): 3D only, R ghost planes on each side (2D: G1 = 1);
//   zg in [0, G2): R ghost rows on each side.
// The field is zero outside the padded box (Dirichlet condition).  Kernels
// read only nodes of the padded box and substitute zero elsewhere, so ghost
// cells never need clearing.
// ---------------------------------------------------------------------------
constexpr int XO = 32;

// 2D step kernel tile: T2Z rows by 64 - 2R columns of outputs, 256 threads.
// One wave spans the tile's columns plus an R-wide halo on each side: the
// region on which the first of two fused steps is computed.  Problems too
// small to give every CU two such tiles per launch use shorter tiles (more
// tiles, more halo work per tile): T2Z_MID rows down to 384 tiles of T2Z
// rows, T2Z_SMALL rows below that.
constexpr int T2Z = 32;
constexpr int T2Z_MID = 16;
constexpr int T2Z_SMALL = 8;
__host__ __device__ constexpr int t2x(int R) { return 64 - 2 * R; }
// Three-step 2D kernel: the two-step tiles' height by 64 - 4R columns; lane l holds column
// x0 - 2R + l, so a wave row covers the tile plus a 2R-wide halo (the region
// of the first of its three steps).
__host__ __device__ constexpr int t3x(int R) { return 64 - 4 * R; }
// One-step 3D kernel: blocks of 64 (x) by 8 (y) columns, marching T3Z planes in z.
constexpr int T3X = 64;
constexpr int T3Y = 8;
constexpr int T3Z = 12;
// Two-step 3D kernel, whose tiles also key the 3D injection tables: T3Y2 rows
// (y) by 64 - 2R columns (x), so one wave row spans the tile plus an R-wide
// halo on each side; eight waves; z chunks of Layout::tz3 planes.
constexpr int T3Y2 = 16;

struct Layout {
    int ndim;      // 2 or 3
    int R;         // stencil half-width = order / 2
    int nb;        // absorbing nodes per face
    int S;         // shots in a slot
    int64_t n[3];  // physical nodes x, y, z (2D: n[1] = 1)
    int64_t P[3];  // padded box (2D: P[1] = 1)
    int64_t G[3];  // allocated extents incl. ghosts: G[0] = pitch
    int64_t oy;    // ghost offset along y (R in 3D, 0 in 2D)
    int64_t shot_floats;  // G0 * G1 * G2
    int64_t slot_floats;  // S * shot_floats
    int64_t nphys;        // n0 * n1 * n2
    int64_t npad;         // P0 * P1 * P2
    // tiles of the step kernel (used by the injection tables)
    int tile[3];
    int64_t ntiles[3];
    int tz3;              // 3D: planes per z chunk of the two-step kernel
    int64_t tiles_per_shot;
    // injection map of one tile: extents and origin relative to the tile's
    // first node (2D: 64 x (T2Z + 2R) nodes from (-R, -R); 3D, per plane:
    // 64 x (T3Y2 + 2R) nodes from (-R, -R))
    int map[3];
    int map_org[3];

    // offset (floats, within one shot) of padded node (ix, iy, iz)
    __host__ __device__ inline int64_t pad_off(int64_t ix, int64_t iy, int64_t iz) const {
        return ((iz + R) * G[1] + (iy + oy)) * G[0] + XO + ix;
    }
};

// Stencil/physics constants passed to the step kernels.
struct Physics {
    float c[5];        // Laplacian weights divided by h^2 (c[0] centre per axis)
    float hd_max;      // dmax * dt / 2 (damping at the outermost node, per axis)
    float inv_nb;      // 1 / nbl (0 when nbl == 0)
};

// Point-source injection into one step.  A segment is the ordered run of
// (source index, weight) entries of one target node.  tile_dense[tile] is -1
// for a tile whose map holds no source node, else the index of its dense map:
// dense[map * map_nodes + local node] = segment of that node or -1.  A node
// inside several tiles' maps has the same segment contents in each.
struct InjectTables {
    const int32_t *tile_dense; // [S * tiles_per_shot]
    const int32_t *dense;      // [maps][nodes per tile]
    const int32_t *seg_ent;    // [nseg + 1] entry ranges
    const int32_t *ent_idx;    // [nent] source index (receiver id or 0)
    const float *ent_w;        // [nent] interpolation weight
    const int32_t *col_z;      // 3D: [S * ntiles_y * ntiles_x][2] first and last plane with a map (empty: lo > hi)
};

// Amplitudes injected at step k: amp[shot * shot_stride + k * k_stride + idx] * scale
struct Amplitude {
    const float *ptr;
    int64_t shot_stride;
    int64_t k_stride;
    float scale;
};

// Sampling: per shot, nsmp points with a base offset and 2^D weights.
struct SampleTables {
    int32_t nsmp;             // samples per shot (receivers or 1 source)
    const int32_t *base;      // [S][nsmp] offset of the base node within a shot field
    const float *w;           // [S][nsmp][2^D]
    float *out;               // out[shot * out_shot_stride + k * out_k_stride + i] = scale * sum
    int64_t out_shot_stride;
    int64_t out_k_stride;
    float scale;
};

// One launch advances one or two leapfrog steps.  Time runs forward (u^k ->
// u^{k+1}) or backward (adjoint: lambda^k -> lambda^{k-1}); "next" is the
// level after `cur` in the direction of the loop.
struct StepArgs {
    const float *cur;   // u^k (slot base, shot 0)
    const float *prev;  // u^{k-1}
    float *next;        // u^{k+1}
    float *next2;       // u^{k+2} (launches of two or three steps)
    float *next3;       // u^{k+3} (three-step launches only)
    const float *beta;  // dt^2 / m_pad, one shot-sized field
    const float *prev2; // the level before `prev` (sampled only)
    int nstep;          // 1, 2 or 3 (3: 2D only)
    int k;              // time index of `cur`: amplitudes of the first step, sample row of `cur`
    int k2;             // amplitude index of the second step
    int k3;             // amplitude index of the third step
    int kp;             // time index of `prev` (its sample row)
    int kp2;            // time index of `prev2` (its sample row)
    int inject;         // 0/1
    int do_sample;      // 0/1: sample `cur` at row k
    int sample_prev;    // 0/1: sample `prev` at row kp
    int sample_prev2;   // 0/1: sample `prev2` at row kp2 (the middle level of a three-step launch)
    InjectTables inj;
    Amplitude amp;
    SampleTables smp;
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All are asynchronous on `stream`.
// ---------------------------------------------------------------------------
hipError_t launch_step(const Layout &L, const Physics &ph, const StepArgs &a, hipStream_t stream);
hipError_t launch_sample_only(const Layout &L, const float *field, int k, const SampleTables &smp,
                              hipStream_t stream);
hipError_t launch_model_prep(const Layout &L, const float *m, double dt, float m_min, float *beta, int32_t *flags,
                             hipStream_t stream);
hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t stream);
// Identity of a probed forward pass (problem sizes and probe set), kept after
// ubar in its state buffer.
struct StateHeader {
    static constexpr int kWords = 16;
    int32_t w[kWords];
};
// check == 0: write h into hdr; check == 1: set flags bit 2 where hdr differs from h.
hipError_t launch_state_header(const StateHeader &h, void *hdr, int32_t *flags, int check, hipStream_t stream);
hipError_t launch_probe_gen(int kind, int r, uint64_t seed, int nt, int shot0, int nshots, float *Z,
                            hipStream_t stream);
hipError_t launch_probe_copy(const float *Zsrc, int64_t n, float *Zdst, hipStream_t stream);

// ubar[shot][j][p] += sum_{s=s_lo}^{s_hi} Z[shot][s][j] * u^s[p]  (physical p)
hipError_t launch_accum_fwd(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi,
                            const float *Z, int nt, int r, float *ubar, hipStream_t stream);
// w^s from the buffered field f: f^{s-1} - 2 f^s + f^{s+1} (sd == 1) or f^s
// (sd == 0), s = s_lo..s_hi; either
//   vbar[shot][j][p] += sum_s Z[shot][s][j] w^s[p]          (fold == 0), or
//   gpart[shot][p]   += -c sum_s w^s[p] sum_j Z[s][j] ubar_j[p]   (fold == 1)
hipError_t launch_accum_adj(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi,
                            const float *Z, int nt, int r, int fold, int sd, const float *ubar, float c,
                            float *vbar, float *gpart, hipStream_t stream);
// The same contractions on the matrix cores, r a multiple of 16.  parts = 1
// for probes exact in bfloat16 (three bf16 products per tile), 3 for any
// other probes (each value split in three; six products).  zpk: the probes
// packed by launch_pack_probes (parts * S * ceil(nt/16) * r/16 * 64 entries of
// 8 bytes).
//   out[shot][j][p] += sum_s Z[shot][s][j] w^s[p]      (launch_accum_mfma)
//   gpart[shot][p]  += -c sum_s w^s[p] sum_j Z[s][j] ubar_j[p]   (launch_fold_mfma, Z as floats, 16-byte aligned)
// w^s as above (sd selects the second difference); s_lo >= 0.
size_t pack_probes_bytes(int S, int nt, int r, int parts);
hipError_t launch_pack_probes(int S, int nt, int r, int parts, const float *Z, void *zpk, hipStream_t stream);
hipError_t launch_accum_mfma(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const void *zpk,
                             int parts, int nt, int r, int sd, float *out, hipStream_t stream);
hipError_t launch_fold_mfma(const Layout &L, const float *ring, int nslots, int s_lo, int s_hi, const float *Z,
                            int parts, int nt, int r, int sd, const float *ubar, float c, float *gpart,
                            hipStream_t stream);
// gpart[shot][p] += - sum_s u^s[p] w^s[p], u^s from the full history (slot s)
hipError_t launch_accum_full(const Layout &L, const float *hist, const float *ring, int nslots, int s_lo,
                             int s_hi, float *gpart, hipStream_t stream);
// g[p] = sum_shot gpart[shot][p]   or   g[p] = -c sum_shot sum_j ubar vbar
hipError_t launch_image_sum(const Layout &L, const float *gpart, float *g, hipStream_t stream);
hipError_t launch_image_probed(const Layout &L, int r, float c, const float *ubar, const float *vbar, float *g,
                               hipStream_t stream);
// g = -c sum_shot sum_j grad ubar_j . grad vbar_j (centred differences, grid step h;
// 0 on the outermost physical nodes)
hipError_t launch_image_graddot(const Layout &L, double h, int r, float c, const float *ubar, const float *vbar,
                                float *g, hipStream_t stream);
// Probes from the range of the data covariance: Z[S][nt][r] holds the shots'
// Rademacher probes on entry and Q = qr(D D^T Z) on exit.  W (S*nrec*r), Y
// (S*nt*r) and X (rf_scratch_doubles) are FP64 scratch.  r <= 64, nt >= r.
size_t rf_scratch_doubles(int S, int nt, int nrec, int r);   // X below, in doubles
hipError_t launch_range_finder(int S, int nt, int nrec, int r, const float *d_obs, float *Z, double *W, double *Y,
                               double *X, hipStream_t stream);
// res = d - d_obs; J = 1/2 sum res^2 (deterministic two-pass FP64 reduction)
hipError_t launch_residual(const float *d, const float *dobs, float *res, int64_t n, double *partials,
                           int nparts, double *J, hipStream_t stream);
int residual_parts(int64_t n);

// Host runtime (runtime.cpp).  The probed gradient of tpx_gradient_probed run
// in `scratch` (scratch_bytes long) without any allocation by the library:
// geometry tables are copied from pageable host memory (the call waits for
// that copy), contractions run in stream order.  Returns TPX_E_NOMEM, with a
// message, when the problem needs more than scratch_bytes.
tpx_status gradient_probed_in_scratch(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                      const float *m, const float *d_obs, float *g, double *J, float *d_out,
                                      void *scratch, size_t scratch_bytes, void *stream);
// Record `msg` as the calling thread's tpx_last_error.
void set_error(tpx_status st, const char *msg);

}  // namespace tpx
