// U-Net kernels for gfx950: bf16 MFMA implicit-GEMM convolutions with FP32
// accumulation, and the pointwise / pooling / resampling / loss / optimiser
// kernels around them.  Activations are NHWC with a channel count that is a
// multiple of 32.
//
// MFMA v_mfma_f32_16x16x32_bf16 operand layout (64 lanes):
//   A (16 x 32): lane l holds row l % 16, k = 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16): lane l holds col l % 16, the same k range
//   D (16 x 16): lane l holds col l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3
#include <algorithm>
#include <array>
#include <map>
#include <mutex>

#include "unet_internal.h"

namespace helm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Raw buffer loads (descriptor word 3 of the gfx9 family: 32-bit data
// format, no swizzle).  An offset at or past num_records returns zero
// without touching memory; BUF_NONE is such an offset for every buffer
// below 2 GB.
constexpr int BUF_DWORD3 = 0x00020000;
constexpr int BUF_NONE = 0x7fffffff;
__device__ __forceinline__ uint4 ld_buf16(__amdgpu_buffer_rsrc_t r, int off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// 8 bf16 channels <-> 8 floats (16-byte vectors)
struct f8 {
    float v[8];
};
__device__ __forceinline__ f8 ld8(const bf16 *p)
{
    uint4 u = *reinterpret_cast<const uint4 *>(p);
    const bf16 *e = reinterpret_cast<const bf16 *>(&u);
    f8 r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r.v[q] = (float)e[q];
    return r;
}
__device__ __forceinline__ f8 u4_to_f8(const uint4 &u)
{
    const bf16 *e = reinterpret_cast<const bf16 *>(&u);
    f8 r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r.v[q] = (float)e[q];
    return r;
}
__device__ __forceinline__ void st8(bf16 *p, const f8 &r)
{
    uint4 u;
    bf16 *e = reinterpret_cast<bf16 *>(&u);
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = (bf16)r.v[q];
    *reinterpret_cast<uint4 *>(p) = u;
}

// Bilinear x2 upsampling with half-pixel centres: fine index o of a line of
// n coarse samples reads coarse i0 and i1 with weights 1 - l1 and l1 (edges
// clamped); up_blend8 blends eight channels of the four coarse samples.
__device__ __forceinline__ void up_src(int o, int n, int &i0, int &i1, float &l1)
{
    float src = (o + 0.5f) * 0.5f - 0.5f;
    src = src < 0.f ? 0.f : src;
    i0 = (int)src;
    i1 = i0 + 1 < n ? i0 + 1 : n - 1;
    l1 = src - (float)i0;
}

__device__ __forceinline__ f8 up_blend8(const f8 &a00, const f8 &a01, const f8 &a10, const f8 &a11, float ly,
                                        float lx)
{
    f8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        o.v[q] = (1.f - ly) * ((1.f - lx) * a00.v[q] + lx * a01.v[q]) + ly * ((1.f - lx) * a10.v[q] + lx * a11.v[q]);
    return o;
}

// Epilogue of a finished tile: rows y0 .. y0 + MF - 1 of this wavefront,
// pixel x = lane % 16 column of the tile, channels co0 + 16 nf + 4 (lane /
// 16) .. + 3 of fragment nf.  bn(c, sc, sh) gives the folded BN of block
// channels c .. c + 3.  Clears acc.
// Issues (without waiting) the context-map loads of the epilogue below for
// the same tile rows, pixel and channels: branch-free buffer loads, pieces
// outside the image or Cout read as zero.
template <int MF, int NF>
__device__ __forceinline__ void conv_cmap_issue(f16x4 (&mp)[MF][NF], int lane, int y0, int x, int H, int W, int Cout,
                                                int co0, const ConvEpi &epi)
{
    const bool full_co = co0 + 16 * NF <= Cout;
    const __amdgpu_buffer_rsrc_t mr =
        __builtin_amdgcn_make_buffer_rsrc((void *)epi.cmap, 0, (int)((size_t)H * W * Cout * 2), BUF_DWORD3);
#pragma unroll
    for (int mf = 0; mf < MF; ++mf)
#pragma unroll
        for (int nf = 0; nf < NF; ++nf) {
            const int y = y0 + mf, c = co0 + 4 * (lane >> 4) + nf * 16;
            const bool ok = y < H && x < W && (full_co || c < Cout);
            mp[mf][nf] = __builtin_bit_cast(
                f16x4, __builtin_amdgcn_raw_buffer_load_b64(mr, ok ? ((y * W + x) * Cout + c) * 2 : BUF_NONE, 0, 0));
        }
}

// PRE: the caller has issued the context-map loads into mp with
// conv_cmap_issue (so that they overlap its MFMAs), and PREWAIT vector memory
// operations issued after them may stay in flight when they are waited for;
// otherwise the epilogue issues them itself.  The plain epilogue (EPI 0)
// stores with buffer stores on every lane (pieces outside the image or Cout
// fall outside the buffer's range and are dropped), so it issues a fixed
// number of vector memory operations: MF NF / 2 in mode 1, MF NF in mode 0.
template <int MF, int NF, int EPI, bool PRE = false, int PREWAIT = 0, class BN>
__device__ __forceinline__ void conv_epilogue(f32x4 (&acc)[MF][NF], f16x4 (&mp)[MF][NF], int lane, int b, int y0,
                                              int x, int H, int W, int Cout, int co0, int mode,
                                              float *__restrict__ out32, bf16 *__restrict__ out16, float slope,
                                              const ConvEpi &epi, BN bn)
{
    constexpr int CO = 16 * NF;
    if constexpr (EPI == 0) {
        static_assert(NF % 2 == 0, "fragment pairs");
        // the tile is complete: lane (l % 16, l / 16) holds pixel x0 + l % 16
        // of each row and channels 4 (l / 16) .. + 3 of each fragment
        const bool full_co = co0 + CO <= Cout;
        // folded BN of the four output channels each lane stores (Cout is
        // a multiple of 32, so the four are in range together)
        float4 sc[NF], sh[NF];
#pragma unroll
        for (int nf = 0; nf < NF; ++nf) bn(nf * 16 + 4 * (lane >> 4), sc[nf], sh[nf]);
        // the context map of the whole tile first (all loads issue before
        // the first wait)
        if (mode == 1 && epi.cmap) {
            if constexpr (!PRE) conv_cmap_issue<MF, NF>(mp, lane, y0, x, H, W, Cout, co0, epi);
            // one wait here, on every lane
            if constexpr (PRE && PREWAIT > 0)
                __builtin_amdgcn_s_waitcnt((PREWAIT & 15) | ((PREWAIT >> 4) << 14) | (7 << 4) | (15 << 8));
            else
                __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0); expcnt, lgkmcnt untouched
        } else {
#pragma unroll
            for (int mf = 0; mf < MF; ++mf)
#pragma unroll
                for (int nf = 0; nf < NF; ++nf) mp[mf][nf] = f16x4{};
        }
        // this wavefront's rows: yw .. yw + rows - 1 of image b
        const int yw = __builtin_amdgcn_readfirstlane(y0);
        const int rows = max(0, min(MF, H - yw));  // 0 for rows past a ragged image's end
        const size_t row0 = ((size_t)b * H + yw) * W;
        const bool x_ok = x < W;
        typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        if (mode == 1) {
            // 16-byte stores: lanes l and l ^ 16 swap one of their two
            // fragments' 8 bytes, so that lane (x, q) holds 8 consecutive
            // channels of fragment pair np: 4 q .. 4 q + 7 of fragment np (q
            // even) or 16 + 4 (q - 1) .. of fragment np + 1 (q odd)
            const int q = lane >> 4;
            const bool odd = q & 1;
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const __amdgpu_buffer_rsrc_t r16 = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(out16 + row0 * Cout), 0, (int)((size_t)rows * W * Cout * 2), BUF_DWORD3);
#pragma unroll
            for (int mf = 0; mf < MF; ++mf) {
#pragma unroll
                for (int np = 0; np < NF; np += 2) {
                    uint2 o[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int nf = np + h;
                        const f32x4 v = acc[mf][nf];
                        const f16x4 m = mp[mf][nf];
                        float z0 = (v[0] + (float)m[0]) * sc[nf].x + sh[nf].x;
                        float z1 = (v[1] + (float)m[1]) * sc[nf].y + sh[nf].y;
                        float z2 = (v[2] + (float)m[2]) * sc[nf].z + sh[nf].z;
                        float z3 = (v[3] + (float)m[3]) * sc[nf].w + sh[nf].w;
                        z0 = z0 > 0.f ? z0 : slope * z0;
                        z1 = z1 > 0.f ? z1 : slope * z1;
                        z2 = z2 > 0.f ? z2 : slope * z2;
                        z3 = z3 > 0.f ? z3 : slope * z3;
                        const bf16x4 t = {(bf16)z0, (bf16)z1, (bf16)z2, (bf16)z3};
                        o[h] = __builtin_bit_cast(uint2, t);
                        acc[mf][nf] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
                    const uint2 snd = odd ? o[0] : o[1];
                    const uint2 rcv =
                        make_uint2((unsigned)__shfl_xor((int)snd.x, 16), (unsigned)__shfl_xor((int)snd.y, 16));
                    const u32x4 d = odd ? u32x4{rcv.x, rcv.y, o[1].x, o[1].y} : u32x4{o[0].x, o[0].y, rcv.x, rcv.y};
                    const int ch = odd ? (np + 1) * 16 + 4 * (q - 1) : np * 16 + 4 * q;
                    const bool ok = mf < rows && x_ok && (full_co || co0 + ch < Cout);
                    const int off = ok ? (int)((((size_t)mf * W + x) * Cout + co0 + ch) * 2) : BUF_NONE;
                    if (epi.nt)
                        __builtin_amdgcn_raw_buffer_store_b128(d, r16, off, 0, 2);  // nontemporal
                    else
                        __builtin_amdgcn_raw_buffer_store_b128(d, r16, off, 0, 0);
                }
            }
        } else {
            // raw FP32 (or FP16 with raw16) output, optionally routed by
            // channel range
            const __amdgpu_buffer_rsrc_t r32 = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(out32 + row0 * Cout), 0, (int)((size_t)rows * W * Cout * 4), BUF_DWORD3);
#pragma unroll
            for (int nf = 0; nf < NF; ++nf) {
                // the channel range holding fragment nf (range ends are
                // multiples of 16, so the choice is the same on every lane)
                const int c0 = __builtin_amdgcn_readfirstlane(co0 + nf * 16), c = c0 + 4 * (lane >> 4);
                const bool c_ok = full_co || c < Cout;
                __amdgpu_buffer_rsrc_t rr = r32;
                int cs = Cout, cc = c;
                if (epi.raw16) {
                    rr = __builtin_amdgcn_make_buffer_rsrc((void *)(epi.raw16 + row0 * Cout), 0,
                                                           (int)((size_t)rows * W * Cout * 2), BUF_DWORD3);
                } else if (epi.nseg) {
                    int k = 0, lo = 0;
                    while (k < epi.nseg - 1 && c0 >= epi.seg_hi[k]) {
                        lo = epi.seg_hi[k];
                        ++k;
                    }
                    if (epi.seg_p[k]) {
                        cs = epi.seg_C[k];
                        cc = c - lo;
                        rr = __builtin_amdgcn_make_buffer_rsrc((void *)(epi.seg_p[k] + row0 * cs), 0,
                                                               (int)((size_t)rows * W * cs * 4), BUF_DWORD3);
                    }
                }
#pragma unroll
                for (int mf = 0; mf < MF; ++mf) {
                    const f32x4 v = acc[mf][nf];
                    const bool ok = mf < rows && x_ok && c_ok;
                    if (epi.raw16) {
                        const f16x4 h4 = {(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
                        const int off = ok ? (int)((((size_t)mf * W + x) * Cout + c) * 2) : BUF_NONE;
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, h4), rr, off, 0, 0);
                    } else {
                        const int off = ok ? (int)((((size_t)mf * W + x) * cs + cc) * 4) : BUF_NONE;
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rr, off, 0, 0);
                    }
                    acc[mf][nf] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            }
        }
    } else {
        // inference epilogue with pooling (EPI 1) or the 1x1 head (EPI 2):
        // lane (l % 16, l / 16) holds pixel x0 + l % 16 of each row and
        // channels 4 (l / 16) .. + 3 of each fragment
        const int cl = 4 * (lane >> 4);
        const bool full_co = co0 + CO <= Cout;
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        float s0[MF], s1[MF];  // head partial sums per row
#pragma unroll
        for (int mf = 0; mf < MF; ++mf) s0[mf] = s1[mf] = 0.f;
        // one channel fragment at a time (bounds the live registers)
#pragma unroll
        for (int nf = 0; nf < NF; ++nf) {
            const int co = co0 + nf * 16 + cl;
            const bool co_ok = full_co || co < Cout;
            float4 sc, sh;
            bn(nf * 16 + cl, sc, sh);
            const float scv[4] = {sc.x, sc.y, sc.z, sc.w}, shv[4] = {sh.x, sh.y, sh.z, sh.w};
            // folded BN and LeakyReLU, rounded to bf16 (kept as floats)
#pragma unroll
            for (int mf = 0; mf < MF; ++mf) {
                const int y = y0 + mf;
                float mv[4] = {0.f, 0.f, 0.f, 0.f};
                if (epi.cmap && y < H && x < W && co_ok) {
                    const f16x4 m = *reinterpret_cast<const f16x4 *>(epi.cmap + ((size_t)y * W + x) * Cout + co);
#pragma unroll
                    for (int q = 0; q < 4; ++q) mv[q] = (float)m[q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float z = (acc[mf][nf][q] + mv[q]) * scv[q] + shv[q];
                    z = z > 0.f ? z : slope * z;
                    acc[mf][nf][q] = (float)(bf16)z;
                }
            }
            if (EPI != 2) {
#pragma unroll
                for (int mf = 0; mf < MF; ++mf) {
                    const int y = y0 + mf;
                    if (y < H && x < W && co_ok) {
                        const f32x4 v = acc[mf][nf];
                        bf16x4 o = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
                        *reinterpret_cast<bf16x4 *>(out16 + (((size_t)b * H + y) * W + x) * Cout + co) = o;
                    }
                }
            }
            if (EPI == 1) {
                // 2x2 max pooling: rows mf, mf + 1 of this wavefront, pixels
                // x, x + 1 in lanes l, l ^ 1 (H and W are even)
#pragma unroll
                for (int mf = 0; mf < MF; mf += 2) {
                    const int y = y0 + mf;
                    float m[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        m[q] = fmaxf(acc[mf][nf][q], acc[mf + 1][nf][q]);
                        m[q] = fmaxf(m[q], __shfl_xor(m[q], 1));
                    }
                    if ((x & 1) == 0 && y < H && x < W && co_ok) {
                        bf16x4 o = {(bf16)m[0], (bf16)m[1], (bf16)m[2], (bf16)m[3]};
                        *reinterpret_cast<bf16x4 *>(
                            epi.pool + (((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cout + co) = o;
                    }
                }
            }
            if (EPI == 2 && co_ok) {
                const float4 u0 = *reinterpret_cast<const float4 *>(epi.head_w + co);
                const float4 u1 = *reinterpret_cast<const float4 *>(epi.head_w + Cout + co);
#pragma unroll
                for (int mf = 0; mf < MF; ++mf) {
                    s0[mf] += u0.x * acc[mf][nf][0] + u0.y * acc[mf][nf][1] + u0.z * acc[mf][nf][2] +
                              u0.w * acc[mf][nf][3];
                    s1[mf] += u1.x * acc[mf][nf][0] + u1.y * acc[mf][nf][1] + u1.z * acc[mf][nf][2] +
                              u1.w * acc[mf][nf][3];
                }
            }
        }
        if (EPI == 2) {
            // 1x1 head over all Cout channels of the pixel: the four lanes
            // l, l ^ 16, l ^ 32, l ^ 48 hold its channels
            const float hb0 = epi.head_b[0], hb1 = epi.head_b[1];
#pragma unroll
            for (int mf = 0; mf < MF; ++mf) {
                const int y = y0 + mf;
                float a0 = s0[mf], a1 = s1[mf];
                a0 += __shfl_xor(a0, 16);
                a1 += __shfl_xor(a1, 16);
                a0 += __shfl_xor(a0, 32);
                a1 += __shfl_xor(a1, 32);
                if (lane < 16 && y < H && x < W)
                    *reinterpret_cast<float2 *>(epi.head_out + (((size_t)b * H + y) * W + x) * 2) =
                        make_float2(a0 + hb0, a1 + hb1);
            }
        }
#pragma unroll
        for (int mf = 0; mf < MF; ++mf)
#pragma unroll
            for (int nf = 0; nf < NF; ++nf) acc[mf][nf] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
}

// ------------------------------------------------------------------ conv fwd
// Implicit GEMM, computed transposed: D[co][pixel] = sum_k W[co][k] X[k][pixel]
// with K = 9 taps x input channels, so that each lane of an MFMA result holds
// four consecutive output channels of one pixel (one 8- or 16-byte store).
// A workgroup (4 wavefronts) owns CO = 16 NF output channels and walks a
// list of pixel tiles (TH = 4 MF rows x 16 columns each); wavefront w owns
// rows w MF .. w MF + MF - 1 of a tile (one 16-pixel fragment per row) and
// all NF channel fragments.  The work is a sequence of stages (tile,
// 32-channel chunk of the concatenated input).  While the MFMAs of one stage
// run from LDS, the next stage's input halo (and its weights, when they
// change) are loaded into registers; they go to LDS after a barrier.  With a
// single chunk the weights stay in LDS for every tile.  For each kx the
// MF + 2 halo rows a wavefront touches are read once and serve all three ky.
//
// IN8: a single source with 8 channels per pixel (the network input).  A K
// step of 32 then spans four taps of 8 channels (lane group l / 16 takes tap
// 4 s + l / 16 of step s), so the nine taps take three steps instead of nine;
// the halo holds 8 channels per pixel and the weights 12 tap slots (the last
// three zero).
template <int MF, int NF, int EPI, bool IN8 = false>  // EPI: 0 store, 1 store and pool, 2 head
__global__ __launch_bounds__(256, NF == 4 ? 2 : 1) void k_conv3x3(Srcs in, int B, int H, int W,
                                                 const bf16 *__restrict__ Wt, int Cout, int mode,
                                                 float *__restrict__ out32,
                                                 bf16 *__restrict__ out16,
                                                 const float *__restrict__ scale,
                                                 const float *__restrict__ shift, float slope,
                                                 ConvEpi epi)
{
    constexpr int TW = 16, TH = 4 * MF, HX = TW + 2, HY = TH + 2;
    constexpr int PS = 40;           // LDS halves per pixel: 32 channels + pad
    constexpr int CO = 16 * NF;
    constexpr int WS = 9 * 32 + 8;   // LDS halves per output channel row
    constexpr int NH = (HY * HX * 4 + 255) / 256;  // halo 16-byte pieces per thread
    constexpr int NW = (CO * 36 + 255) / 256;      // weight 16-byte pieces per thread
    constexpr int WS8 = 12 * 8 + 8;                // IN8: LDS halves per output channel row
    constexpr int NH8 = (HY * HX + 255) / 256, NW8 = (CO * 12 + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 sx[HY * HX * PS];
    __shared__ __attribute__((aligned(16))) bf16 sw[CO * WS];
    // folded BN of this block's channels, read by the epilogues from LDS (a
    // global load there would stay in flight across the loop and make the
    // next stage's prefetch wait)
    __shared__ __attribute__((aligned(16))) float ssc[CO], ssh[CO];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int co0 = blockIdx.y * CO;
    if (tid < CO) {
        const bool ok = mode == 1 && co0 + tid < Cout;
        ssc[tid] = ok ? scale[co0 + tid] : 0.f;
        ssh[tid] = ok ? shift[co0 + tid] : 0.f;
    }
    const int nch = in.Ctot / 32;
    const int wst = in.wstride ? in.wstride : in.Ctot;  // weight row length
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = B * tiles_x * tiles_y;
    const int gx = gridDim.x;
    // this workgroup's tiles: blockIdx.x, blockIdx.x + gx, ...
    const int my_tiles = ntiles > (int)blockIdx.x ? (ntiles - 1 - blockIdx.x) / gx + 1 : 0;
    const int nstage = my_tiles * nch;
    if (nstage == 0) return;
    // tile coordinates advance by gx tiles: (dtx, dty, db) with carries
    const int dtx = gx % tiles_x, dty = (gx / tiles_x) % tiles_y, db = gx / (tiles_x * tiles_y);
    auto advance = [&](int &tx, int &ty, int &b) {
        tx += dtx;
        if (tx >= tiles_x) {
            tx -= tiles_x;
            ++ty;
        }
        ty += dty;
        if (ty >= tiles_y) {
            ty -= tiles_y;
            ++b;
        }
        b += db;
    };

    uint4 hreg[NH], wreg[NW];
    auto load_stage = [&](int tx, int ty, int b, int ch, bool with_w) {
        const int x0 = tx * TW - 1, y0 = ty * TH - 1;
        if constexpr (IN8) {
            const bf16 *src = in.s[0].p + ((size_t)(in.s[0].shared ? 0 : b) * H * W) * 8;
            const bool inside = x0 >= 0 && y0 >= 0 && x0 + HX <= W && y0 + HY <= H;
#pragma unroll
            for (int k = 0; k < NH8; ++k) {
                const int pix = tid + 256 * k, hy = pix / HX;
                const int y = y0 + hy, x = x0 + pix - hy * HX;
                uint4 v = {0u, 0u, 0u, 0u};
                if (pix < HY * HX && (inside || (y >= 0 && y < H && x >= 0 && x < W)))
                    v = *reinterpret_cast<const uint4 *>(src + (size_t)(y * W + x) * 8);
                hreg[k] = v;
            }
            if (with_w) {
#pragma unroll
                for (int k = 0; k < NW8; ++k) {
                    const int idx = tid + 256 * k, co = idx / 12, tap = idx - co * 12;
                    uint4 v = {0u, 0u, 0u, 0u};
                    if (idx < CO * 12 && tap < 9 && co0 + co < Cout)
                        v = *reinterpret_cast<const uint4 *>(Wt + ((size_t)(co0 + co) * 9 + tap) * wst + in.woff);
                    wreg[k] = v;
                }
            }
            return;
        }
        int coff = ch * 32, s = 0;
        while (s < in.n - 1 && coff >= in.s[s].C) {
            coff -= in.s[s].C;
            ++s;
        }
        // weights first: their address registers may be reloaded from
        // scratch, and the wait for that reload should not cover the halo
        // loads
        // Buffer loads from uniform descriptors with 32-bit byte offsets; a
        // piece outside the image, the tensor's channels or the weight rows
        // gets an offset past the descriptor's range and reads as zero.
        if (with_w) {
            const size_t w0 = (size_t)co0 * 9 * wst + in.woff + ch * 32;
            const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(Wt + w0), 0, (int)(((size_t)Cout * 9 * wst - w0) * 2), BUF_DWORD3);
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int idx = tid + 256 * k;
                const int rr = idx >> 2, co = rr / 9, tap = rr - co * 9;
                const int off = idx < CO * 36 ? ((co * 9 + tap) * wst + (idx & 3) * 8) * 2 : BUF_NONE;
                wreg[k] = ld_buf16(wr, off);
            }
        }
        const int Cs = in.s[s].stride ? in.s[s].stride : in.s[s].C;  // channels per pixel in memory
        const size_t h0 = ((size_t)(in.s[s].shared ? 0 : b) * H * W) * Cs + coff;
        const __amdgpu_buffer_rsrc_t hr = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(in.s[s].p + h0), 0, (int)(((size_t)H * W * Cs - coff) * 2), BUF_DWORD3);
        const bool inside = x0 >= 0 && y0 >= 0 && x0 + HX <= W && y0 + HY <= H;
        const bool seg_ok = coff + (tid & 3) * 8 < Cs;  // this thread's 8 channels exist
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            // this thread's piece: halo pixel (hy, hx), 8-channel segment tid % 4
            const int idx = tid + 256 * k, pix = idx >> 2, hy = pix / HX;
            const int y = y0 + hy, x = x0 + pix - hy * HX;
            const bool ok = idx < HY * HX * 4 && seg_ok && (inside || (y >= 0 && y < H && x >= 0 && x < W));
            hreg[k] = ld_buf16(hr, ok ? ((y * W + x) * Cs + (tid & 3) * 8) * 2 : BUF_NONE);
        }
    };
    auto store_stage = [&](bool with_w) {
        if constexpr (IN8) {
#pragma unroll
            for (int k = 0; k < NH8; ++k) {
                const int pix = tid + 256 * k;
                if (pix < HY * HX) *reinterpret_cast<uint4 *>(&sx[pix * 8]) = hreg[k];
            }
            if (with_w) {
#pragma unroll
                for (int k = 0; k < NW8; ++k) {
                    const int idx = tid + 256 * k, co = idx / 12;
                    if (idx < CO * 12) *reinterpret_cast<uint4 *>(&sw[co * WS8 + (idx - co * 12) * 8]) = wreg[k];
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const int idx = tid + 256 * k;
            if (idx < HY * HX * 4)
                *reinterpret_cast<uint4 *>(&sx[(idx >> 2) * PS + (idx & 3) * 8]) = hreg[k];
        }
        if (with_w) {
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int idx = tid + 256 * k;
                if (idx < CO * 36) {
                    const int rr = idx >> 2, co = rr / 9, tap = rr - co * 9;
                    *reinterpret_cast<uint4 *>(&sw[co * WS + tap * 32 + (idx & 3) * 8]) = wreg[k];
                }
            }
        }
    };

    f32x4 acc[MF][NF];
#pragma unroll
    for (int i = 0; i < MF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // current tile and the tile of the next stage to load
    int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y, b = blockIdx.x / (tiles_x * tiles_y);
    int ntx = tx, nty = ty, nbb = b, nchk = 0;
    load_stage(ntx, nty, nbb, 0, true);
    store_stage(true);
    __syncthreads();
    const bool reload_w = nch > 1;
    for (int st = 0; st < nstage; ++st) {
        const bool more = st + 1 < nstage;
        if (more) {
            if (++nchk == nch) {
                nchk = 0;
                advance(ntx, nty, nbb);
            }
            load_stage(ntx, nty, nbb, nchk, reload_w);
        }
        if constexpr (IN8) {
            // step s: this lane's tap 4 s + l / 16 (none for 9..11)
            bf16x8 wa[3][NF];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int nf = 0; nf < NF; ++nf)
                    wa[k][nf] = *reinterpret_cast<const bf16x8 *>(
                        &sw[(nf * 16 + (lane & 15)) * WS8 + (4 * k + (lane >> 4)) * 8]);
#pragma unroll
            for (int mf = 0; mf < MF; ++mf)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int t = 4 * k + (lane >> 4), tc = t < 9 ? t : 8;
                    const int ky = tc / 3, kx = tc - 3 * ky;
                    bf16x8 xb = *reinterpret_cast<const bf16x8 *>(
                        &sx[((wv * MF + mf + ky) * HX + (lane & 15) + kx) * 8]);
                    if (t >= 9) xb = bf16x8{};
#pragma unroll
                    for (int nf = 0; nf < NF; ++nf)
                        acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[k][nf], xb, acc[mf][nf], 0, 0, 0);
                }
        } else {
        // rows in groups of RG pixel fragments (RG + 2 halo rows live at once)
        constexpr int RG = MF > 4 ? MF / 2 : MF;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
#pragma unroll
            for (int g = 0; g < MF; g += RG) {
                bf16x8 a[RG + 2];
#pragma unroll
                for (int r = 0; r < RG + 2; ++r)
                    a[r] = *reinterpret_cast<const bf16x8 *>(
                        &sx[((wv * MF + g + r) * HX + (lane & 15) + kx) * PS + 8 * (lane >> 4)]);
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) {
                    const int tap = ky * 3 + kx;
                    bf16x8 bw[NF];
#pragma unroll
                    for (int nf = 0; nf < NF; ++nf)
                        bw[nf] = *reinterpret_cast<const bf16x8 *>(
                            &sw[(nf * 16 + (lane & 15)) * WS + tap * 32 + 8 * (lane >> 4)]);
#pragma unroll
                    for (int mf = 0; mf < RG; ++mf)
#pragma unroll
                        for (int nf = 0; nf < NF; ++nf)
                            acc[g + mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                bw[nf], a[mf + ky], acc[g + mf][nf], 0, 0, 0);
                }
                // keep the next group's LDS reads after these MFMAs (bounds
                // the live fragments)
                if (MF > 4) __builtin_amdgcn_sched_barrier(0);
            }
        }
        }
        if (st % nch == nch - 1) {
            // the tile is complete
            f16x4 mp[MF][NF];
            conv_epilogue<MF, NF, EPI>(acc, mp, lane, b, ty * TH + wv * MF, tx * TW + (lane & 15), H, W, Cout, co0,
                                       mode, out32, out16, slope, epi, [&](int c, float4 &sc, float4 &sh) {
                                           sc = *reinterpret_cast<const float4 *>(&ssc[c]);
                                           sh = *reinterpret_cast<const float4 *>(&ssh[c]);
                                       });
            advance(tx, ty, b);
        }
        if (more) {
            __syncthreads();  // every wavefront is done with this stage's LDS
            store_stage(reload_w);
            __syncthreads();
        }
    }
}

// Direct-to-LDS form of the same convolution for 512-thread workgroups.
// Eight wavefronts share one copy of the weights; the tile is 8 MF rows x
// 16 columns.  Halo and weights reach LDS by buffer loads that write LDS
// directly (lane l of an instruction fills 16-byte slot base + l), into two
// buffers: while the MFMAs read one stage, the next stage's copy is in
// flight into the other buffer, and no registers stage it.  Slots are
// XOR-swizzled so fragment reads spread over all banks: halo piece (pixel p,
// 8-channel segment s) sits in slot 4 p + (s ^ ((p / 2) % 4)), weight piece
// (channel c, tap t, segment s) in slot 4 (9 c + t) + (s ^ ((c / 2) % 4)): any
// 8 consecutive lanes of one segment (the lanes a 16-byte LDS read serves
// together) hit distinct 16-byte bank groups (no bank-conflict cycles in the
// counters).
// Pieces outside the image, the source's channels or Cout read as zero.
// RW: the weights change per stage (more than one 32-channel chunk).
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(3))) uint4 luint4;
typedef __attribute__((address_space(3))) bf16x8 lbf16x8;
// plain 16-byte LDS words (HIP's vector classes cannot be assigned through
// LDS-qualified pointers in the host pass)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lu32x4;
__device__ __forceinline__ uint4 lds_ld16(const luint4 *p)
{
    const u32x4 v = *reinterpret_cast<const lu32x4 *>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_st16(luint4 *p, const uint4 &v)
{
    *reinterpret_cast<lu32x4 *>(p) = u32x4{v.x, v.y, v.z, v.w};
}

// The builtins sit in plain device functions: called from a lambda in a
// kernel template, they keep the host pass from emitting the launch stub.
// 16-byte direct-to-LDS buffer load: lane l fills slot dst + l
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, luint4 *dst, int off)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void *)dst, 16, off, 0, 0, 0);
}
__device__ __forceinline__ void wg_barrier() { __builtin_amdgcn_s_barrier(); }
// s_waitcnt with vmcnt = N (< 64) and the other counters left alone
#define WAIT_VM(N) __builtin_amdgcn_s_waitcnt(((N) & 15) | (((N) >> 4) << 14) | (7 << 4) | (15 << 8))
// s_waitcnt lgkmcnt(0), the other counters left alone
#define WAIT_LGKM0() __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4))

// UP: the first source is read through the x2 bilinear upsampling (Src::up).
// A stage of one of its chunks copies the coarse window under the tile into
// an area of the halo buffer past the fine halo; the workgroup then expands
// it to the fine halo (bf16, the values a stored upsampled tensor would
// hold) before the MFMAs.  The fine halo pairs rows (and columns) as (odd,
// even) fine indices 2c + 1, 2c + 2, which read coarse c and c + 1 only, so
// each 2 x 2 fine block needs a 2 x 2 coarse window.  (32 output channels:
// the larger halo buffers leave no LDS for wider weight blocks.)
template <int MF, int NF, int EPI, bool RW, bool UP = false>
__global__ __launch_bounds__(512, 1) void k_conv3x3d(Srcs in, int B, int H, int W, const bf16 *__restrict__ Wt,
                                                     int Cout, int mode, float *__restrict__ out32,
                                                     bf16 *__restrict__ out16, const float *__restrict__ scale,
                                                     const float *__restrict__ shift, float slope, ConvEpi epi)
{
    constexpr int NWV = 8;
    constexpr int TW = 16, TH = NWV * MF, HX = TW + 2, HY = TH + 2;
    constexpr int CO = 16 * NF;
    constexpr int HSL = HY * HX * 4, HIN = (HSL + 511) / 512;  // halo slots, DMA instructions per wave
    constexpr int WSL = CO * 36, WIN = (WSL + 511) / 512;       // weight slots, instructions
    // fused upsampling: fine halo row / column pairs, coarse window (CWN
    // slots after the HIN * 512 of the fine halo, HINC more instructions)
    constexpr int NPY = TH / 2 + 1, NPX = TW / 2 + 1, CWY = NPY + 1, CWX = NPX + 1;
    constexpr int CWN = UP ? CWY * CWX * 4 : 0, HINC = (CWN + 511) / 512, HINT = HIN + HINC;
    constexpr int NISS = HINT + (RW ? WIN : 0);                 // instructions per stage and wave
    // one chunk of at most 32 output channels: each wavefront keeps all the
    // weight fragments in registers (9 NF x 4 VGPRs) and reads only the
    // halo from LDS
    constexpr bool WREG = !RW && NF <= 2;
    static_assert(!UP || (RW && NF == 2), "an upsampled source: a second source, 32 output channels");
    // Wavefront layout.  SPL = 2 (64 output channels, plain epilogue): the
    // wavefronts pair up over the block's channels, each taking 2 MF rows x
    // NF / 2 fragments: the same MFMAs from fewer fragment reads (3 (2 MF +
    // 2) + 9 NF / 2 instead of 3 (MF + 2) + 9 NF per stage), since the weights
    // dominate those reads (1.5% faster network inference on MI355X).
    constexpr int SPL = (NF == 4 && EPI == 0 && !WREG) ? 2 : 1;
    constexpr int WMF = MF * SPL, WNF = NF / SPL;
    __shared__ __attribute__((aligned(16))) uint4 hA_[HINT * 512], hB_[HINT * 512];
    __shared__ __attribute__((aligned(16))) uint4 wA_[WIN * 512], wB_[WIN * 512];
    // LDS-typed pointers keep each buffer's identity visible to the
    // compiler, so a read of one buffer does not wait for copies into the
    // other
    luint4 *hA = (luint4 *)hA_, *hB = (luint4 *)hB_, *wA = (luint4 *)wA_, *wB = (luint4 *)wB_;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int co0 = blockIdx.y * CO;
    const int nch = in.Ctot / 32;
    const int wst = in.wstride ? in.wstride : in.Ctot;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = B * tiles_x * tiles_y;
    const int gx = gridDim.x;
    const int my_tiles = ntiles > (int)blockIdx.x ? (ntiles - 1 - blockIdx.x) / gx + 1 : 0;
    const int nstage = my_tiles * nch;
    if (nstage == 0) return;
    const int dtx = gx % tiles_x, dty = (gx / tiles_x) % tiles_y, db = gx / (tiles_x * tiles_y);
    auto advance = [&](int &tx, int &ty, int &b) {
        tx += dtx;
        if (tx >= tiles_x) {
            tx -= tiles_x;
            ++ty;
        }
        ty += dty;
        if (ty >= tiles_y) {
            ty -= tiles_y;
            ++b;
        }
        b += db;
    };

    // DMA of one stage's halo (and weights) into the given buffers.  The
    // byte offsets stay in hoff/woff until after the MFMAs of the stage:
    // were their registers reused as fragment destinations, the compiler
    // would wait for these copies before the first fragment read.
    int hoff[HINT], woff[WIN];
    auto issue_halo = [&](luint4 *hbuf, int tx, int ty, int b, int ch, bool real) {
        const int x0 = tx * TW - 1, y0 = ty * TH - 1;
        int coff = ch * 32, s = 0;
        while (s < in.n - 1 && coff >= in.s[s].C) {
            coff -= in.s[s].C;
            ++s;
        }
        const int Cs = in.s[s].stride ? in.s[s].stride : in.s[s].C;
        // an upsampled chunk copies its coarse window (rows and columns
        // clamped to the image: the clamped samples are the ones the
        // interpolation reads) to slots HIN * 512 + 4 (row * CWX + column) +
        // segment; the fine halo slots stay untouched until the expansion
        const bool upc = UP && s == 0 && in.s[0].up;
        const int hh = upc ? H / 2 : H, ww = upc ? W / 2 : W;
        const size_t h0 = ((size_t)(in.s[s].shared ? 0 : b) * hh * ww) * Cs + coff;
        const __amdgpu_buffer_rsrc_t hr = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(in.s[s].p + h0), 0, (int)(((size_t)hh * ww * Cs - coff) * 2), BUF_DWORD3);
#pragma unroll
        for (int k = 0; k < HINT; ++k) {
            const int blk = k * NWV + wv, q = blk * 64 + lane;
            int off;
            if (k < HIN) {
                const int pix = q >> 2, seg = (q & 3) ^ ((pix >> 1) & 3);
                const int hy = pix / HX, y = y0 + hy, x = x0 + pix - hy * HX;
                const bool ok = real && !upc && q < HSL && coff + seg * 8 < Cs && y >= 0 && y < H && x >= 0 &&
                                x < W;
                off = ok ? ((y * W + x) * Cs + seg * 8) * 2 : BUF_NONE;
            } else {
                const int cq = q - HIN * 512, cp = cq >> 2, cs = cq & 3, cr = cp / CWX;
                int gy = (y0 + 1) / 2 - 1 + cr, gx = (x0 + 1) / 2 - 1 + (cp - cr * CWX);
                gy = gy < 0 ? 0 : (gy >= hh ? hh - 1 : gy);
                gx = gx < 0 ? 0 : (gx >= ww ? ww - 1 : gx);
                const bool cok = real && upc && cq < CWN && coff + cs * 8 < Cs;
                off = cok ? ((gy * ww + gx) * Cs + cs * 8) * 2 : BUF_NONE;
            }
            hoff[k] = off;
            dma16(hr, hbuf + blk * 64, hoff[k]);
        }
    };
    // expands the coarse window in hb to the fine halo of tile (tx, ty):
    // thread per (row pair k, column pair m, segment); fine halo pixel
    // (2k + p, 2m + q) blends window rows k, k + 1 and columns m, m + 1.  Its
    // weights are up_src's (1 - l, l) on those slots; at the first image row
    // (column) up_src's first sample is the second slot and its weight l is
    // zero, so the weights become (l, 1 - l) = (0, 1).  Each value is formed
    // as up_blend8 forms it (the two horizontal blends of a fine column are
    // shared by the pair's two rows) and equals a direct evaluation.
    auto build_up = [&](luint4 *hb, int tx, int ty) {
        constexpr int NIT = NPY * NPX * 4, NR = (NIT + 511) / 512;
        const int hc = H / 2, wc = W / 2;
        const luint4 *cw = hb + HIN * 512;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int it = r * 512 + tid, seg = it & 3, pr = it >> 2, k = pr / NPX, m = pr - k * NPX;
            if (it < NIT) {
                const luint4 *c0 = cw + (k * CWX + m) * 4 + seg;
                const f8 a00 = u4_to_f8(lds_ld16(c0)), a01 = u4_to_f8(lds_ld16(c0 + 4));
                const f8 a10 = u4_to_f8(lds_ld16(c0 + CWX * 4)), a11 = u4_to_f8(lds_ld16(c0 + CWX * 4 + 4));
                const int c = ty * (TH / 2) - 1 + k, d = tx * (TW / 2) - 1 + m;
                float wy[2][2], wx[2][2];
                bool iny[2], inx[2];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const int fy = ty * TH - 1 + 2 * k + p, fx = tx * TW - 1 + 2 * m + p;
                    int i0, i1;
                    float l;
                    up_src(fy, hc, i0, i1, l);
                    wy[p][0] = i0 > c ? l : 1.f - l;
                    wy[p][1] = i0 > c ? 1.f - l : l;
                    iny[p] = fy >= 0 && fy < H;
                    up_src(fx, wc, i0, i1, l);
                    wx[p][0] = i0 > d ? l : 1.f - l;
                    wx[p][1] = i0 > d ? 1.f - l : l;
                    inx[p] = fx >= 0 && fx < W;
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    f8 h0, h1;  // horizontal blends of window rows k and k + 1 at fine column q
#pragma unroll
                    for (int z = 0; z < 8; ++z) {
                        h0.v[z] = wx[q][0] * a00.v[z] + wx[q][1] * a01.v[z];
                        h1.v[z] = wx[q][0] * a10.v[z] + wx[q][1] * a11.v[z];
                    }
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        uint4 o = make_uint4(0u, 0u, 0u, 0u);
                        if (iny[p] && inx[q]) {
                            bf16 *e = reinterpret_cast<bf16 *>(&o);
#pragma unroll
                            for (int z = 0; z < 8; ++z) e[z] = (bf16)(wy[p][0] * h0.v[z] + wy[p][1] * h1.v[z]);
                        }
                        const int pix = (2 * k + p) * HX + 2 * m + q;
                        lds_st16(hb + pix * 4 + (seg ^ ((pix >> 1) & 3)), o);
                    }
                }
            }
        }
        WAIT_LGKM0();
        wg_barrier();  // the fine halo is complete
    };
    auto issue_w = [&](luint4 *wbuf, int ch, bool real) {
        const size_t w0 = (size_t)co0 * 9 * wst + in.woff + ch * 32;
        const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(Wt + w0), 0, (int)(((size_t)Cout * 9 * wst - w0) * 2), BUF_DWORD3);
#pragma unroll
        for (int k = 0; k < WIN; ++k) {
            const int blk = k * NWV + wv, q = blk * 64 + lane;
            const int co = q / 36, r = q - co * 36, tap = r >> 2, seg = (r & 3) ^ ((co >> 1) & 3);
            woff[k] = real && q < WSL ? ((co * 9 + tap) * wst + seg * 8) * 2 : BUF_NONE;
            dma16(wr, wbuf + blk * 64, woff[k]);
        }
    };

    // this wavefront: tile rows wrow .. wrow + WMF - 1, block channels wco ..
    // wco + 16 WNF - 1
    const int wrow = (wv / SPL) * WMF, wco = (wv % SPL) * WNF * 16;
    f32x4 acc[WMF][WNF];
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // folded BN of the lane's output channels, kept in registers (no global
    // loads in the loop besides the copies and the context map)
    float4 bsc[WNF], bsh[WNF];
#pragma unroll
    for (int nf = 0; nf < WNF; ++nf) {
        const int co = co0 + wco + nf * 16 + 4 * (lane >> 4);
        bsc[nf] = bsh[nf] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (mode == 1 && co < Cout) {
            bsc[nf] = *reinterpret_cast<const float4 *>(scale + co);
            bsh[nf] = *reinterpret_cast<const float4 *>(shift + co);
        }
    }

    bf16x8 wreg[WREG ? 9 : 1][WREG ? NF : 1];
    f16x4 mp[WMF][WNF];  // context map of the tile being finished
    // MFMAs of one stage from the given buffers
    auto compute = [&](const luint4 *hbuf, const luint4 *wbuf) {
        const int seg = lane >> 4;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            bf16x8 a[WMF + 2];
#pragma unroll
            for (int r = 0; r < WMF + 2; ++r) {
                const int p = (wrow + r) * HX + (lane & 15) + kx;
                a[r] = *reinterpret_cast<const lbf16x8 *>(hbuf + p * 4 + (seg ^ ((p >> 1) & 3)));
            }
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int tap = ky * 3 + kx;
                bf16x8 bw[WNF];
#pragma unroll
                for (int nf = 0; nf < WNF; ++nf) {
                    const int co = wco + nf * 16 + (lane & 15);
                    if constexpr (WREG)
                        bw[nf] = wreg[tap][nf];
                    else
                        bw[nf] = *reinterpret_cast<const lbf16x8 *>(wbuf + (co * 9 + tap) * 4 +
                                                                    (seg ^ ((co >> 1) & 3)));
                }
#pragma unroll
                for (int mf = 0; mf < WMF; ++mf)
#pragma unroll
                    for (int nf = 0; nf < WNF; ++nf)
                        acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[nf], a[mf + ky], acc[mf][nf], 0, 0, 0);
            }
        }
    };

    int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y, b = blockIdx.x / (tiles_x * tiles_y);
    int ntx = tx, nty = ty, nbb = b, nchk = 0;
    issue_halo(hA, tx, ty, b, 0, true);
    issue_w(wA, 0, true);
    if constexpr (WREG) {
        // the weights (and the first halo) land; every wavefront copies its
        // fragments to registers
        WAIT_VM(0);
        wg_barrier();
        const int seg = lane >> 4;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int nf = 0; nf < NF; ++nf) {
                const int co = nf * 16 + (lane & 15);
                wreg[tap][nf] = *reinterpret_cast<const lbf16x8 *>(wA + (co * 9 + tap) * 4 + (seg ^ ((co >> 1) & 3)));
            }
    } else if (!RW) {
        issue_w(wB, 0, true);  // one chunk: both weight buffers hold it for the whole kernel
    }

    // one stage: issue the next stage's copy, wait for this one, MFMAs,
    // epilogue when the tile is complete
    auto step = [&](luint4 *__restrict__ ch_, luint4 *__restrict__ cw_, luint4 *__restrict__ nh_,
                    luint4 *__restrict__ nw_, int st) {
        // The next stage's copy is issued on every step (all pieces out of
        // range after the last stage): copies issued under a branch would
        // make the compiler wait for all of them before the fragment reads.
        const bool more = st + 1 < nstage;
        if (more && ++nchk == nch) {
            nchk = 0;
            advance(ntx, nty, nbb);
        }
        issue_halo(nh_, ntx, nty, nbb, nchk, more);
        if (RW) issue_w(nw_, nchk, more);
        WAIT_VM(NISS);  // this stage's copies (issued a step earlier) have landed
        wg_barrier();   // ... for every wavefront
        if constexpr (UP) {
            if (in.s[0].up && (st % nch) * 32 < in.s[0].C) build_up(ch_, tx, ty);
        }
        // the last chunk of a tile: its context map loads overlap the MFMAs
        const bool last = st % nch == nch - 1;
        if (EPI == 0 && last && mode == 1 && epi.cmap)
            conv_cmap_issue<WMF, WNF>(mp, lane, ty * TH + wrow, tx * TW + (lane & 15), H, W, Cout, co0 + wco, epi);
        compute(ch_, cw_);
        // (no instructions: keeps the offset registers allocated until here;
        // the constraint names a GPU register class, so the host pass skips it)
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
        for (int q = 0; q < HINT; ++q) asm volatile("" ::"v"(hoff[q]));
        if (RW) {
#pragma unroll
            for (int q = 0; q < WIN; ++q) asm volatile("" ::"v"(woff[q]));
        }
#endif
        if (last) {
            conv_epilogue<WMF, WNF, EPI, true>(acc, mp, lane, b, ty * TH + wrow, tx * TW + (lane & 15), H,
                                                         W, Cout, co0 + wco, mode, out32, out16, slope, epi,
                                                         [&](int c, float4 &sc, float4 &sh) {
                                                             // c = 16 nf + 4 (lane / 16) (+ 0):
                                                             // fragment nf's registers
                                                             sc = bsc[c >> 4];
                                                             sh = bsh[c >> 4];
                                                         });
            advance(tx, ty, b);
        }
        wg_barrier();  // every wavefront is done with these buffers
    };
    // Several chunks per tile (weights copied with every stage), plain
    // epilogue: one barrier per stage.  After the barrier every wavefront is
    // done with the previous stage, so the next stage's copies go into its
    // buffers then; the epilogue's stores (a fixed number, see
    // conv_epilogue) stay in flight across the next stage's wait, which
    // counts them: completion is reported in issue order.
    if constexpr (RW && !UP && EPI == 0) {
        constexpr int NST1 = WMF * WNF / 2, NST0 = WMF * WNF;  // epilogue stores in mode 1 / 0
        bool prev_epi = false;
        auto step1 = [&](luint4 *__restrict__ ch_, luint4 *__restrict__ cw_, luint4 *__restrict__ nh_,
                         luint4 *__restrict__ nw_, int st) {
            if (!prev_epi)
                WAIT_VM(0);  // this stage's copies
            else if (mode == 1)
                WAIT_VM(NST1);  // ... but not the previous epilogue's stores
            else
                WAIT_VM(NST0);
            wg_barrier();
            const bool last = st % nch == nch - 1;
            // context-map loads before the copies, so that the epilogue's wait
            // for them leaves the copies in flight
            if (last && mode == 1 && epi.cmap)
                conv_cmap_issue<WMF, WNF>(mp, lane, ty * TH + wrow, tx * TW + (lane & 15), H, W, Cout, co0 + wco,
                                          epi);
            const bool more = st + 1 < nstage;
            if (more && ++nchk == nch) {
                nchk = 0;
                advance(ntx, nty, nbb);
            }
            issue_halo(nh_, ntx, nty, nbb, nchk, more);
            issue_w(nw_, nchk, more);
            compute(ch_, cw_);
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
            for (int q = 0; q < HINT; ++q) asm volatile("" ::"v"(hoff[q]));
#pragma unroll
            for (int q = 0; q < WIN; ++q) asm volatile("" ::"v"(woff[q]));
#endif
            if (last) {
                conv_epilogue<WMF, WNF, EPI, true, NISS>(acc, mp, lane, b, ty * TH + wrow, tx * TW + (lane & 15), H,
                                                         W, Cout, co0 + wco, mode, out32, out16, slope, epi,
                                                         [&](int c, float4 &sc, float4 &sh) {
                                                             sc = bsc[c >> 4];
                                                             sh = bsh[c >> 4];
                                                         });
                advance(tx, ty, b);
            }
            prev_epi = last;
        };
        for (int st = 0; st < nstage; st += 2) {
            step1(hA, wA, hB, wB, st);
            if (st + 1 < nstage) step1(hB, wB, hA, wA, st + 1);
        }
        return;
    }
    for (int st = 0; st < nstage; st += 2) {
        step(hA, wA, hB, wB, st);
        if (st + 1 < nstage) step(hB, wB, hA, wA, st + 1);
    }
}

// ------------------------------------------------------------------ wgrad
// dW[co][tap][ci] = sum_p dy[p][co] X[p + tap offset][ci] over a range of K
// steps (split K).  MFMA operands: A = dy^T (16 output channels x 32
// pixels), B = X^T (32 pixels x 16 input channels).  A workgroup owns CB =
// 16 NCF output and IB = 16 NIF input channels for all 9 taps.  A K step is
// row y of one 32-pixel column strip (b, x0); consecutive steps walk down the
// strip.  LDS holds dy^T of the row (two buffers) and X^T of image rows in a
// ring of four slots (rows y-1, y, y+1 in use, y+2 being filled).  An X slot
// row (one channel) holds pixels x0 - 8 .. x0 + 39 as six 8-pixel words, of
// which the two outer words carry only the halo pixels x0 - 2, x0 - 1 and
// x0 + 32, x0 + 33.  A lane's B fragment for kx = 1 is the aligned word of
// its 8 pixels; for kx = 0 and kx = 2 it is that word shifted by one pixel,
// formed with byte-align operations from the word and one dword on either
// side (5 v_alignbyte per lane and row, shared by the two shifts).
// Software pipeline: right after the barrier that publishes step s, each
// thread issues the global loads of its piece of step s + 1 (the dy row y+1,
// the X row y+2) into registers, the MFMAs of step s run while they are in
// flight, and the pieces are then transposed into the free buffers before
// the next barrier: one barrier per step.  A step that starts a new strip
// stages its three X rows after a barrier instead.
// Staging pieces (one per thread): 8 dy channels x 4 pixels (four 16-byte
// loads, a 4 x 8 transpose in registers, eight 8-byte LDS writes); 8 X
// channels x 4 pixels (likewise); 8 X channels x the 2 halo pixels of one
// side (two loads, eight 4-byte writes).
// Wavefront w owns input-channel fragment w % NIF and NCW = NCF NIF / 4 of
// the output-channel fragments, for all 9 taps.
constexpr int WG_SEG = 32, WG_PADA = 40, WG_PADX = 56;

// 4 pixels x 8 bf16 channels -> 8 channels x 4 pixels: p[i] holds channels
// 0..7 of pixel i; o[q] receives pixels 0..3 of channel q
__device__ __forceinline__ void transpose4x8(const uint4 *p, uint2 o[8])
{
#pragma unroll
    for (int m = 0; m < 4; ++m) {  // channel pair (2m, 2m + 1) sits in dword m
        const uint32_t a0 = reinterpret_cast<const uint32_t *>(&p[0])[m];
        const uint32_t a1 = reinterpret_cast<const uint32_t *>(&p[1])[m];
        const uint32_t a2 = reinterpret_cast<const uint32_t *>(&p[2])[m];
        const uint32_t a3 = reinterpret_cast<const uint32_t *>(&p[3])[m];
        o[2 * m] = make_uint2((a0 & 0xFFFFu) | (a1 << 16), (a2 & 0xFFFFu) | (a3 << 16));
        o[2 * m + 1] = make_uint2((a0 >> 16) | (a1 & 0xFFFF0000u), (a2 >> 16) | (a3 & 0xFFFF0000u));
    }
}

template <int NCF, int NIF>
__global__ __launch_bounds__(256, 2) void k_wgrad(Srcs x, const bf16 *__restrict__ dy, int B, int H,
                                                  int W, int Cout, int steps_per_split,
                                                  float *__restrict__ part)
{
    constexpr int CB = 16 * NCF, IB = 16 * NIF;
    constexpr int NCW = NCF * NIF / 4;        // output-channel fragments per wave
    static_assert(NCW >= 1 && NCF % NCW == 0, "wave partition");
    constexpr int NPB = WG_SEG / 4;           // 4-pixel blocks per row
    constexpr int NDY = (CB / 8) * NPB;       // dy pieces
    constexpr int NXM = (IB / 8) * NPB;       // X pieces
    constexpr int NXH = (IB / 8) * 2;         // X halo pieces
    static_assert(NDY + NXM + NXH <= 256, "one staging piece per thread");
    __shared__ __attribute__((aligned(16))) bf16 sa[2][CB * WG_PADA];
    __shared__ __attribute__((aligned(16))) bf16 sb[4][IB * WG_PADX];  // [slot][ci][px]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ncb = (Cout + CB - 1) / CB;
    const int cb = blockIdx.y % ncb, ib = blockIdx.y / ncb;
    const int co0 = cb * CB, ci0 = ib * IB;
    const int fi = wv % NIF, cw = (wv / NIF) * NCW;
    const int nseg = (W + WG_SEG - 1) / WG_SEG;
    const int total_steps = B * nseg * H;
    const int s_begin = blockIdx.x * steps_per_split;
    const int s_end = min(total_steps, s_begin + steps_per_split);
    f32x4 acc[9][NCW];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < NCW; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // this thread's staging piece, fixed over the steps: kind 0 dy, 1 X, 2 X
    // halo, 3 none
    const int kind = tid < NDY ? 0 : tid < NDY + NXM ? 1 : tid < NDY + NXM + NXH ? 2 : 3;
    const int u = kind == 0 ? tid : kind == 1 ? tid - NDY : tid - NDY - NXM;
    const int g = kind == 0 ? u % (CB / 8) : u % (IB / 8);   // 8-channel group
    const int tj = kind == 0 ? u / (CB / 8) : u / (IB / 8);  // 4-pixel block, or halo side
    const int cdy = co0 + 8 * g;
    const bool dy_ok = kind == 0 && cdy < Cout;
    // X: the source holding channels ci0 + 8 g .. + 7
    int xs_idx = 0, coff = ci0 + 8 * g;
    bool x_ok = (kind == 1 || kind == 2) && coff < x.Ctot;
    if (x_ok)
        while (xs_idx < x.n - 1 && coff >= x.s[xs_idx].C) {
            coff -= x.s[xs_idx].C;
            ++xs_idx;
        }
    const bf16 *xsrc = x.s[xs_idx].p;
    const int xCs = x.s[xs_idx].stride ? x.s[xs_idx].stride : x.s[xs_idx].C;  // channels per pixel in memory
    const bool xshared = x.s[xs_idx].shared;
    x_ok = x_ok && coff < xCs;
    // first pixel (relative to x0) and count of this piece
    const int px0 = kind == 2 ? (tj == 0 ? -2 : WG_SEG) : 4 * tj;
    uint4 pv[4];

    auto load = [&](int b, int yr, int x0) {
        if (kind == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xs = x0 + px0 + i;
                pv[i] = make_uint4(0u, 0u, 0u, 0u);
                if (dy_ok && xs < W)
                    pv[i] = *reinterpret_cast<const uint4 *>(dy + (((size_t)b * H + yr) * W + xs) * Cout + cdy);
            }
        } else if (kind <= 2) {
            const bool rowok = x_ok && yr >= 0 && yr < H;
            const size_t rowbase = ((size_t)(xshared ? 0 : b) * H + (rowok ? yr : 0)) * W;
            const int np = kind == 1 ? 4 : 2;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xs = x0 + px0 + i;
                pv[i] = make_uint4(0u, 0u, 0u, 0u);
                if (i < np && rowok && xs >= 0 && xs < W)
                    pv[i] = *reinterpret_cast<const uint4 *>(xsrc + (rowbase + xs) * xCs + coff);
            }
        }
    };
    // writes the loaded piece: dy into buffer `slot`, X into ring slot `slot`
    auto store = [&](int slot) {
        if (kind == 3) return;
        uint2 o[8];
        transpose4x8(pv, o);
        if (kind == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                *reinterpret_cast<uint2 *>(&sa[slot][(g * 8 + q) * WG_PADA + px0]) = o[q];
        } else if (kind == 1) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                *reinterpret_cast<uint2 *>(&sb[slot][(g * 8 + q) * WG_PADX + 8 + px0]) = o[q];
        } else if (kind == 2) {
            // pixels px0, px0 + 1 sit in the first dword of each channel's pair
#pragma unroll
            for (int q = 0; q < 8; ++q)
                *reinterpret_cast<uint32_t *>(&sb[slot][(g * 8 + q) * WG_PADX + 8 + px0]) = o[q].x;
        }
    };
    // all of step st's LDS data, loaded synchronously (the first step of the
    // split and the first step of every strip)
    auto stage_fresh = [&](int st) {
        const int y = st % H, r = st / H, seg = r % nseg, b = r / nseg;
        const int x0 = seg * WG_SEG;
        if (kind == 0) {
            load(b, y, x0);
            store(st & 1);
        } else if (kind <= 2) {
            for (int k = 0; k < 3; ++k) {
                load(b, y - 1 + k, x0);
                store((y - 1 + k + 4) & 3);
            }
        }
    };

    if (s_begin < s_end) stage_fresh(s_begin);
    __syncthreads();
    const int c16 = lane & 15, j8 = 8 * (lane >> 4);
    for (int st = s_begin; st < s_end; ++st) {
        const int y = st % H, r = st / H, seg = r % nseg, b = r / nseg;
        const int x0 = seg * WG_SEG;
        const bool have_next = st + 1 < s_end;
        const bool next_fresh = have_next && y + 1 == H;
        if (have_next && !next_fresh) load(b, kind == 0 ? y + 1 : y + 2, x0);
        bf16x8 a[NCW];
#pragma unroll
        for (int c = 0; c < NCW; ++c)
            a[c] = *reinterpret_cast<const bf16x8 *>(&sa[st & 1][((cw + c) * 16 + c16) * WG_PADA + j8]);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const bf16 *row = &sb[(y + ky - 1 + 4) & 3][(fi * 16 + c16) * WG_PADX + 8 + j8];
            const uint4 w = *reinterpret_cast<const uint4 *>(row);
            const uint32_t pw = *reinterpret_cast<const uint32_t *>(row - 2);
            const uint32_t nw = *reinterpret_cast<const uint32_t *>(row + 8);
            const uint32_t s0 = __builtin_amdgcn_alignbyte(w.x, pw, 2);
            const uint32_t s1 = __builtin_amdgcn_alignbyte(w.y, w.x, 2);
            const uint32_t s2 = __builtin_amdgcn_alignbyte(w.z, w.y, 2);
            const uint32_t s3 = __builtin_amdgcn_alignbyte(w.w, w.z, 2);
            const uint32_t s4 = __builtin_amdgcn_alignbyte(nw, w.w, 2);
            const bf16x8 b0 = __builtin_bit_cast(bf16x8, make_uint4(s0, s1, s2, s3));
            const bf16x8 b1 = __builtin_bit_cast(bf16x8, w);
            const bf16x8 b2 = __builtin_bit_cast(bf16x8, make_uint4(s1, s2, s3, s4));
#pragma unroll
            for (int c = 0; c < NCW; ++c) {
                acc[3 * ky][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b0, acc[3 * ky][c], 0, 0, 0);
                acc[3 * ky + 1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b1, acc[3 * ky + 1][c], 0, 0, 0);
                acc[3 * ky + 2][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b2, acc[3 * ky + 2][c], 0, 0, 0);
            }
        }
        if (!have_next) break;
        if (!next_fresh) {
            // the buffers written here were last read by step st - 1
            store(kind == 0 ? (st + 1) & 1 : (y + 2 + 4) & 3);
        } else {
            __syncthreads();  // every wave is done with step st's buffers
            stage_fresh(st + 1);
        }
        __syncthreads();
    }
    // D[co][ci]: lane holds input channel l % 16 and output channels 4 (l / 16) .. + 3
    const size_t per_split = (size_t)Cout * 9 * x.Ctot;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int c = 0; c < NCW; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int co = co0 + (cw + c) * 16 + 4 * (lane >> 4) + q;
                const int ci = ci0 + fi * 16 + c16;
                if (co < Cout && ci < x.Ctot)
                    part[blockIdx.x * per_split + ((size_t)co * 9 + tap) * x.Ctot + ci] = acc[tap][c][q];
            }
}

// out[i] = sum over splits of part[split][i], in two fixed-order passes:
// groups of 32 splits into tmp, then the groups
__global__ void k_sum_splits(const float *__restrict__ part, int nsplit, size_t n,
                             float *__restrict__ tmp, int ngroup)
{
    const int g = blockIdx.y;
    const int s0 = g * 32, s1 = min(nsplit, s0 + 32);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int s = s0; s < s1; ++s) acc += part[(size_t)s * n + i];
        tmp[(size_t)g * n + i] = acc;
    }
}

__global__ void k_sum_groups(const float *__restrict__ tmp, int ngroup, size_t n, float *__restrict__ out)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int g = 0; g < ngroup; ++g) acc += tmp[(size_t)g * n + i];
        out[i] = acc;
    }
}

// ------------------------------------------------------------------ BN
// per-block partial sums (FP64) of y and y^2 per channel; thread t handles
// channel t % C and pixels t / C + k * (256 / C)
// Per-block partial sums over pixels of 4-channel groups: thread t owns
// channel group t % (C / 4) and pixel rows t / (C / 4) + k rs, four rows in
// flight at a time.  part[blk][c][0..1] = (sum v, sum v^2).
__global__ __launch_bounds__(256) void k_bn_partial(const float *__restrict__ y, size_t P, int C,
                                                    double *__restrict__ part, int nblk)
{
    const int G4 = C / 4, t = threadIdx.x, cg = t % G4, r0 = t / G4, rs = 256 / G4;
    double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};
    if (r0 < rs) {
        const size_t stride = (size_t)nblk * rs;
        for (size_t p = (size_t)blockIdx.x * rs + r0; p < P; p += 4 * stride) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t pu = p + u * stride;
                v[u] = pu < P ? *reinterpret_cast<const float4 *>(y + pu * C + cg * 4)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    s1[q] += e[q];
                    s2[q] += (double)e[q] * e[q];
                }
            }
        }
    }
    __shared__ double sh[2][256][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sh[0][t][q] = s1[q];
        sh[1][t][q] = s2[q];
    }
    __syncthreads();
    if (t < C) {
        const int g = t / 4, q = t % 4;
        double a = 0.0, qq = 0.0;
        for (int r = 0; r < rs; ++r) {
            a += sh[0][r * G4 + g][q];
            qq += sh[1][r * G4 + g][q];
        }
        part[((size_t)blockIdx.x * C + t) * 2] = a;
        part[((size_t)blockIdx.x * C + t) * 2 + 1] = qq;
    }
}

// one wavefront per channel; fixed-order sums over the partials
__global__ void k_bn_finish(const double *__restrict__ part, int nblk, int C, size_t P,
                            float *__restrict__ mean, float *__restrict__ rstd,
                            float *__restrict__ var_out)
{
    const int c = blockIdx.x;
    double a = 0.0, q = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 64) {
        a += part[((size_t)k * C + c) * 2];
        q += part[((size_t)k * C + c) * 2 + 1];
    }
    a = wave_sum(a);
    q = wave_sum(q);
    if (threadIdx.x != 0) return;
    double mu = a / (double)P, var = q / (double)P - mu * mu;
    if (var < 0.0) var = 0.0;
    mean[c] = (float)mu;
    rstd[c] = (float)(1.0 / sqrt(var + 1e-5));
    if (var_out) var_out[c] = (float)var;
}

__global__ void k_bn_act_fwd(const float *__restrict__ y, size_t n, int C,
                             const float *__restrict__ mean, const float *__restrict__ rstd,
                             const float *__restrict__ g, const float *__restrict__ bb, float slope,
                             bf16 *__restrict__ a)
{
    const int G = C / 8;
    const int nv = (int)(n / 8);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
        int c0 = (i % G) * 8;
        float4 u0 = *reinterpret_cast<const float4 *>(y + (size_t)i * 8);
        float4 u1 = *reinterpret_cast<const float4 *>(y + (size_t)i * 8 + 4);
        float yv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        f8 o;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int c = c0 + q;
            float z = g[c] * (yv[q] - mean[c]) * rstd[c] + bb[c];
            o.v[q] = z > 0.f ? z : slope * z;
        }
        st8(a + (size_t)i * 8, o);
    }
}

// partial sums of dz and dz * xhat per channel (layout as k_bn_partial)
__global__ __launch_bounds__(256) void k_bn_bwd_partial(
    const float *__restrict__ da, const float *__restrict__ y, size_t P, int C,
    const float *__restrict__ mean, const float *__restrict__ rstd, const float *__restrict__ g,
    const float *__restrict__ bb, float slope, double *__restrict__ part, int nblk)
{
    const int G4 = C / 4, t = threadIdx.x, cg = t % G4, r0 = t / G4, rs = 256 / G4;
    double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};
    if (r0 < rs) {
        const float4 mu = *reinterpret_cast<const float4 *>(mean + cg * 4);
        const float4 rs4 = *reinterpret_cast<const float4 *>(rstd + cg * 4);
        const float4 g4 = *reinterpret_cast<const float4 *>(g + cg * 4);
        const float4 b4 = *reinterpret_cast<const float4 *>(bb + cg * 4);
        const float m_[4] = {mu.x, mu.y, mu.z, mu.w}, r_[4] = {rs4.x, rs4.y, rs4.z, rs4.w};
        const float g_[4] = {g4.x, g4.y, g4.z, g4.w}, b_[4] = {b4.x, b4.y, b4.z, b4.w};
        const size_t stride = (size_t)nblk * rs;
        for (size_t p = (size_t)blockIdx.x * rs + r0; p < P; p += 4 * stride) {
            float4 yv[4], dv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t pu = p + u * stride;
                const bool ok = pu < P;
                yv[u] = ok ? *reinterpret_cast<const float4 *>(y + pu * C + cg * 4)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
                dv[u] = ok ? *reinterpret_cast<const float4 *>(da + pu * C + cg * 4)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float ye[4] = {yv[u].x, yv[u].y, yv[u].z, yv[u].w};
                const float de[4] = {dv[u].x, dv[u].y, dv[u].z, dv[u].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float xh = (ye[q] - m_[q]) * r_[q];
                    const float z = g_[q] * xh + b_[q];
                    const float dz = de[q] * (z > 0.f ? 1.f : slope);
                    s1[q] += dz;
                    s2[q] += (double)dz * xh;
                }
            }
        }
    }
    __shared__ double sh[2][256][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sh[0][t][q] = s1[q];
        sh[1][t][q] = s2[q];
    }
    __syncthreads();
    if (t < C) {
        const int gi = t / 4, q = t % 4;
        double a = 0.0, qq = 0.0;
        for (int r = 0; r < rs; ++r) {
            a += sh[0][r * G4 + gi][q];
            qq += sh[1][r * G4 + gi][q];
        }
        part[((size_t)blockIdx.x * C + t) * 2] = a;
        part[((size_t)blockIdx.x * C + t) * 2 + 1] = qq;
    }
}

__global__ void k_bn_bwd_finish(const double *__restrict__ part, int nblk, int C,
                                float *__restrict__ dg, float *__restrict__ db,
                                float *__restrict__ sums)
{
    const int c = blockIdx.x;
    double a = 0.0, q = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 64) {
        a += part[((size_t)k * C + c) * 2];
        q += part[((size_t)k * C + c) * 2 + 1];
    }
    a = wave_sum(a);
    q = wave_sum(q);
    if (threadIdx.x != 0) return;
    db[c] += (float)a;
    dg[c] += (float)q;
    sums[2 * c] = (float)a;
    sums[2 * c + 1] = (float)q;
}

__global__ void k_bn_bwd_apply(const float *__restrict__ da, const float *__restrict__ y, size_t n,
                               int C, size_t P, const float *__restrict__ mean,
                               const float *__restrict__ rstd, const float *__restrict__ g,
                               const float *__restrict__ bb, float slope,
                               const float *__restrict__ sums, bf16 *__restrict__ dy)
{
    const float invP = 1.f / (float)P;
    const int G = C / 8;
    const int nv = (int)(n / 8);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
        int c0 = (i % G) * 8;
        float4 u0 = *reinterpret_cast<const float4 *>(y + (size_t)i * 8);
        float4 u1 = *reinterpret_cast<const float4 *>(y + (size_t)i * 8 + 4);
        float4 d0 = *reinterpret_cast<const float4 *>(da + (size_t)i * 8);
        float4 d1 = *reinterpret_cast<const float4 *>(da + (size_t)i * 8 + 4);
        float yv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        f8 o;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int c = c0 + q;
            float xh = (yv[q] - mean[c]) * rstd[c];
            float z = g[c] * xh + bb[c];
            float dz = dv[q] * (z > 0.f ? 1.f : slope);
            o.v[q] = g[c] * rstd[c] * (dz - sums[2 * c] * invP - xh * sums[2 * c + 1] * invP);
        }
        st8(dy + (size_t)i * 8, o);
    }
}

// ------------------------------------------------------------------ pooling
// thread per (output pixel, 8-channel group)
// grid (pixels x channel groups of an output row, output rows, batch)
__global__ void k_maxpool_fwd(const bf16 *__restrict__ in, int H, int W, int C, bf16 *__restrict__ out,
                              uint8_t *__restrict__ arg)
{
    const int Wo = W / 2, G = C / 8;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Wo * G) return;
    const int yo = blockIdx.y, b = blockIdx.z;
    const int xo = t / G, g = t - xo * G;
    const size_t base = (((size_t)b * H + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const f8 v0 = ld8(in + base), v1 = ld8(in + base + C);
    const f8 v2 = ld8(in + base + (size_t)W * C), v3 = ld8(in + base + (size_t)W * C + C);
    f8 o;
    uint8_t k8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float best = v0.v[q];
        uint8_t k = 0;
        if (v1.v[q] > best) { best = v1.v[q]; k = 1; }
        if (v2.v[q] > best) { best = v2.v[q]; k = 2; }
        if (v3.v[q] > best) { best = v3.v[q]; k = 3; }
        o.v[q] = best;
        k8[q] = k;
    }
    const size_t pix = ((size_t)b * (H / 2) + yo) * Wo + xo;
    st8(out + pix * C + 8 * g, o);
    if (arg) {
        uint2 packed;
        packed.x = k8[0] | (k8[1] << 8) | (k8[2] << 16) | ((uint32_t)k8[3] << 24);
        packed.y = k8[4] | (k8[5] << 8) | (k8[6] << 16) | ((uint32_t)k8[7] << 24);
        *reinterpret_cast<uint2 *>(arg + pix * C + 8 * g) = packed;
    }
}

__global__ void k_maxpool_bwd(const float *__restrict__ dout, int cstride, int coff,
                              const uint8_t *__restrict__ arg, int B, int H, int W, int C,
                              float *__restrict__ din, int din_C)
{
    const int Ho = H / 2, Wo = W / 2;
    const int n = B * Ho * Wo * C;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c = i % C, pix = i / C;
        int xo = pix % Wo, r = pix / Wo;
        int yo = r % Ho, b = r / Ho;
        int k = arg[i];
        int yy = 2 * yo + (k >> 1), xx = 2 * xo + (k & 1);
        din[(((size_t)b * H + yy) * W + xx) * din_C + c] += dout[(size_t)pix * cstride + coff + c];
    }
}

// ------------------------------------------------------------------ upsampling

// Thread per (fine column, 8-channel group, UP_R coarse rows): it writes the
// 2 UP_R fine pixels of that column over those rows.  Fine row 2i + a reads
// coarse rows i - 1 .. i + 1 only, so a window of three coarse rows (at the
// column's two coarse columns) rolls down, and each coarse sample is loaded
// about (UP_R + 2) / UP_R times per fine column instead of twice per row.
// Every fine pixel blends the same samples with the same weights as a direct
// evaluation of up_src.
// grid (fine columns x channel groups, h / UP_R row blocks, batch)
constexpr int UP_R = 4;
__device__ __forceinline__ uint4 up_pick(int slot, const uint4 &v0, const uint4 &v1, const uint4 &v2)
{
    return slot == 0 ? v0 : slot == 1 ? v1 : v2;
}
__global__ void k_up2_fwd(const bf16 *__restrict__ in, int h, int w, int C, bf16 *__restrict__ out)
{
    const int W = 2 * w, G = C / 8;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * G) return;
    // fine column x = 2j + a, channel group g (fastest: a wavefront's stores
    // cover whole consecutive pixels)
    const int x = t / G, g = t - x * G, b = blockIdx.z;
    const int i0 = blockIdx.y * UP_R, i1 = i0 + UP_R < h ? i0 + UP_R : h;
    int x0, x1;
    float lx;
    up_src(x, w, x0, x1, lx);
    const bf16 *pb = in + (size_t)b * h * w * C + 8 * g;
    auto ldrow = [&](int r, uint4 (&v)[2]) {
        r = r < 0 ? 0 : (r >= h ? h - 1 : r);
        const bf16 *pr = pb + (size_t)r * w * C;
        v[0] = *reinterpret_cast<const uint4 *>(pr + (size_t)x0 * C);
        v[1] = *reinterpret_cast<const uint4 *>(pr + (size_t)x1 * C);
    };
    uint4 win[3][2];  // coarse rows i - 1, i, i + 1 at columns x0, x1
    ldrow(i0 - 1, win[0]);
    ldrow(i0, win[1]);
    for (int i = i0; i < i1; ++i) {
        ldrow(i + 1, win[2]);
#pragma unroll
        for (int ar = 0; ar < 2; ++ar) {
            int y0, y1;
            float ly;
            up_src(2 * i + ar, h, y0, y1, ly);
            const int r0 = y0 - i + 1, r1 = y1 - i + 1;
            const f8 a00 = u4_to_f8(up_pick(r0, win[0][0], win[1][0], win[2][0]));
            const f8 a01 = u4_to_f8(up_pick(r0, win[0][1], win[1][1], win[2][1]));
            const f8 a10 = u4_to_f8(up_pick(r1, win[0][0], win[1][0], win[2][0]));
            const f8 a11 = u4_to_f8(up_pick(r1, win[0][1], win[1][1], win[2][1]));
            st8(out + (((size_t)b * 2 * h + 2 * i + ar) * W + x) * C + 8 * g,
                up_blend8(a00, a01, a10, a11, ly, lx));
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            win[0][q] = win[1][q];
            win[1][q] = win[2][q];
        }
    }
}

// 1D adjoint weights of the half-pixel x2 interpolation: coarse i receives
// from fine 2i-1 (1/4), 2i (3/4, +1/4 at i = 0), 2i+1 (3/4, +1/4 at i = n-1),
// 2i+2 (1/4).
__device__ __forceinline__ void up_adj(int i, int n, int *o, float *wt)
{
    o[0] = 2 * i - 1; wt[0] = i >= 1 ? 0.25f : 0.f;
    o[1] = 2 * i;     wt[1] = 0.75f + (i == 0 ? 0.25f : 0.f);
    o[2] = 2 * i + 1; wt[2] = 0.75f + (i == n - 1 ? 0.25f : 0.f);
    o[3] = 2 * i + 2; wt[3] = i <= n - 2 ? 0.25f : 0.f;
}

__global__ void k_up2_bwd(const float *__restrict__ dout, int cstride, int coff, int B, int h, int w,
                          int C, float *__restrict__ din, int accumulate)
{
    const int H = 2 * h, W = 2 * w;
    const int n = B * h * w * C;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c = i % C, r = i / C;
        int xi = r % w, r2 = r / w;
        int yi = r2 % h, b = r2 / h;
        int oy[4], ox[4];
        float wy[4], wx[4];
        up_adj(yi, h, oy, wy);
        up_adj(xi, w, ox, wx);
        float acc = 0.f;
        for (int a = 0; a < 4; ++a) {
            if (wy[a] == 0.f) continue;
            for (int d = 0; d < 4; ++d) {
                if (wx[d] == 0.f) continue;
                acc += wy[a] * wx[d] *
                       dout[(((size_t)b * H + oy[a]) * W + ox[d]) * cstride + coff + c];
            }
        }
        din[i] = accumulate ? din[i] + acc : acc;
    }
}

// The same for 8 consecutive channels per thread (two 16-byte loads per
// fine pixel; C, cstride and coff multiples of 4): the same products summed
// in the same order.
__global__ void k_up2_bwd8(const float *__restrict__ dout, int cstride, int coff, int B, int h, int w,
                           int C, float *__restrict__ din, int accumulate)
{
    const int H = 2 * h, W = 2 * w, C8 = C / 8;
    const size_t n = (size_t)B * h * w * C8;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C8) * 8;
        const size_t r = i / C8;
        const int xi = (int)(r % w);
        const size_t r2 = r / w;
        const int yi = (int)(r2 % h), b = (int)(r2 / h);
        int oy[4], ox[4];
        float wy[4], wx[4];
        up_adj(yi, h, oy, wy);
        up_adj(xi, w, ox, wx);
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int a = 0; a < 4; ++a) {
            if (wy[a] == 0.f) continue;
            for (int d = 0; d < 4; ++d) {
                if (wx[d] == 0.f) continue;
                const float wt = wy[a] * wx[d];
                const float *src = dout + (((size_t)b * H + oy[a]) * W + ox[d]) * cstride + coff + c;
                const float4 u = *reinterpret_cast<const float4 *>(src);
                const float4 v = *reinterpret_cast<const float4 *>(src + 4);
                acc[0] += wt * u.x;
                acc[1] += wt * u.y;
                acc[2] += wt * u.z;
                acc[3] += wt * u.w;
                acc[4] += wt * v.x;
                acc[5] += wt * v.y;
                acc[6] += wt * v.z;
                acc[7] += wt * v.w;
            }
        }
        float4 *o = reinterpret_cast<float4 *>(din + r * C + c);
        if (accumulate) {
            const float4 p0 = o[0], p1 = o[1];
            o[0] = make_float4(p0.x + acc[0], p0.y + acc[1], p0.z + acc[2], p0.w + acc[3]);
            o[1] = make_float4(p1.x + acc[4], p1.y + acc[5], p1.z + acc[6], p1.w + acc[7]);
        } else {
            o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
            o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
        }
    }
}

__global__ void k_slice_add(const float *__restrict__ src, int cstride, int coff, size_t P, int C,
                            float *__restrict__ dst, int accumulate)
{
    const int n = (int)(P * C);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int p = i / C, c = i % C;
        float v = src[(size_t)p * cstride + coff + c];
        dst[i] = accumulate ? dst[i] + v : v;
    }
}

__global__ void k_f32_to_bf16(const float *__restrict__ x, size_t n, bf16 *__restrict__ y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] = (bf16)x[i];
}

// ------------------------------------------------------------------ head
__global__ void k_head_fwd(const bf16 *__restrict__ a, size_t P, int C, const float *__restrict__ Wh,
                           const float *__restrict__ bh, float *__restrict__ out)
{
    __shared__ float w[2 * 256];
    for (int t = threadIdx.x; t < 2 * C; t += blockDim.x) w[t] = Wh[t];
    __syncthreads();
    const int np = (int)P;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
        float s0 = bh[0], s1 = bh[1];
        const bf16 *ap = a + (size_t)p * C;
        for (int c0 = 0; c0 < C; c0 += 8) {
            f8 v = ld8(ap + c0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                s0 += w[c0 + q] * v.v[q];
                s1 += w[C + c0 + q] * v.v[q];
            }
        }
        *reinterpret_cast<float2 *>(out + 2 * (size_t)p) = make_float2(s0, s1);
    }
}

// da[p][c] = sum_k Wh[k][c] dout[p][k] (thread per pixel and 8-channel group)
__global__ void k_head_bwd_da(const float *__restrict__ dout, int P, int C,
                              const float *__restrict__ Wh, float *__restrict__ da)
{
    const int G = C / 8, n = P * G;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int g = i % G, p = i / G;
        float2 d = *reinterpret_cast<const float2 *>(dout + 2 * (size_t)p);
        float o[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] = Wh[8 * g + q] * d.x + Wh[C + 8 * g + q] * d.y;
        float4 *dst = reinterpret_cast<float4 *>(da + (size_t)p * C + 8 * g);
        dst[0] = make_float4(o[0], o[1], o[2], o[3]);
        dst[1] = make_float4(o[4], o[5], o[6], o[7]);
    }
}

// per-block partial sums: entries k*C + c = sum_p dout[p][k] a[p][c], and
// 2C + k = sum_p dout[p][k]; thread t handles channel t % C
__global__ __launch_bounds__(256) void k_head_bwd(const float *__restrict__ dout,
                                                  const bf16 *__restrict__ a, size_t P, int C,
                                                  const float *__restrict__ Wh,
                                                  float *__restrict__ da,
                                                  double *__restrict__ part, int nblk)
{
    (void)Wh;
    (void)da;
    const int t = threadIdx.x, c = t % C, r0 = t / C, rs = 256 / C;
    double s0 = 0.0, s1 = 0.0, b0 = 0.0, b1 = 0.0;
    if (r0 < rs)
        for (size_t p = (size_t)blockIdx.x * rs + r0; p < P; p += (size_t)nblk * rs) {
            float2 d = *reinterpret_cast<const float2 *>(dout + 2 * p);
            float v = (float)a[p * C + c];
            s0 += (double)d.x * v;
            s1 += (double)d.y * v;
            if (c == 0) {
                b0 += d.x;
                b1 += d.y;
            }
        }
    __shared__ double sh[4][256];
    sh[0][t] = s0;
    sh[1][t] = s1;
    sh[2][t] = b0;
    sh[3][t] = b1;
    __syncthreads();
    const int ncol = 2 * C + 2;
    for (int col = t; col < ncol; col += 256) {
        double acc = 0.0;
        if (col < 2 * C) {
            int k = col / C, cc = col % C;
            for (int r = 0; r < rs; ++r) acc += sh[k][r * C + cc];
        } else {
            int k = col - 2 * C;
            for (int r = 0; r < rs; ++r) acc += sh[2 + k][r * C];
        }
        part[(size_t)blockIdx.x * ncol + col] = acc;
    }
}

__global__ void k_head_bwd_finish(const double *__restrict__ part, int nblk, int C,
                                  float *__restrict__ dWh, float *__restrict__ dbh)
{
    const int ncol = 2 * C + 2;
    const int t = blockIdx.x;
    if (t >= ncol) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 64) s += part[(size_t)k * ncol + t];
    s = wave_sum(s);
    if (threadIdx.x != 0) return;
    if (t < 2 * C)
        dWh[t] += (float)s;
    else
        dbh[t - 2 * C] += (float)s;
}

// ------------------------------------------------------------------ wrapper
// rc = R(h^2 f r) (full weighting, zero outside) and partial sums of
// |rc|^2, with f = fscale[rhs] (1 without fscale) applied to each sample of r
// as it is loaded.  Thread per pair of coarse points (I, 2K), (I, 2K + 1):
// fine rows 2I - 1 .. 2I + 1, columns 4K - 1 .. 4K + 3 (one float2 and two
// float4 loads a row).
__global__ __launch_bounds__(256) void k_restrict_scaled(const float2 *__restrict__ r, size_t rs,
                                                         int n, float2 *__restrict__ rc,
                                                         double *__restrict__ part, int nblk,
                                                         const int *__restrict__ idx,
                                                         const double *__restrict__ fscale)
{
    const int b = blockIdx.y, nc = n / 2, hp = nc / 2;
    const float h2 = 1.f / ((float)n * (float)n);
    const int ib = idx ? idx[b] : b;
    const float f = fscale ? (float)fscale[ib] : 1.f;
    const float2 *rb = r + (size_t)ib * rs;
    double acc = 0.0;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < nc * hp; t += nblk * 256) {
        const int I = t / hp, K = t - I * hp;
        float s0r = 0.f, s0i = 0.f, s1r = 0.f, s1i = 0.f;
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            const int i = 2 * I + a;
            if (i < 0 || i >= n) continue;
            const float wr = a == 0 ? 0.5f : 0.25f;
            const float2 *row = rb + (size_t)i * n + 4 * K;
            float2 m1 = K > 0 ? row[-1] : make_float2(0.f, 0.f);
            float4 p01 = *reinterpret_cast<const float4 *>(row);
            float4 p23 = *reinterpret_cast<const float4 *>(row + 2);
            m1 = make_float2(m1.x * f, m1.y * f);
            p01 = make_float4(p01.x * f, p01.y * f, p01.z * f, p01.w * f);
            p23 = make_float4(p23.x * f, p23.y * f, p23.z * f, p23.w * f);
            // coarse 2K: columns 4K - 1, 4K, 4K + 1; coarse 2K + 1: 4K + 1, 4K + 2, 4K + 3
            s0r += wr * (0.25f * m1.x + 0.5f * p01.x + 0.25f * p01.z);
            s0i += wr * (0.25f * m1.y + 0.5f * p01.y + 0.25f * p01.w);
            s1r += wr * (0.25f * p01.z + 0.5f * p23.x + 0.25f * p23.z);
            s1i += wr * (0.25f * p01.w + 0.5f * p23.y + 0.25f * p23.w);
        }
        s0r *= h2;
        s0i *= h2;
        s1r *= h2;
        s1i *= h2;
        *reinterpret_cast<float4 *>(rc + (size_t)b * nc * nc + (size_t)I * nc + 2 * K) =
            make_float4(s0r, s0i, s1r, s1i);
        acc += (double)s0r * s0r + (double)s0i * s0i + (double)s1r * s1r + (double)s1i * s1i;
    }
    acc = wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)b * nblk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_rms(const double *__restrict__ part, int nblk, int nc, double *__restrict__ s)
{
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    double a = 0.0;
    for (int k = 0; k < nblk; ++k) a += part[(size_t)b * nblk + k];
    s[b] = sqrt(a / ((double)nc * nc));
}

// grid (coarse columns, coarse rows, batch)
__global__ void k_pack_input(const float2 *__restrict__ rc, const double *__restrict__ s, int n,
                             const float *__restrict__ kf, const float *__restrict__ kc,
                             bf16 *__restrict__ x0, int xs)
{
    const int nc = n / 2;
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nc) return;
    const int I = blockIdx.y, b = blockIdx.z;
    const size_t i = ((size_t)b * nc + I) * nc + J;
    const double sb = s[b];
    const float inv = sb > 0.0 ? (float)(1.0 / sb) : 0.f;
    const float2 v = rc[i];
    const float kap = kf ? kf[(size_t)(2 * I) * n + 2 * J] : kc[i];
    f8 head;
    head.v[0] = v.x * inv;
    head.v[1] = v.y * inv;
    head.v[2] = kap;
#pragma unroll
    for (int q = 3; q < 8; ++q) head.v[q] = 0.f;
    // channels 8 .. xs - 1 (if any) are zero from allocation on
    st8(x0 + i * xs, head);
}

// e (+)= P(s (out0 + i out1)), P bilinear prolongation (transposed stride-2
// convolution with (1/4)[1 2 1; 2 4 2; 1 2 1]).  Thread per fine row i and
// coarse column J: fine pixels (i, 2J) (coarse column J, weight 1) and
// (i, 2J + 1) (columns J, J + 1, weight 1/2 each); fine row i reads coarse
// row i / 2 (even i, weight 1) or rows (i - 1) / 2 and (i + 1) / 2 (odd i,
// weight 1/2 each), zero outside.
// grid (coarse columns, fine rows, right-hand sides)
__global__ void k_net_output(const float *__restrict__ out, const double *__restrict__ s, int n,
                             float2 *__restrict__ e, size_t es, int accumulate,
                             const int *__restrict__ mask, const int *__restrict__ pos)
{
    const int nc = n / 2;
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nc) return;
    const int i = blockIdx.y, b = blockIdx.z;
    {
        float4 *pe = reinterpret_cast<float4 *>(e + (size_t)b * es + (size_t)i * n + 2 * J);
        const int q = pos ? pos[b] : b;  // the right-hand side's sample in the network batch
        if (q < 0 || (mask && !mask[b])) {
            if (!accumulate) *pe = make_float4(0.f, 0.f, 0.f, 0.f);
            return;
        }
        const float2 *ob = reinterpret_cast<const float2 *>(out + (size_t)q * nc * nc * 2);
        float2 c0 = make_float2(0.f, 0.f), c1 = c0;  // rows blended at columns J and J + 1
        const int Ia = i >> 1, Ib = (i + 1) >> 1;
        const int nrow = (i & 1) ? 2 : 1;
        for (int u = 0; u < nrow; ++u) {
            const int I = u ? Ib : Ia;
            if (I >= nc) continue;
            const float2 v0 = ob[(size_t)I * nc + J];
            const float2 v1 = J + 1 < nc ? ob[(size_t)I * nc + J + 1] : make_float2(0.f, 0.f);
            c0.x += v0.x;
            c0.y += v0.y;
            c1.x += v1.x;
            c1.y += v1.y;
        }
        const float wi = (i & 1) ? 0.5f : 1.f;
        const float sc = (float)s[q] * wi;
        float4 val = make_float4(sc * c0.x, sc * c0.y, 0.5f * sc * (c0.x + c1.x), 0.5f * sc * (c0.y + c1.y));
        if (accumulate) {
            const float4 o = *pe;
            val.x += o.x;
            val.y += o.y;
            val.z += o.z;
            val.w += o.w;
        }
        *pe = val;
    }
}

// d = P(out_b) - e_b / s_b on the fine grid, partial sums of |d|^2
__global__ __launch_bounds__(256) void k_loss_fine(const float *__restrict__ out,
                                                   const double *__restrict__ s, int n,
                                                   const float2 *__restrict__ e,
                                                   float2 *__restrict__ d,
                                                   double *__restrict__ part, int nblk)
{
    const int b = blockIdx.y, nc = n / 2;
    const float *ob = out + (size_t)b * nc * nc * 2;
    const float inv = s[b] > 0.0 ? (float)(1.0 / s[b]) : 0.f;
    double acc = 0.0;
    for (int pix = blockIdx.x * 256 + threadIdx.x; pix < n * n; pix += nblk * 256) {
        int i = pix / n, j = pix - i * n;
        float sr = 0.f, si = 0.f;
        int Ia = i >> 1, Ib = (i + 1) >> 1, Ja = j >> 1, Jb = (j + 1) >> 1;
        float wi = (i & 1) ? 0.5f : 1.f, wj = (j & 1) ? 0.5f : 1.f;
        for (int u = 0; u < ((i & 1) ? 2 : 1); ++u) {
            int I = u ? Ib : Ia;
            if (I >= nc) continue;
            for (int v = 0; v < ((j & 1) ? 2 : 1); ++v) {
                int J = v ? Jb : Ja;
                if (J >= nc) continue;
                sr += ob[((size_t)I * nc + J) * 2];
                si += ob[((size_t)I * nc + J) * 2 + 1];
            }
        }
        float2 t = e[(size_t)b * n * n + pix];
        float dr = wi * wj * sr - t.x * inv, di = wi * wj * si - t.y * inv;
        d[(size_t)b * n * n + pix] = make_float2(dr, di);
        acc += (double)dr * dr + (double)di * di;
    }
    acc = wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)b * nblk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dout = (2 / (B n^2)) P^T d with P^T = 4 R
__global__ void k_loss_back(const float2 *__restrict__ d, int nb, int n, float *__restrict__ dout)
{
    const int nc = n / 2;
    const float k = 8.f / ((float)nb * (float)n * (float)n);
    const size_t total = (size_t)nb * nc * nc;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        int b = (int)(idx / ((size_t)nc * nc));
        size_t pix = idx % ((size_t)nc * nc);
        int I = (int)(pix / nc), J = (int)(pix % nc);
        const float2 *db = d + (size_t)b * n * n;
        float sr = 0.f, si = 0.f;
        for (int a = -1; a <= 1; ++a)
            for (int c = -1; c <= 1; ++c) {
                int i = 2 * I + a, j = 2 * J + c;
                if (i < 0 || j < 0 || i >= n || j >= n) continue;
                float wgt = (a == 0 ? 0.5f : 0.25f) * (c == 0 ? 0.5f : 0.25f);
                float2 v = db[(size_t)i * n + j];
                sr += wgt * v.x;
                si += wgt * v.y;
            }
        dout[2 * idx] = k * sr;
        dout[2 * idx + 1] = k * si;
    }
}

__global__ void k_loss_finish(const double *__restrict__ part, int nblk, int nb, int n,
                              double *__restrict__ loss)
{
    double a = 0.0;
    for (int k = threadIdx.x; k < nb * nblk; k += 64) a += part[k];
    a = wave_sum(a);
    if (threadIdx.x == 0) *loss = a / ((double)n * n) / nb;
}

// ------------------------------------------------------------------ params
__global__ void k_pack_weights(const float *__restrict__ Wc, int Cout, int Cin,
                               const int *__restrict__ map, int Cpad, bf16 *__restrict__ Wp,
                               bf16 *__restrict__ Wd)
{
    const size_t total = (size_t)Cout * 9 * Cpad;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        int cp = (int)(i % Cpad);
        int tap = (int)((i / Cpad) % 9);
        int co = (int)(i / ((size_t)Cpad * 9));
        int ci = map[cp];
        float w = ci >= 0 ? Wc[((size_t)co * Cin + ci) * 9 + tap] : 0.f;
        float wf = ci >= 0 ? Wc[((size_t)co * Cin + ci) * 9 + (8 - tap)] : 0.f;
        Wp[i] = (bf16)w;
        Wd[((size_t)cp * 9 + tap) * Cout + co] = (bf16)wf;
    }
}

__global__ void k_unpack_wgrad(const float *__restrict__ dW, int Cout, int Cin,
                               const int *__restrict__ map, int Cpad, float *__restrict__ gW)
{
    const size_t total = (size_t)Cout * 9 * Cpad;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        int cp = (int)(i % Cpad);
        int tap = (int)((i / Cpad) % 9);
        int co = (int)(i / ((size_t)Cpad * 9));
        int ci = map[cp];
        if (ci >= 0) gW[((size_t)co * Cin + ci) * 9 + tap] += dW[i];
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.f - b1) * gi;
        float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_bn_running(float *__restrict__ rm, float *__restrict__ rv,
                             const float *__restrict__ mean, const float *__restrict__ var, int C,
                             float mom, float unb)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    rm[c] = (1.f - mom) * rm[c] + mom * mean[c];
    rv[c] = (1.f - mom) * rv[c] + mom * var[c] * unb;
}

__global__ void k_fold_bn(const float *__restrict__ g, const float *__restrict__ b,
                          const float *__restrict__ rm, const float *__restrict__ rv, int C,
                          float eps, float *__restrict__ scale, float *__restrict__ shift)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float sc = g[c] / sqrtf(rv[c] + eps);
    scale[c] = sc;
    shift[c] = b[c] - rm[c] * sc;
}

__global__ void k_nchw_to_nhwc(const float *__restrict__ x, int B, int C, int H, int W, int Cp,
                               bf16 *__restrict__ y)
{
    const size_t n = (size_t)B * H * W * Cp;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        int c = (int)(i % Cp);
        size_t p = i / Cp;
        int xx = (int)(p % W), yy = (int)((p / W) % H);
        size_t b = p / ((size_t)W * H);
        y[i] = c < C ? (bf16)x[((b * C + c) * H + yy) * W + xx] : (bf16)0.f;
    }
}

__global__ void k_nhwc_to_nchw(const float *__restrict__ x, int B, int C, int H, int W,
                               float *__restrict__ y)
{
    const size_t n = (size_t)B * H * W * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        int xx = (int)(i % W), yy = (int)((i / W) % H);
        int c = (int)((i / ((size_t)W * H)) % C);
        size_t b = i / ((size_t)W * H * C);
        y[i] = x[((b * H + yy) * W + xx) * C + c];
    }
}

inline int grid_for(size_t n, int block = 256, int cap = 8192)
{
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

// blocks of the BN partial-sum kernels: about 16 rows per thread, at most
// as many as the 8 MB reduction scratch holds (2 nblk C doubles + C floats)
inline int red_blocks(size_t P, int C)
{
    size_t rows = 256 / (C / 4);
    size_t b = (P + rows * 16 - 1) / (rows * 16);
    size_t cap = std::min<size_t>(4096, ((size_t)1 << 19) / C - 1);
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

// ================================================================== launchers

namespace {

// one source of 8 channels per pixel padded to a 32-channel block: the
// three-step form of k_conv3x3
bool conv_in8(const Srcs &in)
{
    return in.n == 1 && in.Ctot == 32 && in.s[0].stride == 8;
}

// launch shape of one convolution: the kernel (0: k_conv3x3, 256 threads,
// tile height 4 MF; 1: k_conv3x3d, 512 threads, tile height 8 MF), pixel
// rows per wavefront and the number of workgroups walking the tiles
struct ConvShape {
    int mf, blocks, kind = 1;
};

void conv_dispatch(const ConvShape &c, const Srcs &in, int B, int H, int W, const bf16 *Wt, int Cout,
                   int mode, float *out32, bf16 *out16, const float *scale, const float *shift,
                   float slope, hipStream_t s, const ConvEpi &epi)
{
    const int NF = Cout >= 64 ? 4 : 2;
    const int CO = 16 * NF;
    const int ncob = (Cout + CO - 1) / CO;
    const int ep = epi.head_out ? 2 : (epi.pool ? 1 : 0);
    // an upsampled first source (plain epilogue, more than one chunk, at
    // most 32 output channels) runs on k_conv3x3d only
    const bool upsrc = in.s[0].up != 0;
    if ((c.kind == 1 || upsrc) && !conv_in8(in)) {
        const long long ntiles = (long long)B * ((H + 8 * c.mf - 1) / (8 * c.mf)) * ((W + 15) / 16);
        dim3 grid((unsigned)std::max<long long>(1, std::min<long long>(ntiles, c.blocks)), ncob);
        const bool rw = in.Ctot > 32;
#define CONVUP(mf, nf)                                                                                         \
    hipLaunchKernelGGL((k_conv3x3d<mf, nf, 0, true, true>), grid, dim3(512), 0, s, in, B, H, W, Wt, Cout, mode, \
                       out32, out16, scale, shift, slope, epi)
        if (upsrc) {  // 32 output channels (NF == 2) only
            if (c.mf == 4)
                CONVUP(4, 2);
            else
                CONVUP(2, 2);
            return;
        }
#undef CONVUP
#define CONVD1(mf, nf, rw)                                                                                    \
    do {                                                                                                     \
        if (ep == 2)                                                                                         \
            hipLaunchKernelGGL((k_conv3x3d<mf, nf, 2, rw>), grid, dim3(512), 0, s, in, B, H, W, Wt, Cout, mode, \
                               out32, out16, scale, shift, slope, epi);                                       \
        else if (ep == 1)                                                                                    \
            hipLaunchKernelGGL((k_conv3x3d<mf, nf, 1, rw>), grid, dim3(512), 0, s, in, B, H, W, Wt, Cout, mode, \
                               out32, out16, scale, shift, slope, epi);                                       \
        else                                                                                                 \
            hipLaunchKernelGGL((k_conv3x3d<mf, nf, 0, rw>), grid, dim3(512), 0, s, in, B, H, W, Wt, Cout, mode, \
                               out32, out16, scale, shift, slope, epi);                                       \
    } while (0)
#define CONVD(mf, nf)            \
    do {                         \
        if (rw)                  \
            CONVD1(mf, nf, true);  \
        else                     \
            CONVD1(mf, nf, false); \
    } while (0)
        if (c.mf == 4 && NF == 4)
            CONVD(4, 4);
        else if (c.mf == 4)
            CONVD(4, 2);
        else if (NF == 4)
            CONVD(2, 4);
        else
            CONVD(2, 2);
#undef CONVD
#undef CONVD1
        return;
    }
    const long long ntiles = (long long)B * ((H + 4 * c.mf - 1) / (4 * c.mf)) * ((W + 15) / 16);
    // (shapes chosen for the 512-thread kernel count half-size workgroups
    // four times: about the same number of threads in flight)
    const int blocks = c.kind == 1 ? 4 * c.blocks : c.blocks;
    dim3 grid((unsigned)std::max<long long>(1, std::min<long long>(ntiles, blocks)), ncob);
    if (conv_in8(in) && ep == 0) {
        if (c.mf == 4 && NF == 4)
            hipLaunchKernelGGL((k_conv3x3<4, 4, 0, true>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,
                               out32, out16, scale, shift, slope, epi);
        else if (c.mf == 4)
            hipLaunchKernelGGL((k_conv3x3<4, 2, 0, true>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,
                               out32, out16, scale, shift, slope, epi);
        else if (NF == 4)
            hipLaunchKernelGGL((k_conv3x3<2, 4, 0, true>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,
                               out32, out16, scale, shift, slope, epi);
        else
            hipLaunchKernelGGL((k_conv3x3<2, 2, 0, true>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,
                               out32, out16, scale, shift, slope, epi);
        return;
    }
#define CONV_LAUNCH(mf, nf)                                                                                 \
    do {                                                                                                    \
        if (ep == 2)                                                                                        \
            hipLaunchKernelGGL((k_conv3x3<mf, nf, 2>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,    \
                               out32, out16, scale, shift, slope, epi);                                      \
        else if (ep == 1)                                                                                   \
            hipLaunchKernelGGL((k_conv3x3<mf, nf, 1>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,    \
                               out32, out16, scale, shift, slope, epi);                                      \
        else                                                                                                \
            hipLaunchKernelGGL((k_conv3x3<mf, nf, 0>), grid, dim3(256), 0, s, in, B, H, W, Wt, Cout, mode,    \
                               out32, out16, scale, shift, slope, epi);                                      \
    } while (0)
    if (c.mf == 4 && NF == 4)
        CONV_LAUNCH(4, 4);
    else if (c.mf == 4)
        CONV_LAUNCH(4, 2);
    else if (NF == 4)
        CONV_LAUNCH(2, 4);
    else
        CONV_LAUNCH(2, 2);
#undef CONV_LAUNCH
}

// Heuristic: 16-row tiles for large images, 8-row tiles for small ones;
// about eight workgroups per compute unit in total.
ConvShape conv_default(int H, int Cout)
{
    const int ncob = (Cout + (Cout >= 64 ? 63 : 31)) / (Cout >= 64 ? 64 : 32);
    return ConvShape{H >= 128 ? 4 : 2, std::max(1, 512 / ncob), 1};
}

// epilogue and source variant of a convolution (part of the tuning key)
int conv_variant(const Srcs &in, int mode, const ConvEpi &epi)
{
    return mode | ((epi.pool != nullptr) << 1) | ((epi.head_out != nullptr) << 2) |
           ((epi.cmap != nullptr) << 3) | ((in.wstride != 0 && in.wstride != in.Ctot) << 4) |
           (conv_in8(in) << 5) | ((epi.raw16 != nullptr) << 6) | ((in.s[0].up != 0) << 7) | ((epi.nseg > 0) << 8);
}

struct Tuner {
    std::mutex mu;
    int enabled = 0;
    std::map<std::array<int, 6>, ConvShape> table;
    // a launch shape forced on every convolution (kind, mf, workgroups per
    // compute unit as in the candidate list), kind < 0 = none
    int force_kind = -1, force_mf = 0, force_per_cu = 0;
};
Tuner g_tune;

// the candidate of conv_tune for (kind, mf, per_cu)
ConvShape conv_candidate(int kind, int mf, int per_cu, int Cout)
{
    const int ncob = (Cout + (Cout >= 64 ? 63 : 31)) / (Cout >= 64 ? 64 : 32);
    return ConvShape{mf, std::max(1, 256 * per_cu * (kind ? 1 : 2) / ncob), kind};
}

// Times every candidate launch shape for this convolution (three runs each,
// HIP events on the caller's stream) and keeps the fastest.  Each run
// recomputes the same output, so tuning leaves the result unchanged.
ConvShape conv_tune(const Srcs &in, int B, int H, int W, const bf16 *Wt, int Cout, int mode, float *out32,
                    bf16 *out16, const float *scale, const float *shift, float slope, hipStream_t s,
                    const ConvEpi &epi)
{
    ConvShape best = conv_default(H, Cout);
    float best_ms = 1e30f;
    // the timing runs write everything to out32 (the caller's launch after
    // tuning routes the ranges)
    ConvEpi tepi = epi;
    tepi.nseg = 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return best;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return best;
    }
    for (int kind : {0, 1})
    for (int mf : {2, 4})
        for (int per_cu : {1, 2, 4, 8}) {
            if (kind == 0 && in.s[0].up) continue;  // runs on k_conv3x3d only
            ConvShape c = conv_candidate(kind, mf, per_cu, Cout);
            conv_dispatch(c, in, B, H, W, Wt, Cout, mode, out32, out16, scale, shift, slope, s, tepi);  // warm
            hipEventRecord(e0, s);
            for (int r = 0; r < 3; ++r)
                conv_dispatch(c, in, B, H, W, Wt, Cout, mode, out32, out16, scale, shift, slope, s, tepi);
            hipEventRecord(e1, s);
            float ms = 0.f;
            if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best;
}

}  // namespace

// bf16 outputs above this size are stored nontemporally (MI355X: 256 MB of
// last-level cache; a smaller output can still be read back from it by the
// next layer)
constexpr size_t CONV_NT_BYTES = 320ull << 20;

void launch_conv3x3(const Srcs &in, int B, int H, int W, const bf16 *Wt, int Cout, int mode,
                    float *out32, bf16 *out16, const float *scale, const float *shift,
                    float slope, hipStream_t s, const ConvEpi &epi_in)
{
    ConvEpi epi = epi_in;
    epi.nt = (size_t)B * H * W * Cout * sizeof(bf16) > CONV_NT_BYTES;
    ConvShape c = conv_default(H, Cout);
    {
        std::lock_guard<std::mutex> lk(g_tune.mu);
        if (g_tune.force_kind >= 0) {
            c = conv_candidate(g_tune.force_kind, g_tune.force_mf, g_tune.force_per_cu, Cout);
            conv_dispatch(c, in, B, H, W, Wt, Cout, mode, out32, out16, scale, shift, slope, s, epi);
            return;
        }
    }
    if (g_tune.enabled) {
        // batch sizes share an entry per power-of-two bucket: a batch that
        // shrinks as right-hand sides converge is not tuned again each time
        int Bk = 1;
        while (Bk < B) Bk *= 2;
        const std::array<int, 6> key{Bk, H, W, in.Ctot, Cout, conv_variant(in, mode, epi)};
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            std::lock_guard<std::mutex> lk(g_tune.mu);
            auto it = g_tune.table.find(key);
            if (it == g_tune.table.end())
                it = g_tune.table.emplace(key, conv_tune(in, B, H, W, Wt, Cout, mode, out32, out16, scale,
                                                          shift, slope, s, epi)).first;
            c = it->second;
        } else {
            std::lock_guard<std::mutex> lk(g_tune.mu);
            auto it = g_tune.table.find(key);
            if (it != g_tune.table.end()) c = it->second;
        }
    }
    conv_dispatch(c, in, B, H, W, Wt, Cout, mode, out32, out16, scale, shift, slope, s, epi);
}

int conv_autotune(int enable)
{
    std::lock_guard<std::mutex> lk(g_tune.mu);
    const int prev = g_tune.enabled;
    g_tune.enabled = enable ? 1 : 0;
    if (enable < 0) g_tune.table.clear();
    return prev;
}

int conv_force(int kind, int mf, int per_cu)
{
    if (kind >= 0 && (kind > 1 || (mf != 2 && mf != 4) || per_cu < 1 || per_cu > 64)) return -1;
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.force_kind = kind < 0 ? -1 : kind;
    g_tune.force_mf = mf;
    g_tune.force_per_cu = per_cu;
    return 0;
}

int conv_autotune_entries()
{
    std::lock_guard<std::mutex> lk(g_tune.mu);
    return (int)g_tune.table.size();
}

static int wgrad_nsplit(int B, int H, int W, int Cout, int Ctot)
{
    const int steps = B * H * ((W + WG_SEG - 1) / WG_SEG);
    const int CB = Cout >= 64 ? 64 : 32, IB = Ctot >= 64 ? 64 : 32;
    const int blocks = ((Cout + CB - 1) / CB) * ((Ctot + IB - 1) / IB);
    // as many workgroups as the CUs hold at once (the kernels' register use
    // allows 2, 3 or 5 per CU), at least 32 steps per split
    const int per_cu = (CB == 64 && IB == 64) ? 2 : (CB == 64 || IB == 64) ? 3 : 5;
    int want = std::max(1, 256 * per_cu / blocks);
    return std::max(1, std::min(want, (steps + 31) / 32));
}

size_t wgrad_scratch(int B, int H, int W, int Cout, int Ctot)
{
    // the partials, then the 32-split group sums
    const size_t n = (size_t)Cout * 9 * Ctot;
    const size_t ns = (size_t)wgrad_nsplit(B, H, W, Cout, Ctot);
    return ns * n + ((ns + 31) / 32) * n;
}

void launch_wgrad(const Srcs &x, const bf16 *dy, int B, int H, int W, int Cout, float *dW,
                  float *part, hipStream_t s)
{
    const int steps = B * H * ((W + WG_SEG - 1) / WG_SEG);
    int nsplit = wgrad_nsplit(B, H, W, Cout, x.Ctot);
    const int per = (steps + nsplit - 1) / nsplit;
    nsplit = (steps + per - 1) / per;
    const int CB = Cout >= 64 ? 64 : 32, IB = x.Ctot >= 64 ? 64 : 32;
    dim3 grid(nsplit, ((Cout + CB - 1) / CB) * ((x.Ctot + IB - 1) / IB));
    if (CB == 64 && IB == 64)
        hipLaunchKernelGGL((k_wgrad<4, 4>), grid, dim3(256), 0, s, x, dy, B, H, W, Cout, per, part);
    else if (CB == 64)
        hipLaunchKernelGGL((k_wgrad<4, 2>), grid, dim3(256), 0, s, x, dy, B, H, W, Cout, per, part);
    else if (IB == 64)
        hipLaunchKernelGGL((k_wgrad<2, 4>), grid, dim3(256), 0, s, x, dy, B, H, W, Cout, per, part);
    else
        hipLaunchKernelGGL((k_wgrad<2, 2>), grid, dim3(256), 0, s, x, dy, B, H, W, Cout, per, part);
    const size_t n = (size_t)Cout * 9 * x.Ctot;
    const int ngroup = (nsplit + 31) / 32;
    float *tmp = part + (size_t)nsplit * n;
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(n), ngroup), dim3(256), 0, s, part, nsplit, n, tmp, ngroup);
    hipLaunchKernelGGL(k_sum_groups, dim3(grid_for(n)), dim3(256), 0, s, tmp, ngroup, n, dW);
}

void launch_bn_stats(const float *y, size_t P, int C, double *part, float *mean, float *rstd,
                     float *var_out, hipStream_t s)
{
    int nblk = red_blocks(P, C);
    hipLaunchKernelGGL(k_bn_partial, dim3(nblk), dim3(256), 0, s, y, P, C, part, nblk);
    hipLaunchKernelGGL(k_bn_finish, dim3(C), dim3(64), 0, s, part, nblk, C, P, mean, rstd, var_out);
}

void launch_bn_act_fwd(const float *y, size_t P, int C, const float *mean, const float *rstd,
                       const float *g, const float *b, float slope, bf16 *a, hipStream_t s)
{
    size_t n = P * C;
    hipLaunchKernelGGL(k_bn_act_fwd, dim3(grid_for(n / 8)), dim3(256), 0, s, y, n, C, mean, rstd, g, b,
                       slope, a);
}

void launch_bn_act_bwd(const float *da, const float *y, size_t P, int C, const float *mean,
                       const float *rstd, const float *g, const float *b, float slope,
                       double *part, float *dg, float *db, bf16 *dy, hipStream_t s)
{
    int nblk = red_blocks(P, C);
    hipLaunchKernelGGL(k_bn_bwd_partial, dim3(nblk), dim3(256), 0, s, da, y, P, C, mean, rstd, g, b,
                       slope, part, nblk);
    // per-channel sums (dbeta, dgamma) go to the tail of `part`
    float *sums = reinterpret_cast<float *>(part + (size_t)nblk * C * 2);
    hipLaunchKernelGGL(k_bn_bwd_finish, dim3(C), dim3(64), 0, s, part, nblk, C, dg, db, sums);
    size_t n = P * C;
    hipLaunchKernelGGL(k_bn_bwd_apply, dim3(grid_for(n / 8)), dim3(256), 0, s, da, y, n, C, P, mean, rstd,
                       g, b, slope, sums, dy);
}

void launch_maxpool_fwd(const bf16 *in, int B, int H, int W, int C, bf16 *out, uint8_t *arg,
                        hipStream_t s)
{
    const int row = (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_maxpool_fwd, dim3((row + 255) / 256, H / 2, B), dim3(256), 0, s, in, H, W, C, out,
                       arg);
}

void launch_maxpool_bwd(const float *dout, const uint8_t *arg, int B, int H, int W, int C,
                        int cstride_in, int coff_in, float *din, int din_C, hipStream_t s)
{
    size_t n = (size_t)B * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid_for(n)), dim3(256), 0, s, dout, cstride_in, coff_in, arg,
                       B, H, W, C, din, din_C);
}

void launch_up2_fwd(const bf16 *in, int B, int h, int w, int C, bf16 *out, hipStream_t s)
{
    const int row = 2 * w * (C / 8);
    hipLaunchKernelGGL(k_up2_fwd, dim3((row + 255) / 256, (h + UP_R - 1) / UP_R, B), dim3(256), 0, s, in, h, w,
                       C, out);
}

void launch_up2_bwd(const float *dout, int cstride, int coff, int B, int h, int w, int C,
                    float *din, int accumulate, hipStream_t s)
{
    size_t n = (size_t)B * h * w * C;
    if (C % 8 == 0 && cstride % 4 == 0 && coff % 4 == 0) {
        hipLaunchKernelGGL(k_up2_bwd8, dim3(grid_for(n / 8)), dim3(256), 0, s, dout, cstride, coff, B, h, w, C,
                           din, accumulate);
        return;
    }
    hipLaunchKernelGGL(k_up2_bwd, dim3(grid_for(n)), dim3(256), 0, s, dout, cstride, coff, B, h, w, C,
                       din, accumulate);
}

void launch_slice_add(const float *src, int cstride, int coff, size_t P, int C, float *dst,
                      int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_slice_add, dim3(grid_for(P * C)), dim3(256), 0, s, src, cstride, coff, P, C,
                       dst, accumulate);
}

void launch_nchw_to_nhwc(const float *x, int B, int C, int H, int W, int Cp, bf16 *y, hipStream_t s)
{
    size_t n = (size_t)B * H * W * Cp;
    hipLaunchKernelGGL(k_nchw_to_nhwc, dim3(grid_for(n)), dim3(256), 0, s, x, B, C, H, W, Cp, y);
}

void launch_nhwc_to_nchw(const float *x, int B, int C, int H, int W, float *y, hipStream_t s)
{
    size_t n = (size_t)B * H * W * C;
    hipLaunchKernelGGL(k_nhwc_to_nchw, dim3(grid_for(n)), dim3(256), 0, s, x, B, C, H, W, y);
}

void launch_f32_to_bf16(const float *x, size_t n, bf16 *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(n)), dim3(256), 0, s, x, n, y);
}

void launch_head_fwd(const bf16 *a, size_t P, int C, const float *Wh, const float *bh, float *out,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_head_fwd, dim3(grid_for(P)), dim3(256), 0, s, a, P, C, Wh, bh, out);
}

void launch_head_bwd(const float *dout, const bf16 *a, size_t P, int C, const float *Wh,
                     float *da, double *part, float *dWh, float *dbh, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_bwd_da, dim3(grid_for(P * C / 8)), dim3(256), 0, s, dout, (int)P, C, Wh, da);
    int nblk = red_blocks(P, C);
    hipLaunchKernelGGL(k_head_bwd, dim3(nblk), dim3(256), 0, s, dout, a, P, C, Wh, da, part, nblk);
    hipLaunchKernelGGL(k_head_bwd_finish, dim3(2 * C + 2), dim3(64), 0, s, part, nblk, C, dWh, dbh);
}

void launch_net_input(const float2 *r, size_t rstride, int nb, int n, const float *kappa_fine,
                      const float *kappa_c, float2 *rc, double *part, double *s, bf16 *x0, int x0_stride,
                      hipStream_t st, const int *idx, const double *fscale)
{
    int nc = n / 2;
    int nblk = (int)std::min<size_t>(256, std::max<size_t>(1, ((size_t)nc * nc / 2 + 511) / 512));
    hipLaunchKernelGGL(k_restrict_scaled, dim3(nblk, nb), dim3(256), 0, st, r, rstride, n, rc, part,
                       nblk, idx, fscale);
    hipLaunchKernelGGL(k_rms, dim3(nb), dim3(64), 0, st, part, nblk, nc, s);
    hipLaunchKernelGGL(k_pack_input, dim3((nc + 255) / 256, nc, nb), dim3(256), 0, st, rc, s, n, kappa_fine,
                       kappa_c, x0, x0_stride);
}

void launch_net_output(const float *out, const double *s, int nb, int n, float2 *e, size_t estride,
                       int accumulate, hipStream_t st, const int *mask, const int *pos)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_net_output, dim3((n / 2 + 255) / 256, n, nb), dim3(256), 0, st, out, s, n, e, estride,
                       accumulate, mask, pos);
}

void launch_loss_grad(const float *out, const double *s, int nb, int n, const float2 *e,
                      float2 *dfine, double *part, float *dout, double *loss_out, hipStream_t st)
{
    int nblk = (int)std::min<size_t>(256, std::max<size_t>(1, ((size_t)n * n + 1023) / 1024));
    hipLaunchKernelGGL(k_loss_fine, dim3(nblk, nb), dim3(256), 0, st, out, s, n, e, dfine, part, nblk);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(64), 0, st, part, nblk, nb, n, loss_out);
    size_t tot = (size_t)nb * (n / 2) * (n / 2);
    hipLaunchKernelGGL(k_loss_back, dim3(grid_for(tot)), dim3(256), 0, st, dfine, nb, n, dout);
}

void launch_pack_weights(const float *W, int Cout, int Cin, const int *map, int Cpad, bf16 *Wp,
                         bf16 *Wd, hipStream_t s)
{
    size_t n = (size_t)Cout * 9 * Cpad;
    hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(n)), dim3(256), 0, s, W, Cout, Cin, map, Cpad, Wp,
                       Wd);
}

void launch_unpack_wgrad(const float *dW, int Cout, int Cin, const int *map, int Cpad, float *gW,
                         hipStream_t s)
{
    size_t n = (size_t)Cout * 9 * Cpad;
    hipLaunchKernelGGL(k_unpack_wgrad, dim3(grid_for(n)), dim3(256), 0, s, dW, Cout, Cin, map, Cpad,
                       gW);
}

void launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                 float b2, float eps, int step, hipStream_t s)
{
    float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
}

void launch_bn_running(float *rm, float *rv, const float *mean, const float *var, int C,
                       float momentum, double count, hipStream_t s)
{
    float unb = count > 1.0 ? (float)(count / (count - 1.0)) : 1.f;
    hipLaunchKernelGGL(k_bn_running, dim3((C + 63) / 64), dim3(64), 0, s, rm, rv, mean, var, C,
                       momentum, unb);
}

void launch_fold_bn(const float *g, const float *b, const float *rm, const float *rv, int C,
                    float eps, float *scale, float *shift, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold_bn, dim3((C + 63) / 64), dim3(64), 0, s, g, b, rm, rv, C, eps, scale,
                       shift);
}

}  // namespace helm
