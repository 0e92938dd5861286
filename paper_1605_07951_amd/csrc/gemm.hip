// Batched complex GEMMs on the CDNA4 matrix cores.
//
// A complex product C += A*B is computed as real MFMA products by splitting
// the complex inner index k into two real indices k' = 2k + c (c = 0 real
// part, c = 1 imaginary part):
//     Re C(i,j) = sum_k' A'(i,k') Br'(k',j),   A'(i,2k+c) = c ? Im A : Re A,
//     Im C(i,j) = sum_k' A'(i,k') Bi'(k',j),   Br'(2k+c,j) = c ? -Im B : Re B,
//                                              Bi'(2k+c,j) = c ?  Re B : Im B.
// (4 real multiplies per complex multiply-add, the "4M" form.)  A' is the
// interleaved complex storage read one float per lane, so the operands come
// straight from the interleaved layout staged in LDS.  The MFMA operand
// slots are swapped (the MFMA "A" operand carries B' and its "B" operand
// carries A'), which makes the output lane index run along rows i: 32 (or 16)
// consecutive lanes then store one contiguous column segment of C.
#include "common.h"
#include "kernels.h"

namespace rsrr {

// ----------------------------------------------------------------------------
// complex FP32: v_mfma_f32_32x32x2f32.  The workgroup has WR x WC waves; each
// wave owns BR x BC blocks of 32x32 outputs, so the WG tile is
// (32 WR BR) x (32 WC BC).  In this 4M form it serves the 128x32 products of
// the panel recursion; wider products go to the 3M kernel below.  The 4M
// kernel is kept general (a 128x128 tile of 2x2 waves of 2x2 blocks runs at
// two waves per SIMD).  beta*C is loaded into the accumulators before
// the k loop (its latency overlaps the first LDS stage), alpha is folded
// into the A operand, and the epilogue only stores.
// ----------------------------------------------------------------------------
constexpr int CG_KT = 16, CG_NT = 256;

// Tile t of a matrix -> (row tile, column tile): groups of TG_ROWS row tiles
// sweep the columns together, so the workgroups in flight on one XCD share a
// few row slices of A and column slices of B in its L2 instead of streaming
// all of A once per column of tiles.
constexpr int TG_ROWS = 8;
__device__ __forceinline__ void tile_order(int t, int tilesM, int tilesN, int* ti, int* tj)
{
    const int span = TG_ROWS * tilesN;
    const int g = t / span, first = g * TG_ROWS;
    const int rows = min(tilesM - first, TG_ROWS);
    const int in = t - g * span;
    *ti = first + in % rows;
    *tj = in / rows;
}

template <int WR, int WC, int BR, int BC, bool VEC, int TAG>
__global__ __launch_bounds__(CG_NT, 2) void cgemm_mfma_kernel(
    int M, int N, int K, float alpha,
    const float2* __restrict__ A, int lda, long sA,
    const float2* __restrict__ B, int ldb, long sB,
    float beta, float2* __restrict__ C, int ldc, long sC,
    int tilesM, int tilesN, int batch, long total_padded)
{
    constexpr int BM = 32 * WR * BR, BN = 32 * WC * BC;
    constexpr int AQ = BM * CG_KT / 2 / CG_NT;   // float4 (2 complex) A loads per thread per stage
    constexpr int BQ = BN * CG_KT / 2 / CG_NT;   // float4 B loads per thread per stage
    static_assert(AQ >= 1 && BQ >= 1, "tile too small for the loader");
    // B rows padded by 4 complex (32 B): the staging stores write 8 k-rows of one
    // column per wave, which then fall on different LDS banks
    __shared__ __attribute__((aligned(16))) float As[2][CG_KT][2 * BM];
    __shared__ __attribute__((aligned(16))) float2 Bs[2][CG_KT][BN + 4];

    const long tile = xcd_remap(blockIdx.x, total_padded);
    const long per = (long)tilesM * tilesN;
    const long b = tile / per;
    if (b >= batch) return;
    const int t = (int)(tile - b * per);
    int ti, tj;
    tile_order(t, tilesM, tilesN, &ti, &tj);
    const int i0 = ti * BM;
    const int j0 = tj * BN;
    const float2* Ab = A + b * sA;
    const float2* Bb = B + b * sB;
    float2* Cb = C + b * sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = wave % WR, wj = wave / WR;
    const int li = lane & 31, half = lane >> 5;
    const int wrow = i0 + wi * BR * 32, wcol = j0 + wj * BC * 32;

    // ---- prologue: acc = (beta / alpha) C, scaled by alpha once at the end (bitwise the same
    // for alpha = +-1); output layout: lane li = row, reg r = column 8(r/4)+4 half+r%4 ----
    const bool prod = alpha != 0.f;
    const float cs = prod ? beta / alpha : beta, os = prod ? alpha : 1.f;
    floatx16 accR[BR][BC], accI[BR][BC];
#pragma unroll
    for (int x = 0; x < BR; ++x)
#pragma unroll
        for (int y = 0; y < BC; ++y) {
            const int i = wrow + x * 32 + li;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                float2 c = make_float2(0.f, 0.f);
                if (beta != 0.f && i < M && j < N) c = Cb[i + (long)j * ldc];
                accR[x][y][r] = cs * c.x;
                accI[x][y][r] = cs * c.y;
            }
        }

    floatx4 ra[AQ], rb[BQ];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            const int gi = i0 + ip, gk = k0 + k;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gk < K) {
                const float2* src = Ab + gi + (long)gk * lda;
                if (VEC && gi + 1 < M) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gi < M) { float2 e = src[0]; v[0] = e.x; v[1] = e.y; }
                    if (gi + 1 < M) { float2 e = src[1]; v[2] = e.x; v[3] = e.y; }
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + CG_NT * q;
            const int j = p / (CG_KT / 2), kp = (p % (CG_KT / 2)) * 2;
            const int gj = j0 + j, gk = k0 + kp;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gj < N) {
                const float2* src = Bb + gk + (long)gj * ldb;
                if (VEC && gk + 1 < K) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gk < K) { float2 e = src[0]; v[0] = e.x; v[1] = e.y; }
                    if (gk + 1 < K) { float2 e = src[1]; v[2] = e.x; v[3] = e.y; }
                }
            }
            rb[q] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            *reinterpret_cast<floatx4*>(&As[buf][k][2 * ip]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + CG_NT * q;
            const int j = p / (CG_KT / 2), kp = (p % (CG_KT / 2)) * 2;
            Bs[buf][kp][j] = make_float2(rb[q][0], rb[q][1]);
            Bs[buf][kp + 1][j] = make_float2(rb[q][2], rb[q][3]);
        }
    };

    const int nst = prod ? (K + CG_KT - 1) / CG_KT : 0;
    if (nst > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
    }
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) gload((s + 1) * CG_KT);
#pragma unroll 4
        for (int k = 0; k < CG_KT; ++k) {
            float a[BR], br[BC], bi[BC];
#pragma unroll
            for (int x = 0; x < BR; ++x) a[x] = As[buf][k][2 * (wi * BR * 32 + x * 32 + li) + half];
#pragma unroll
            for (int y = 0; y < BC; ++y) {
                const float2 bv = Bs[buf][k][wj * BC * 32 + y * 32 + li];
                br[y] = half ? -bv.y : bv.x;
                bi[y] = half ? bv.x : bv.y;
            }
#pragma unroll
            for (int x = 0; x < BR; ++x)
#pragma unroll
                for (int y = 0; y < BC; ++y) {
                    accR[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(br[y], a[x], accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(bi[y], a[x], accI[x][y], 0, 0, 0);
                }
        }
        if (s + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue: store ----
#pragma unroll
    for (int x = 0; x < BR; ++x) {
        const int i = wrow + x * 32 + li;
        if (i >= M) continue;
#pragma unroll
        for (int y = 0; y < BC; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (j < N) Cb[i + (long)j * ldc] = make_float2(os * accR[x][y][r], os * accI[x][y][r]);
            }
    }
}

// ----------------------------------------------------------------------------
// complex FP32, "3M" form (Gauss's three-product trick): with A = Ar + i Ai and
// B = Br + i Bi, the three real products T1 = Ar Br, T2 = Ai Bi and
// T3 = (Ar + Ai)(Br + Bi) give Re AB = T1 - T2 and Im AB = T3 - T1 - T2: 3
// real multiplies per complex multiply-add instead of 4.  Here the MFMA's
// inner index of 2 runs over two consecutive complex k (lanes 0-31: k, lanes
// 32-63: k + 1), so one stage of CG_KT complex k takes 3 * CG_KT / 2 MFMAs per
// 32x32 block against 2 * CG_KT for the 4M kernel.  Staging, tile order and
// output layout are those of the 4M kernel; the sums Ar + Ai and Br + Bi are
// formed in registers from the staged values.  beta C enters the
// accumulators as T1 = beta Re C, T2 = 0, T3 = beta (Re C + Im C).  The error
// is bounded normwise like that of the 4M form with a slightly larger
// constant (Higham, "Stability of a method for multiplying complex matrices
// with three real matrix multiplications", SIMAX 1992), which the FP64
// refinement downstream absorbs.  Three accumulator sets per block: with
// 2x2 blocks per wave that is one wave per SIMD, with two blocks two.  The
// workgroup has 64 WR WC threads.
// ----------------------------------------------------------------------------
template <int WR, int WC, int BR, int BC, bool VEC, int TAG>
__global__ __launch_bounds__(64 * WR * WC, (BR * BC <= 2) ? 512 / (64 * WR * WC) : 1) void cgemm3m_mfma_kernel(
    int M, int N, int K, float alpha,
    const float2* __restrict__ A, int lda, long sA,
    const float2* __restrict__ B, int ldb, long sB,
    float beta, float2* __restrict__ C, int ldc, long sC,
    int tilesM, int tilesN, int batch, long total_padded)
{
    constexpr int NT = 64 * WR * WC;
    constexpr int BM = 32 * WR * BR, BN = 32 * WC * BC;
    constexpr int AQ = BM * CG_KT / 2 / NT;
    constexpr int BQ = BN * CG_KT / 2 / NT;
    static_assert(AQ >= 1 && BQ >= 1, "tile too small for the loader");
    static_assert(CG_KT % 2 == 0, "stages hold pairs of k");
    __shared__ __attribute__((aligned(16))) float As[2][CG_KT][2 * BM];
    __shared__ __attribute__((aligned(16))) float2 Bs[2][CG_KT][BN + 4];

    const long tile = xcd_remap(blockIdx.x, total_padded);
    const long per = (long)tilesM * tilesN;
    const long b = tile / per;
    if (b >= batch) return;
    const int t = (int)(tile - b * per);
    int ti, tj;
    tile_order(t, tilesM, tilesN, &ti, &tj);
    const int i0 = ti * BM;
    const int j0 = tj * BN;
    const float2* Ab = A + b * sA;
    const float2* Bb = B + b * sB;
    float2* Cb = C + b * sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = wave % WR, wj = wave / WR;
    const int li = lane & 31, half = lane >> 5;
    const int wrow = i0 + wi * BR * 32, wcol = j0 + wj * BC * 32;

    // alpha leaves the inner loop: the accumulators hold (beta / alpha) C + A B and
    // are scaled by alpha once at the end (bitwise the same for alpha = +-1)
    const bool prod = alpha != 0.f;
    const float cs = prod ? beta / alpha : beta, os = prod ? alpha : 1.f;
    floatx16 t1[BR][BC], t2[BR][BC], t3[BR][BC];
#pragma unroll
    for (int x = 0; x < BR; ++x)
#pragma unroll
        for (int y = 0; y < BC; ++y) {
            const int i = wrow + x * 32 + li;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                float2 c = make_float2(0.f, 0.f);
                if (beta != 0.f && i < M && j < N) c = Cb[i + (long)j * ldc];
                t1[x][y][r] = cs * c.x;
                t2[x][y][r] = 0.f;
                t3[x][y][r] = cs * (c.x + c.y);
            }
        }

    floatx4 ra[AQ], rb[BQ];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            const int gi = i0 + ip, gk = k0 + k;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gk < K) {
                const float2* src = Ab + gi + (long)gk * lda;
                if (VEC && gi + 1 < M) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gi < M) { float2 e = src[0]; v[0] = e.x; v[1] = e.y; }
                    if (gi + 1 < M) { float2 e = src[1]; v[2] = e.x; v[3] = e.y; }
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + NT * q;
            const int j = p / (CG_KT / 2), kp = (p % (CG_KT / 2)) * 2;
            const int gj = j0 + j, gk = k0 + kp;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gj < N) {
                const float2* src = Bb + gk + (long)gj * ldb;
                if (VEC && gk + 1 < K) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gk < K) { float2 e = src[0]; v[0] = e.x; v[1] = e.y; }
                    if (gk + 1 < K) { float2 e = src[1]; v[2] = e.x; v[3] = e.y; }
                }
            }
            rb[q] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            *reinterpret_cast<floatx4*>(&As[buf][k][2 * ip]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + NT * q;
            const int j = p / (CG_KT / 2), kp = (p % (CG_KT / 2)) * 2;
            Bs[buf][kp][j] = make_float2(rb[q][0], rb[q][1]);
            Bs[buf][kp + 1][j] = make_float2(rb[q][2], rb[q][3]);
        }
    };

    const int nst = prod ? (K + CG_KT - 1) / CG_KT : 0;
    if (nst > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
    }
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) gload((s + 1) * CG_KT);
#pragma unroll 2
        for (int kk = 0; kk < CG_KT; kk += 2) {
            const int k = kk + half;
            float ar[BR], ai[BR], as[BR], br[BC], bi[BC], bs[BC];
#pragma unroll
            for (int x = 0; x < BR; ++x) {
                const float2 av = *reinterpret_cast<const float2*>(&As[buf][k][2 * (wi * BR * 32 + x * 32 + li)]);
                ar[x] = av.x;
                ai[x] = av.y;
                as[x] = av.x + av.y;
            }
#pragma unroll
            for (int y = 0; y < BC; ++y) {
                const float2 bv = Bs[buf][k][wj * BC * 32 + y * 32 + li];
                br[y] = bv.x;
                bi[y] = bv.y;
                bs[y] = bv.x + bv.y;
            }
#pragma unroll
            for (int x = 0; x < BR; ++x)
#pragma unroll
                for (int y = 0; y < BC; ++y) {
                    t1[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(br[y], ar[x], t1[x][y], 0, 0, 0);
                    t2[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(bi[y], ai[x], t2[x][y], 0, 0, 0);
                    t3[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(bs[y], as[x], t3[x][y], 0, 0, 0);
                }
        }
        if (s + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int x = 0; x < BR; ++x) {
        const int i = wrow + x * 32 + li;
        if (i >= M) continue;
#pragma unroll
        for (int y = 0; y < BC; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (j < N)
                    Cb[i + (long)j * ldc] = make_float2(os * (t1[x][y][r] - t2[x][y][r]),
                                                        os * (t3[x][y][r] - t1[x][y][r] - t2[x][y][r]));
            }
    }
}

// ----------------------------------------------------------------------------
// complex FP32 with at most 16 output columns (the solves of narrow probe
// blocks and the lowest levels of the panel recursion): v_mfma_f32_16x16x4f32,
// whose inner index of 4 covers two complex k in the 4M split k' = 2k + c
// (lane group g = lane / 16: complex k = k0 + g / 2, part c = g % 2).  A
// 32-wide instruction would leave three quarters of its columns empty at
// N = 8; this one leaves at most half.  With the operands swapped as in the
// kernels above, lane l and register r of a 16x16 block hold row l % 16 and
// column 4 (l / 16) + r.  Four waves of BR 16x16 blocks stacked in rows: the
// workgroup tile is (64 BR) x 16.
// ----------------------------------------------------------------------------
template <int BR, bool VEC, int TAG>
__global__ __launch_bounds__(CG_NT) void cgemm_narrow_kernel(
    int M, int N, int K, float alpha,
    const float2* __restrict__ A, int lda, long sA,
    const float2* __restrict__ B, int ldb, long sB,
    float beta, float2* __restrict__ C, int ldc, long sC,
    int tilesM, int batch, long total_padded)
{
    constexpr int BM = 64 * BR, BN = 16;
    constexpr int AQ = BM * CG_KT / 2 / CG_NT;   // float4 (2 complex) A loads per thread per stage
    constexpr int BLD = BN * CG_KT / 2;          // float4 B loads per stage (fewer than the threads)
    static_assert(AQ >= 1 && AQ * 2 * CG_NT == BM * CG_KT, "A tile must split evenly over the threads");
    static_assert(BLD <= CG_NT, "one B load per thread at most");
    __shared__ __attribute__((aligned(16))) float As[2][CG_KT][2 * BM];
    __shared__ __attribute__((aligned(16))) float2 Bs[2][CG_KT][BN + 4];

    const long tile = xcd_remap(blockIdx.x, total_padded);
    const long b = tile / tilesM;
    if (b >= batch) return;
    const int i0 = (int)(tile - b * tilesM) * BM;
    const float2* Ab = A + b * sA;
    const float2* Bb = B + b * sB;
    float2* Cb = C + b * sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int kc = g >> 1, part = g & 1;
    const int wrow = i0 + wave * BR * 16;

    const bool prod = alpha != 0.f;   // alpha applied once at the end, as in the kernels above
    const float cs = prod ? beta / alpha : beta, os = prod ? alpha : 1.f;
    floatx4 accR[BR], accI[BR];
#pragma unroll
    for (int x = 0; x < BR; ++x) {
        const int i = wrow + x * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 4 * g + r;
            float2 c = make_float2(0.f, 0.f);
            if (beta != 0.f && i < M && j < N) c = Cb[i + (long)j * ldc];
            accR[x][r] = cs * c.x;
            accI[x][r] = cs * c.y;
        }
    }

    floatx4 ra[AQ], rb;
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            const int gi = i0 + ip, gk = k0 + k;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gk < K) {
                const float2* src = Ab + gi + (long)gk * lda;
                if (VEC && gi + 1 < M) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gi < M) { float2 e = src[0]; v[0] = e.x; v[1] = e.y; }
                    if (gi + 1 < M) { float2 e = src[1]; v[2] = e.x; v[3] = e.y; }
                }
            }
            ra[q] = v;
        }
        rb = floatx4{0.f, 0.f, 0.f, 0.f};
        if (tid < BLD) {
            const int j = tid / (CG_KT / 2), kp = (tid % (CG_KT / 2)) * 2;
            const int gk = k0 + kp;
            if (j < N) {
                const float2* src = Bb + gk + (long)j * ldb;
                if (VEC && gk + 1 < K) {
                    rb = *reinterpret_cast<const floatx4*>(src);
                } else {
                    if (gk < K) { float2 e = src[0]; rb[0] = e.x; rb[1] = e.y; }
                    if (gk + 1 < K) { float2 e = src[1]; rb[2] = e.x; rb[3] = e.y; }
                }
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 2), ip = (p % (BM / 2)) * 2;
            *reinterpret_cast<floatx4*>(&As[buf][k][2 * ip]) = ra[q];
        }
        if (tid < BLD) {
            const int j = tid / (CG_KT / 2), kp = (tid % (CG_KT / 2)) * 2;
            Bs[buf][kp][j] = make_float2(rb[0], rb[1]);
            Bs[buf][kp + 1][j] = make_float2(rb[2], rb[3]);
        }
    };

    const int nst = prod ? (K + CG_KT - 1) / CG_KT : 0;
    if (nst > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
    }
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) gload((s + 1) * CG_KT);
#pragma unroll 4
        for (int kk = 0; kk < CG_KT; kk += 2) {
            const int k = kk + kc;
            float a[BR];
#pragma unroll
            for (int x = 0; x < BR; ++x) a[x] = As[buf][k][2 * (wave * BR * 16 + x * 16 + li) + part];
            const float2 bv = Bs[buf][k][li];
            const float br = part ? -bv.y : bv.x;
            const float bi = part ? bv.x : bv.y;
#pragma unroll
            for (int x = 0; x < BR; ++x) {
                accR[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(br, a[x], accR[x], 0, 0, 0);
                accI[x] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi, a[x], accI[x], 0, 0, 0);
            }
        }
        if (s + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int x = 0; x < BR; ++x) {
        const int i = wrow + x * 16 + li;
        if (i >= M) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 4 * g + r;
            if (j < N) Cb[i + (long)j * ldc] = make_float2(os * accR[x][r], os * accI[x][r]);
        }
    }
}

template <int WR, int WC, int BR, int BC, bool M3 = false>
static void cgemm_launch(hipStream_t st, int M, int N, int K, float alpha, const float2* A, int lda, long sA,
                         const float2* B, int ldb, long sB, float beta, float2* C, int ldc, long sC, int batch,
                         int tag, bool vec)
{
    constexpr int BM = 32 * WR * BR, BN = 32 * WC * BC;
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const long total = round_up_l((long)tm * tn * batch, 8);
#define CG_L(V, T)                                                                                                    \
    do {                                                                                                              \
        if constexpr (M3)                                                                                             \
            hipLaunchKernelGGL((cgemm3m_mfma_kernel<WR, WC, BR, BC, V, T>), dim3((unsigned)total), dim3(64 * WR * WC), \
                               0, st,                                                                                 \
                               M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tm, tn, batch, total);       \
        else                                                                                                          \
            hipLaunchKernelGGL((cgemm_mfma_kernel<WR, WC, BR, BC, V, T>), dim3((unsigned)total), dim3(CG_NT), 0, st,   \
                               M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tm, tn, batch, total);       \
    } while (0)
    if (vec) {
        if (tag == 1) CG_L(true, 1); else CG_L(true, 0);
    } else {
        if (tag == 1) CG_L(false, 1); else CG_L(false, 0);
    }
#undef CG_L
}

// Workgroup tile of the complex FP32 trailing update (tag 1), chosen per bucket
// by the ragged batch's autotuner and set around its launches (host thread).
namespace {
thread_local int g_update_tile = UPD_TILE_3M_128x64;
}
void set_update_tile(int t) { g_update_tile = (t >= 0 && t < UPD_TILE_COUNT) ? t : UPD_TILE_3M_128x64; }
int get_update_tile() { return g_update_tile; }
const char* update_tile_name(int t)
{
    switch (t) {
    case UPD_TILE_3M_64x64: return "3m_64x64_4waves";
    case UPD_TILE_4M_128x128: return "4m_128x128_4waves";
    case UPD_TILE_4M_64x64: return "4m_64x64_4waves";
    default: return "3m_128x64_4waves";
    }
}

hipError_t cgemm(hipStream_t st, int M, int N, int K, float alpha,
                 const float2* A, int lda, long sA, const float2* B, int ldb, long sB,
                 float beta, float2* C, int ldc, long sC, int batch, int tag)
{
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && (lda % 2 == 0) && (ldb % 2 == 0)
                     && (sA % 2 == 0) && (sB % 2 == 0);
    // 128x16 tiles of 16x16 blocks for at most 16 columns, 128x32 tiles in the
    // 4M form up to 32 columns (the narrow products of the panel recursion and
    // of narrow probe blocks); 64x64 tiles in the 3M form up to 64 columns (the
    // solves at L = 64); 128x64 tiles in the 3M form for everything wider (trailing
    // updates, U12 products): with two 32x32 blocks per wave the three
    // accumulator sets still leave two waves per SIMD, which measured faster
    // than 128x128 tiles in either form.  The trailing update's tile can be
    // changed per bucket by the ragged batch's autotuner (set_update_tile).
    if (N <= 16) {
        constexpr int BR = 2, BM = 64 * BR;
        const int tm = (M + BM - 1) / BM;
        const long total = round_up_l((long)tm * batch, 8);
#define CN_L(V, T)                                                                                                 \
    hipLaunchKernelGGL((cgemm_narrow_kernel<BR, V, T>), dim3((unsigned)total), dim3(CG_NT), 0, st, M, N, K, alpha, \
                       A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tm, batch, total)
        if (vec) {
            if (tag == 1) CN_L(true, 1); else CN_L(true, 0);
        } else {
            if (tag == 1) CN_L(false, 1); else CN_L(false, 0);
        }
#undef CN_L
    } else if (N <= 32) {
        cgemm_launch<4, 1, 1, 1>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    } else if (tag == 0 && N <= 64) {
        // 33..64 columns (the solves' products at L = 64): 64 x 64 tiles in the 3M form give
        // twice the workgroups of 128 x 64 on these skinny products (solve phase 25.8 -> 21.9 ms
        // per headline step; 64 x 32 and 32 x 64 tiles of two waves, 128 x 32 of four: slower)
        cgemm_launch<2, 2, 1, 1, true>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    } else if (tag == 1 && g_update_tile == UPD_TILE_3M_64x64) {
        cgemm_launch<2, 2, 1, 1, true>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    } else if (tag == 1 && g_update_tile == UPD_TILE_4M_128x128) {
        cgemm_launch<2, 2, 2, 2>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    } else if (tag == 1 && g_update_tile == UPD_TILE_4M_64x64) {
        cgemm_launch<2, 2, 1, 1>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    } else {
        cgemm_launch<4, 1, 1, 2, true>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// real FP32 (the LU of a real NEP at real points): v_mfma_f32_32x32x2f32 with
// the instruction's K = 2 over two consecutive k (lanes 0-31: k, lanes 32-63:
// k + 1).  Same wave/block shapes and output layout as the complex kernel.
// LDS rows are padded so that the staging stores and the two-row operand
// reads spread over the banks.
// ----------------------------------------------------------------------------
constexpr int SG_KT = 16;

template <int WR, int WC, int BR, int BC, bool VEC, int TAG>
__global__ __launch_bounds__(CG_NT, 2) void sgemm_mfma_kernel(
    int M, int N, int K, float alpha,
    const float* __restrict__ A, int lda, long sA,
    const float* __restrict__ B, int ldb, long sB,
    float beta, float* __restrict__ C, int ldc, long sC,
    int tilesM, int tilesN, int batch, long total_padded)
{
    constexpr int BM = 32 * WR * BR, BN = 32 * WC * BC;
    constexpr int AQ = BM * SG_KT / 4 / CG_NT;   // float4 (4 rows) A loads per thread per stage
    constexpr int BLD = BN * SG_KT / 4;            // float4 (4 k) B loads per stage
    constexpr int BQ = (BLD + CG_NT - 1) / CG_NT;  // ... per thread (the last round may be partial)
    static_assert(AQ >= 1 && AQ * 4 * CG_NT == BM * SG_KT, "A tile must split evenly over the threads");
    __shared__ __attribute__((aligned(16))) float As[2][SG_KT][BM + 32];
    __shared__ __attribute__((aligned(16))) float Bs[2][SG_KT][BN + 36];

    const long tile = xcd_remap(blockIdx.x, total_padded);
    const long per = (long)tilesM * tilesN;
    const long b = tile / per;
    if (b >= batch) return;
    const int t = (int)(tile - b * per);
    int ti, tj;
    tile_order(t, tilesM, tilesN, &ti, &tj);
    const int i0 = ti * BM;
    const int j0 = tj * BN;
    const float* Ab = A + b * sA;
    const float* Bb = B + b * sB;
    float* Cb = C + b * sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = wave % WR, wj = wave / WR;
    const int li = lane & 31, half = lane >> 5;
    const int wrow = i0 + wi * BR * 32, wcol = j0 + wj * BC * 32;

    floatx16 acc[BR][BC];
#pragma unroll
    for (int x = 0; x < BR; ++x)
#pragma unroll
        for (int y = 0; y < BC; ++y) {
            const int i = wrow + x * 32 + li;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                acc[x][y][r] = (beta != 0.f && i < M && j < N) ? beta * Cb[i + (long)j * ldc] : 0.f;
            }
        }

    floatx4 ra[AQ], rb[BQ];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 4), i4 = (p % (BM / 4)) * 4;
            const int gi = i0 + i4, gk = k0 + k;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gk < K) {
                const float* src = Ab + gi + (long)gk * lda;
                if (VEC && gi + 3 < M) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (gi + e < M) v[e] = src[e];
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + CG_NT * q;
            const int j = p / (SG_KT / 4), k4 = (p % (SG_KT / 4)) * 4;
            const int gj = j0 + j, gk = k0 + k4;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (p < BLD && j < BN && gj < N) {
                const float* src = Bb + gk + (long)gj * ldb;
                if (VEC && gk + 3 < K) {
                    v = *reinterpret_cast<const floatx4*>(src);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (gk + e < K) v[e] = src[e];
                }
            }
            rb[q] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int p = tid + CG_NT * q;
            const int k = p / (BM / 4), i4 = (p % (BM / 4)) * 4;
            *reinterpret_cast<floatx4*>(&As[buf][k][i4]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int p = tid + CG_NT * q;
            const int j = p / (SG_KT / 4), k4 = (p % (SG_KT / 4)) * 4;
            if (p < BLD) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[buf][k4 + e][j] = rb[q][e];
            }
        }
    };

    const int nst = (K + SG_KT - 1) / SG_KT;
    if (nst > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
    }
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) gload((s + 1) * SG_KT);
#pragma unroll 4
        for (int kp = 0; kp < SG_KT / 2; ++kp) {
            const int k = 2 * kp + half;
            float a[BR], bb[BC];
#pragma unroll
            for (int x = 0; x < BR; ++x) a[x] = alpha * As[buf][k][wi * BR * 32 + x * 32 + li];
#pragma unroll
            for (int y = 0; y < BC; ++y) bb[y] = Bs[buf][k][wj * BC * 32 + y * 32 + li];
#pragma unroll
            for (int x = 0; x < BR; ++x)
#pragma unroll
                for (int y = 0; y < BC; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(bb[y], a[x], acc[x][y], 0, 0, 0);
        }
        if (s + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int x = 0; x < BR; ++x) {
        const int i = wrow + x * 32 + li;
        if (i >= M) continue;
#pragma unroll
        for (int y = 0; y < BC; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wcol + y * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (j < N) Cb[i + (long)j * ldc] = acc[x][y][r];
            }
    }
}

template <int WR, int WC, int BR, int BC>
static void sgemm_launch(hipStream_t st, int M, int N, int K, float alpha, const float* A, int lda, long sA,
                         const float* B, int ldb, long sB, float beta, float* C, int ldc, long sC, int batch, int tag,
                         bool vec)
{
    constexpr int BM = 32 * WR * BR, BN = 32 * WC * BC;
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const long total = round_up_l((long)tm * tn * batch, 8);
#define SG_L(V, T)                                                                                                    \
    hipLaunchKernelGGL((sgemm_mfma_kernel<WR, WC, BR, BC, V, T>), dim3((unsigned)total), dim3(CG_NT), 0, st, M, N, K, \
                       alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tm, tn, batch, total)
    if (vec) {
        if (tag == 1) SG_L(true, 1); else SG_L(true, 0);
    } else {
        if (tag == 1) SG_L(false, 1); else SG_L(false, 0);
    }
#undef SG_L
}

hipError_t sgemm(hipStream_t st, int M, int N, int K, float alpha, const float* A, int lda, long sA,
                 const float* B, int ldb, long sB, float beta, float* C, int ldc, long sC, int batch, int tag)
{
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && (lda % 4 == 0) && (ldb % 4 == 0) &&
                     (sA % 4 == 0) && (sB % 4 == 0);
    if (N <= 32)
        sgemm_launch<4, 1, 1, 1>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    else if (N <= 64)
        sgemm_launch<4, 1, 1, 2>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    else
        sgemm_launch<2, 2, 2, 2>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, tag, vec);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// complex FP64: v_mfma_f64_16x16x4f64, WG tile 64x64, 4 waves of 32x32.
// op(A) = A or A^H, op(B) = B or B^H.
// ----------------------------------------------------------------------------
constexpr int ZG_BM = 64, ZG_BN = 64, ZG_KT = 16, ZG_NT = 256;

template <bool CA, bool CB, int TAG>
__global__ __launch_bounds__(ZG_NT, 2) void zgemm_mfma_kernel(
    int M, int N, int K, double alpha,
    const double2* __restrict__ A, int lda, long sA,
    const double2* __restrict__ B, int ldb, long sB,
    double beta, double2* __restrict__ C, int ldc, long sC,
    int tilesM, int tilesN, int batch, long total_padded)
{
    // rows padded by one complex (16 B) so that column-wise staging stores spread over the banks
    __shared__ __attribute__((aligned(16))) double2 As[2][ZG_KT][ZG_BM + 1];
    __shared__ __attribute__((aligned(16))) double2 Bs[2][ZG_KT][ZG_BN + 1];

    const long tile = xcd_remap(blockIdx.x, total_padded);
    const long per = (long)tilesM * tilesN;
    const long b = tile / per;
    if (b >= batch) return;
    const int t = (int)(tile - b * per);
    int ti, tj;
    tile_order(t, tilesM, tilesN, &ti, &tj);
    const int i0 = ti * ZG_BM;
    const int j0 = tj * ZG_BN;
    const double2* Ab = A + b * sA;
    const double2* Bb = B + b * sB;
    double2* Cb = C + b * sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = wave & 1, wj = wave >> 1;
    const int li = lane & 15, kq = lane >> 4;       // kq = 2*kc + part
    const int kc = kq >> 1, part = kq & 1;

    // acc = (beta / alpha) C, scaled by alpha once at the end (bitwise the same for
    // alpha = +-1); lane li holds row i, register r holds column lane/16 + 4*r
    // (the f64 MFMA interleaves its four output groups by register)
    const bool prod = alpha != 0.0;
    const double cs = prod ? beta / alpha : beta, os = prod ? alpha : 1.0;
    doublex4 accR[2][2], accI[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int i = i0 + wi * 32 + x * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + wj * 32 + y * 16 + kq + 4 * r;
                double2 c = make_double2(0.0, 0.0);
                if (beta != 0.0 && i < M && j < N) c = Cb[i + (long)j * ldc];
                accR[x][y][r] = cs * c.x;
                accI[x][y][r] = cs * c.y;
            }
        }

    // global tiles are fetched two K-tiles ahead into one of two register sets
    // (tile t into set t & 1), so a fetch has two tiles of matrix-core work to
    // arrive in before it is stored to LDS
    double2 ra0[4], rb0[4], ra1[4], rb1[4];
    auto gload = [&](int k0, double2 (&ra)[4], double2 (&rb)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int p = tid + ZG_NT * q;   // 0..1023
            double2 v = make_double2(0.0, 0.0);
            if (!CA) {
                int k = p >> 6, i = p & 63;
                int gi = i0 + i, gk = k0 + k;
                if (gi < M && gk < K) v = Ab[gi + (long)gk * lda];
            } else {
                int i = p >> 4, k = p & 15;
                int gi = i0 + i, gk = k0 + k;
                if (gi < M && gk < K) { v = Ab[gk + (long)gi * lda]; v.y = -v.y; }
            }
            ra[q] = v;
            double2 w = make_double2(0.0, 0.0);
            if (!CB) {
                int j = p >> 4, k = p & 15;
                int gj = j0 + j, gk = k0 + k;
                if (gj < N && gk < K) w = Bb[gk + (long)gj * ldb];
            } else {
                int k = p >> 6, j = p & 63;
                int gj = j0 + j, gk = k0 + k;
                if (gj < N && gk < K) { w = Bb[gj + (long)gk * ldb]; w.y = -w.y; }
            }
            rb[q] = w;
        }
    };
    auto sstore = [&](int buf, const double2 (&ra)[4], const double2 (&rb)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int p = tid + ZG_NT * q;
            if (!CA) As[buf][p >> 6][p & 63] = ra[q];
            else As[buf][p & 15][p >> 4] = ra[q];
            if (!CB) Bs[buf][p & 15][p >> 4] = rb[q];
            else Bs[buf][p >> 6][p & 63] = rb[q];
        }
    };
    auto compute = [&](int buf) {
#pragma unroll 2
        for (int kk = 0; kk < ZG_KT; kk += 2) {
            double a[2], br[2], bi[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                double2 av = As[buf][kk + kc][wi * 32 + x * 16 + li];
                a[x] = part ? av.y : av.x;
            }
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                double2 bv = Bs[buf][kk + kc][wj * 32 + y * 16 + li];
                br[y] = part ? -bv.y : bv.x;
                bi[y] = part ? bv.x : bv.y;
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[y], a[x], accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bi[y], a[x], accI[x][y], 0, 0, 0);
                }
        }
    };

    const int nst = prod ? (K + ZG_KT - 1) / ZG_KT : 0;
    if (nst > 0) {
        gload(0, ra0, rb0);
        sstore(0, ra0, rb0);
        if (nst > 1) gload(ZG_KT, ra1, rb1);
        __syncthreads();
    }
    // tiles in pairs so that the register set of every step is fixed at compile time
    for (int s = 0; s < nst; s += 2) {
        // even tile s: LDS buffer 0; tile s+1 waits in set 1, tile s+2 is fetched into set 0
        if (s + 2 < nst) gload((s + 2) * ZG_KT, ra0, rb0);
        compute(0);
        if (s + 1 < nst) sstore(1, ra1, rb1);
        __syncthreads();
        if (s + 1 >= nst) break;
        // odd tile s+1: LDS buffer 1; tile s+2 waits in set 0, tile s+3 is fetched into set 1
        if (s + 3 < nst) gload((s + 3) * ZG_KT, ra1, rb1);
        compute(1);
        if (s + 2 < nst) sstore(0, ra0, rb0);
        __syncthreads();
    }

    // epilogue: store
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const int i = i0 + wi * 32 + x * 16 + li;
        if (i >= M) continue;
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + wj * 32 + y * 16 + kq + 4 * r;
                if (j < N) Cb[i + (long)j * ldc] = make_double2(os * accR[x][y][r], os * accI[x][y][r]);
            }
    }
}

hipError_t zgemm(hipStream_t st, int opA, int opB, int M, int N, int K, double alpha,
                 const double2* A, int lda, long sA, const double2* B, int ldb, long sB,
                 double beta, double2* C, int ldc, long sC, int batch, int tag)
{
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const int tm = (M + ZG_BM - 1) / ZG_BM, tn = (N + ZG_BN - 1) / ZG_BN;
    const long total = round_up_l((long)tm * tn * batch, 8);
    dim3 g((unsigned)total), blk(ZG_NT);
#define ZG_LAUNCH(CA, CB)                                                                              \
    hipLaunchKernelGGL((zgemm_mfma_kernel<CA, CB, 0>), g, blk, 0, st, M, N, K, alpha, A, lda, sA, B,       \
                       ldb, sB, beta, C, ldc, sC, tm, tn, batch, total)
    if (tag == 1 && !opA && !opB)
        hipLaunchKernelGGL((zgemm_mfma_kernel<false, false, 1>), g, blk, 0, st, M, N, K, alpha, A, lda, sA, B,
                           ldb, sB, beta, C, ldc, sC, tm, tn, batch, total);
    else if (!opA && !opB) ZG_LAUNCH(false, false);
    else if (opA && !opB) ZG_LAUNCH(true, false);
    else if (!opA && opB) ZG_LAUNCH(false, true);
    else ZG_LAUNCH(true, true);
#undef ZG_LAUNCH
    return hipGetLastError();
}

}  // namespace rsrr
