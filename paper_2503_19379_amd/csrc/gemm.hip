// Matrix-core (MFMA) kernels of the Rayleigh-Ritz step of the block
// eigensolver (Section 5.1): the Gram products of the basis S = [X W P] and the
// block update with the Ritz coefficients.  FP64, v_mfma_f64_16x16x4f64.
//
// Operand layouts of the 16x16x4 FP64 MFMA (lane l of a 64-wide wave):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 r][l % 16], r = 0..3
// Complex products use three real products per 16x16x4 step:
//   conj(s) t : re = sr tr + si ti,  im = (sr - si)(tr + ti) - sr tr + si ti
//   s c       : re = sr cr - si ci,  im = (sr + si)(cr + ci) - sr cr - si ci
#include "common.h"
#include "solver.h"

#include <type_traits>

namespace mfd {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Gram: for the K basis columns S (K = mb + 2 na under soft locking, at most
// 3 mb; the column map gives their places in V) and their images AS,
//   G_S = S^H S, G_A = S^H AS (both Hermitian: only the 16x16 tiles of one
//   triangle are formed; gram_scatter_kernel mirrors them).
// Workgroup w sums rows [w rows_per, (w+1) rows_per) into its own partial
// tile set; reduce_parts_kernel adds the partials in a fixed order.
// ---------------------------------------------------------------------------
constexpr int GM_PF = 8;        // prefetch registers (complex) per thread

struct GramTiles {
    int n;                      // number of tiles
    short ti[80], tj[80];       // tile row (of G_S / G_A, 16 units) and column
    unsigned char half[80];     // 0: G_S, 1: G_A
};

// In mixed precision the W, P, AW, AP columns (basis columns [mb, 3mb) and
// [4mb, 6mb)) are stored in FP32 (V32, same column positions) and promoted on
// load; X and AX stay FP64.
__device__ __forceinline__ bool col_is_f32(int c, int mb) { return (c >= mb && c < 3 * mb) || c >= 4 * mb; }

// Prefetches keep the raw bits (an FP32 pair in .x) so that no conversion
// waits on a load in flight; widen() promotes when the slab is written.
__device__ __forceinline__ double2 widen(double2 raw, bool f32) {
    if (!f32) return raw;
    const float2 v = __builtin_bit_cast(float2, raw.x);
    return mk<double2>((double)v.x, (double)v.y);
}

// One wave per 16-column block g of S.  Block g is the A operand of exactly
// T + 1 tiles (T = ceil(K / 16)): the G_S tiles (g, b), b >= g, and the G_A
// tiles (g, a), a <= g, so the wave loads its A fragment once per 4 rows and
// reuses it for all of them.  Two LDS slabs alternate: the next slab is
// loaded into registers and written to the free slab while the current one is
// consumed by the matrix cores, with one barrier per slab.  The two waves of a
// block (alternate 4-row steps) add their tiles through LDS at the end, so a
// workgroup writes one partial tile set.
// SUBS waves per block of S take alternate 4-row steps of a slab of KS rows
// (two for T <= 4; one for T = 5, whose accumulators would not fit beside a
// second wave's registers); KS rows per slab.
template <int T, int SUBS = 2, int GM_KS = 32>
__global__ __launch_bounds__(64 * SUBS * T) void gram_mfma_kernel(const double2* __restrict__ V,
                                                                   const float2* __restrict__ V32, size_t ld,
                                                                   size_t n, BasisMap bm, size_t rows_per,
                                                                   double2* __restrict__ part) {
    constexpr int NT = 64 * SUBS * T;   // SUBS waves per block of S, each taking every SUBS-th 4 rows
    constexpr int TG = T + 1;     // tiles per wave
    extern __shared__ unsigned char smem_raw[];
    double2* slabs = reinterpret_cast<double2*>(smem_raw);   // [2][GM_KS][2K + 1]
    const int K = bm.K;
    const int C2 = 2 * K;
    // slab rows are 2K + 1 elements apart: the fill writes one column of 32
    // consecutive rows per instruction, and with a stride of 2K elements
    // (8K dwords, a multiple of 16) those rows would share four or eight of
    // the 32 LDS banks
    const int RS = C2 + 1;
    const int SL = GM_KS * RS;
    const int tid = threadIdx.x;
    const int lane = tid & 63, g = (tid >> 6) / SUBS, sub = (tid >> 6) % SUBS;
    const size_t r0 = (size_t)blockIdx.x * rows_per;
    const size_t r1 = min(n, r0 + rows_per);
    d4 acc[TG][3];
#pragma unroll
    for (int t = 0; t < TG; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[t][q] = d4{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    // A operand: column 16 g + li of S; B operands: S columns 16 b + li (b = g..T-1),
    // then AS columns 16 a + li (a = 0..g)
    const int ia = 16 * g + li;
    const bool va = ia < K;
    int ob[TG];
    bool vb[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        const int j = (t < T - g) ? 16 * (g + t) + li : 16 * (t - (T - g)) + li;
        const bool as = t >= T - g;
        vb[t] = j < K;
        ob[t] = vb[t] ? (as ? K + j : j) : 0;
    }
    // element tid + q NT of a slab: row tid % GM_KS and load ordinal
    // tid / GM_KS + q NT / GM_KS, the same in every slab: resolve the columns once
    const int srow = tid % GM_KS;
    int scol[GM_PF], vcol[GM_PF];
    unsigned f32m = 0, okm = 0;
#pragma unroll
    for (int q = 0; q < GM_PF; ++q) {
        const int o = tid / GM_KS + q * (NT / GM_KS);
        scol[q] = vcol[q] = 0;
        if (o < C2) {
            scol[q] = bm.lc[o];
            vcol[q] = bm.pc[o];
            okm |= 1u << q;
            if (V32 && col_is_f32(vcol[q], bm.mb)) f32m |= 1u << q;
        }
    }
    // FP32 and FP64 columns prefetch into separate registers, and rows past
    // the end are clamped to the last row and zeroed when the slab is
    // written, so that the loads are the only writes to these registers: a
    // wave may hold both kinds, and a register written on one side of the
    // exec-masked branch while the other side's load is in flight makes the
    // compiler drain every load before it
    double2 pf[GM_PF];
    float2 pf32[GM_PF];
    auto prefetch = [&](size_t s0) {
        const size_t row = min(s0 + srow, r1 - 1);
        // nothing is in flight here (the previous slab's registers were
        // written to LDS), but the compiler's wait tracking does not see it
        // through the exec-masked branches below and would otherwise drain
        // the loads one q at a time: vmcnt(0), the other counters left open
        __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
        for (int q = 0; q < GM_PF; ++q) {
            if ((okm >> q) & 1u) {
                const size_t o = (size_t)vcol[q] * ld + row;
                if ((f32m >> q) & 1u) pf32[q] = V32[o];
                else pf[q] = V[o];
            }
        }
    };
    // the registers are read on every lane, outside the branch on the
    // ordinal, so that the wait for the loads is not conditional either
    auto fill = [&](double2* slab, size_t s0) {
        const bool inb = s0 + srow < r1;
#pragma unroll
        for (int q = 0; q < GM_PF; ++q) {
            double2 v = ((f32m >> q) & 1u) ? mk<double2>((double)pf32[q].x, (double)pf32[q].y) : pf[q];
            if (!inb) v = mk<double2>(0.0, 0.0);
            if ((okm >> q) & 1u) slab[srow * RS + scol[q]] = v;
        }
    };
    prefetch(r0);
    fill(slabs, r0);
    __syncthreads();
    int buf = 0;
    for (size_t s0 = r0; s0 < r1; s0 += GM_KS) {
        const bool more = s0 + GM_KS < r1;
        if (more) prefetch(s0 + GM_KS);
        const double2* slab = slabs + buf * SL;
#pragma unroll
        for (int k0 = 4 * sub; k0 < GM_KS; k0 += 4 * SUBS) {
            const double2* srow_p = slab + (k0 + lk) * RS;
            // every fragment of the step is read before the first product, so
            // that one LDS round trip, not one per tile, precedes the matrix
            // work (T = 5 has no registers to spare for it)
            constexpr bool ALLB = T <= 4;
            const double2 a = va ? srow_p[ia] : mk<double2>(0.0, 0.0);
            double2 bt[TG];
            if constexpr (ALLB) {
#pragma unroll
                for (int t = 0; t < TG; ++t) bt[t] = vb[t] ? srow_p[ob[t]] : mk<double2>(0.0, 0.0);
            }
            const double amd = a.x - a.y;
#pragma unroll
            for (int t = 0; t < TG; ++t) {
                const double2 b = ALLB ? bt[t] : (vb[t] ? srow_p[ob[t]] : mk<double2>(0.0, 0.0));
                acc[t][0] = mfma64(a.x, b.x, acc[t][0]);
                acc[t][1] = mfma64(a.y, b.y, acc[t][1]);
                acc[t][2] = mfma64(amd, b.x + b.y, acc[t][2]);
            }
        }
        // the free slab was last read before the previous barrier.  After
        // the last slab this writes stale registers into it, which nothing
        // reads; filling unconditionally keeps the wait for the prefetch on
        // every path, so no load appears in flight at the top of the loop
        fill(slabs + (buf ^ 1) * SL, s0 + GM_KS);
        __syncthreads();
        buf ^= 1;
    }
    // sub 1 hands its tiles to sub 0 through LDS (the slabs are free after the
    // last barrier); partial tiles part[w][tile][16][16], tiles of block g at g TG .. g TG + T
    double2* xch = slabs;   // [T TG][4][64]
    if (SUBS == 2 && sub == 1) {
#pragma unroll
        for (int t = 0; t < TG; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double t1 = acc[t][0][r], t2 = acc[t][1][r], t3 = acc[t][2][r];
                xch[((g * TG + t) * 4 + r) * 64 + lane] = mk<double2>(t1 + t2, t3 - t1 + t2);
            }
    }
    __syncthreads();
    if (sub == 0) {
        double2* out = part + (size_t)blockIdx.x * (T * TG) * 256;
#pragma unroll
        for (int t = 0; t < TG; ++t) {
            const int ti = g * TG + t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double t1 = acc[t][0][r], t2 = acc[t][1][r], t3 = acc[t][2][r];
                const double2 o = SUBS == 2 ? xch[((g * TG + t) * 4 + r) * 64 + lane] : mk<double2>(0.0, 0.0);
                out[(size_t)ti * 256 + (lk + 4 * r) * 16 + li] = mk<double2>(t1 + t2 + o.x, t3 - t1 + t2 + o.y);
            }
        }
    }
}

// G (K x 2K row-major) from the summed tiles.  G_S is formed from its upper
// tiles, G_A from its lower tiles, and each is completed by the Hermitian
// mirror.  With X first in the basis, every entry of G_A that pairs an X
// column with a W or P column is then the product with AX (W^H AX), never the
// product with AW or AP: in mixed precision AX is the FP64 one, while AW and AP
// carry the FP32 rounding of the operator.
__global__ void gram_scatter_kernel(const double2* __restrict__ sum, int K, GramTiles tl, double2* __restrict__ G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tl.n * 256) return;
    const int t = e / 256, rc = e % 256;
    const double2 v = sum[e];
    const int i = tl.ti[t] * 16 + rc / 16, j = tl.tj[t] * 16 + rc % 16;
    if (i >= K || j >= K) return;
    const int h = tl.half[t];
    const int off = h * K;
    const bool direct = h == 0 ? (i <= j) : (i >= j);
    const bool mirror = h == 0 ? (i < j) : (i > j);
    if (direct) G[(size_t)i * 2 * K + off + j] = v;
    if (mirror) G[(size_t)j * 2 * K + off + i] = mk<double2>(v.x, -v.y);
}

// Tiles in the order the waves produce them: for block g of S, the G_S tiles
// (g, b), b >= g, then the G_A tiles (g, a), a <= g.
static GramTiles make_tiles(int K) {
    GramTiles tl;
    tl.n = 0;
    const int T = (K + 15) / 16;
    for (int g = 0; g < T; ++g) {
        for (int b = g; b < T; ++b) {
            tl.ti[tl.n] = (short)g;
            tl.tj[tl.n] = (short)b;
            tl.half[tl.n] = 0;
            ++tl.n;
        }
        for (int a = 0; a <= g; ++a) {
            tl.ti[tl.n] = (short)g;
            tl.tj[tl.n] = (short)a;
            tl.half[tl.n] = 1;
            ++tl.n;
        }
    }
    return tl;
}

int gram_mfma_parts(size_t n) { return (int)std::min<size_t>(512, (n + 1023) / 1024); }

size_t gram_mfma_part_elems(int K, int nparts) {
    const int T = (K + 15) / 16;
    return (size_t)(nparts + 1) * T * (T + 1) * 256;   // one partial set per workgroup + their sum
}

// rows per slab of the instance for T column blocks
template <int T> constexpr int gram_ks() { return T == 5 ? 16 : 32; }
template <int T> constexpr int gram_subs() { return T == 5 ? 1 : 2; }

template <int T>
static hipError_t gram_t(const void* V, const void* V32, size_t ld, size_t n, const BasisMap& bm, int nw,
                         size_t rows_per, void* part, hipStream_t s) {
    constexpr int KS = gram_ks<T>(), SUBS = gram_subs<T>();
    // the slab of KS x 2K elements must fit the prefetch registers of the workgroup
    if (KS * 2 * bm.K > GM_PF * 64 * SUBS * T) return hipErrorInvalidValue;
    // two slabs (rows of 2K + 1), or the tile exchange between the two waves of a block at the end if larger
    const size_t lds = std::max((size_t)2 * KS * (2 * bm.K + 1), SUBS == 2 ? (size_t)T * (T + 1) * 4 * 64 : (size_t)0) *
                       sizeof(double2);
    auto kern = gram_mfma_kernel<T, SUBS, KS>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nw), dim3(64 * SUBS * T), lds, s, (const double2*)V, (const float2*)V32, ld, n,
                       bm, rows_per, (double2*)part);
    return hipGetLastError();
}

hipError_t launch_gram_mfma(const void* V, const void* V32, size_t ld, size_t n, const BasisMap& bm, int nparts,
                            void* part, void* G, hipStream_t s, int stages) {
    const int K = bm.K;
    if (K < 1 || K > BASIS_KMAX) return hipErrorInvalidValue;
    const int T = (K + 15) / 16;
    GramTiles tl = make_tiles(K);
    // rows per workgroup: a multiple of 32, hence of every instance's slab
    const size_t rows_per = ((n + nparts - 1) / nparts + 31) / 32 * 32;
    const int nw = (int)((n + rows_per - 1) / rows_per);
    hipError_t e = hipSuccess;
    if (stages & 1) {
        switch (T) {
            case 1: e = gram_t<1>(V, V32, ld, n, bm, nw, rows_per, part, s); break;
            case 2: e = gram_t<2>(V, V32, ld, n, bm, nw, rows_per, part, s); break;
            case 3: e = gram_t<3>(V, V32, ld, n, bm, nw, rows_per, part, s); break;
            case 4: e = gram_t<4>(V, V32, ld, n, bm, nw, rows_per, part, s); break;
            default: e = gram_t<5>(V, V32, ld, n, bm, nw, rows_per, part, s); break;
        }
    }
    if (e != hipSuccess || !(stages & 2)) return e;
    // sum the nw partial tile sets (into the slot after the last), then scatter
    double2* sum = (double2*)part + (size_t)nw * tl.n * 256;
    if ((e = launch_reduce((const double*)part, nw, tl.n * 256 * 2, (double*)sum, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(gram_scatter_kernel, dim3((tl.n * 256 + 255) / 256), dim3(256), 0, s, (const double2*)sum, K, tl,
                       (double2*)G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Update with the Ritz coefficients C (K x mb, row-major), K = 3mb:
//   P' = [W P] C[mb:],  X' = P' + X C[:mb]  (and the same for AP', AX'),
//   R' = AX' - X' diag(theta),  column sums of |R'|^2 and |X'|^2.
// Output U = [X' | R' | P' | AX' | - | AP'].  Each wave owns 16-row strips;
// the coefficients sit in LDS as MFMA B fragments.
// ---------------------------------------------------------------------------
// RB rows per block (16 or 32): RB / 16 strips of 16 rows, one wave per
// (strip, chain), 128 RB / 16 threads; the LDS blocks have column stride RB + 1
// (conflict-free fragment reads).  The 16-row form needs about half the LDS,
// so two workgroups can share a CU.
constexpr int UP_PF = 16;       // prefetch registers (complex) per thread

// Wave w computes rows 16 (w % NS) .. of the block for chain w / NS (0: S ->
// P', X'; 1: AS -> AP', AX').  X' and AX' meet in LDS, where R' = AX' - X' theta
// and the column norms are formed and written out row-contiguously.
template <int MJ, int RB>   // mb <= 16 MJ
__global__ __launch_bounds__(8 * RB) void update_mfma_kernel(const double2* __restrict__ V,
                                                             const float2* __restrict__ V32,
                                                             double2* __restrict__ U, float2* __restrict__ U32,
                                                             size_t ld, size_t n, BasisMap bm,
                                                             const double2* __restrict__ Cg,
                                                             const double* __restrict__ theta,
                                                             double* __restrict__ npart) {
    constexpr int MP = 16 * MJ;
    constexpr int NS = RB / 16;          // strips
    constexpr int NTH = 128 * NS;        // threads
    constexpr int UP_RB = RB;
    constexpr int UP_RBP = RB + 1;
    extern __shared__ unsigned char smem_raw[];
    const int mb = bm.mb;
    const int K = bm.K;
    const int KP = (K + 3) / 4 * 4;
    const int C2 = 2 * K;
    double2* Cs = reinterpret_cast<double2*>(smem_raw);      // [KP][mb]
    double2* slab = Cs + KP * mb;                             // [C2][UP_RBP], column-major
    double2* xo = slab + C2 * UP_RBP;                         // [2][mb][UP_RBP]: X', AX'
    double2* po = xo + 2 * mb * UP_RBP;                       // [2][mb][UP_RBP]: P', AP'
    double* red = reinterpret_cast<double*>(po + 2 * mb * UP_RBP);   // [8][2][MP]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int strip = wave % NS, chain = wave / NS;
    for (int e = tid; e < KP * mb; e += NTH) {
        const int k = e / mb;
        Cs[e] = (k < K) ? Cg[e] : mk<double2>(0.0, 0.0);
    }
    const int li = lane & 15, lk = lane >> 4;
    // R phase mapping: row = tid % RB, columns jg, jg + 8, ... (NTH / RB = 8 groups)
    const int rrow = tid % RB, jg = tid / RB;
    constexpr int NJ = MP / 8;
    double th[NJ], nr[NJ], nx[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        const int j = jg + 8 * c;
        th[c] = (j < mb) ? theta[j] : 0.0;
        nr[c] = nx[c] = 0.0;
    }
    const int nel = UP_RB * C2;
    const size_t nblk = (n + UP_RB - 1) / UP_RB;
    // element tid + NTH q of a block: row tid % UP_RB and load ordinal
    // tid / UP_RB + q NTH / UP_RB, the same in every block: resolve the columns once
    const int srow = tid % UP_RB;
    int scol[UP_PF], vcol[UP_PF];
    unsigned f32m = 0, okm = 0;
#pragma unroll
    for (int q = 0; q < UP_PF; ++q) {
        const int o = tid / UP_RB + q * (NTH / UP_RB);
        scol[q] = vcol[q] = 0;
        if (o < C2) {
            scol[q] = bm.lc[o];
            vcol[q] = bm.pc[o];
            okm |= 1u << q;
            if (V32 && col_is_f32(vcol[q], mb)) f32m |= 1u << q;
        }
    }
    (void)nel;
    double2 pf[UP_PF];
    auto prefetch = [&](size_t blk) {
        const size_t row = blk * UP_RB + srow;
        const bool inb = blk < nblk && row < n;
#pragma unroll
        for (int q = 0; q < UP_PF; ++q) {
            pf[q] = mk<double2>(0.0, 0.0);
            if (((okm >> q) & 1u) && inb) {
                const size_t o = (size_t)vcol[q] * ld + row;
                if ((f32m >> q) & 1u) pf[q].x = __builtin_bit_cast(double, V32[o]);
                else pf[q] = V[o];
            }
        }
    };
    prefetch(blockIdx.x);
    for (size_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const size_t b0 = blk * UP_RB;
#pragma unroll
        for (int q = 0; q < UP_PF; ++q)
            if ((okm >> q) & 1u) slab[scol[q] * UP_RBP + srow] = widen(pf[q], (f32m >> q) & 1u);
        __syncthreads();
        prefetch(blk + gridDim.x);
        d4 acc[MJ][3];
#pragma unroll
        for (int J = 0; J < MJ; ++J)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[J][q] = d4{0.0, 0.0, 0.0, 0.0};
        const double2* arow = slab + (size_t)chain * K * UP_RBP + 16 * strip + li;   // A fragment: row of this lane
        for (int pass = 0; pass < 2; ++pass) {
            const int kb = pass == 0 ? mb : 0;
            const int ke = pass == 0 ? K : mb;
            for (int k0 = kb; k0 < ke; k0 += 4) {
                const int k = k0 + lk;
                const double2 sv = (k < ke) ? arow[k * UP_RBP] : mk<double2>(0.0, 0.0);
#pragma unroll
                for (int J = 0; J < MJ; ++J) {
                    const double2 c = (k < ke && 16 * J + li < mb) ? Cs[k * mb + 16 * J + li] : mk<double2>(0.0, 0.0);
                    acc[J][0] = mfma64(sv.x, c.x, acc[J][0]);
                    acc[J][1] = mfma64(sv.y, c.y, acc[J][1]);
                    acc[J][2] = mfma64(sv.x + sv.y, c.x + c.y, acc[J][2]);
                }
            }
#pragma unroll
            for (int J = 0; J < MJ; ++J) {
                const int j = 16 * J + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rl = 16 * strip + lk + 4 * r;
                    const double t1 = acc[J][0][r], t2 = acc[J][1][r], t3 = acc[J][2][r];
                    const double2 v = mk<double2>(t1 - t2, t3 - t1 - t2);
                    if (j >= mb) continue;
                    if (pass == 0) po[(chain * mb + j) * UP_RBP + rl] = v;   // P' (AP'), stored with X' below
                    else xo[(chain * mb + j) * UP_RBP + rl] = v;
                }
            }
        }
        __syncthreads();
        // R' = AX' - X' theta; write X', AX', R' row-contiguously; column norms
        const size_t row = b0 + rrow;
        if (row < n) {
#pragma unroll
            for (int c = 0; c < NJ; ++c) {
                const int j = jg + 8 * c;
                if (j < mb) {
                    const double2 x = xo[j * UP_RBP + rrow];
                    const double2 ax = xo[(mb + j) * UP_RBP + rrow];
                    const double2 res = mk<double2>(ax.x - th[c] * x.x, ax.y - th[c] * x.y);
                    U[(size_t)j * ld + row] = x;
                    U[(size_t)(3 * mb + j) * ld + row] = ax;
                    if (U32) U32[(size_t)(mb + j) * ld + row] = make_float2((float)res.x, (float)res.y);
                    else U[(size_t)(mb + j) * ld + row] = res;
                    nr[c] += cabs2(res);
                    nx[c] += cabs2(x);
                }
            }
            // P', AP' of every band
#pragma unroll
            for (int c = 0; c < NJ; ++c) {
                const int j = jg + 8 * c;
                if (j < mb) {
                    const double2 pn = po[j * UP_RBP + rrow];
                    const double2 apn = po[(mb + j) * UP_RBP + rrow];
                    if (U32) {
                        U32[(size_t)(2 * mb + j) * ld + row] = make_float2((float)pn.x, (float)pn.y);
                        U32[(size_t)(5 * mb + j) * ld + row] = make_float2((float)apn.x, (float)apn.y);
                    } else {
                        U[(size_t)(2 * mb + j) * ld + row] = pn;
                        U[(size_t)(5 * mb + j) * ld + row] = apn;
                    }
                }
            }
        }
        __syncthreads();
    }
    // column sums over the RB threads of each column group
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        double a = nr[c], b = nx[c];
        for (int o = RB / 2; o > 0; o >>= 1) {
            a += __shfl_down(a, o, RB);
            b += __shfl_down(b, o, RB);
        }
        if (rrow == 0) {
            red[(c * 8 + jg) * 2 + 0] = a;
            red[(c * 8 + jg) * 2 + 1] = b;
        }
    }
    __syncthreads();
    if (tid < 2 * mb) {
        const int which = tid / mb, j = tid % mb;
        const int c = j / 8, g = j % 8;
        npart[(size_t)blockIdx.x * 2 * mb + tid] = red[(c * 8 + g) * 2 + which];
    }
}

template <int MJ, int RB>
static hipError_t update_mj(const void* V, const void* V32, void* U, void* U32, size_t ld, size_t n,
                            const BasisMap& bm, const void* C, const double* theta, int nparts, double* npart,
                            hipStream_t s) {
    constexpr int MP = 16 * MJ;
    constexpr int NTH = 8 * RB;
    const int K = bm.K;
    const int KP = (K + 3) / 4 * 4;
    if (RB * 2 * K > UP_PF * NTH) return hipErrorInvalidValue;
    const int mb = bm.mb;
    const size_t lds = ((size_t)KP * mb + (size_t)(RB + 1) * 2 * K + 4 * (size_t)(RB + 1) * mb) * sizeof(double2) +
                       (size_t)8 * 2 * MP * sizeof(double);
    auto kern = update_mfma_kernel<MJ, RB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nparts), dim3(NTH), lds, s, (const double2*)V, (const float2*)V32, (double2*)U,
                       (float2*)U32, ld, n, bm, (const double2*)C, theta, npart);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The same update with one wave per 16-row strip and no LDS staging of S.
// The product runs transposed, U^T = C^T S^T: the A operand is the first 16
// columns of C^T (LDS), the B operand 4 basis columns x 16 rows of S, loaded
// from HBM straight into registers.  The accumulator tile then holds output
// column lk + 4 r, row li in lane (li, lk), so every store writes 16
// consecutive rows (256 bytes in FP64) of 4 columns, and X' and AX' of a row
// meet in the same lane: R' and the column norms need no exchange.
// Bands 16 .. mb-1 (at most NT of them) would fill a second 16-column tile
// mostly with zeros; they run instead as FP64 vector FMAs on the fragments
// already in registers (lane (li, lk) adds its own basis columns for row li)
// and are summed over the 4 lanes of a row with two shuffles.
// A wave runs the S chain (P', then X') and the AS chain (AP', then AX') of its
// strip; waves share only C, theta and the column map, so no barrier stands
// between strips and the other waves of the SIMD cover a wave's load latency.
// KS0 and KS1 are the k-steps of the two passes (4 basis columns each), at
// least ceil((K - mb) / 4) over the W and P columns and ceil(mb / 4) over X;
// steps past the basis run on zero fragments, so the code has no branch
// between the loads and the matrix products.
// ---------------------------------------------------------------------------
template <int KS0, int KS1, int NT, bool MIX>
__global__ __launch_bounds__(256, 2) void update_wave_kernel(const double2* __restrict__ V,
                                                             const float2* __restrict__ V32,
                                                             double2* __restrict__ U, float2* __restrict__ U32,
                                                             size_t ld, size_t n, BasisMap bm,
                                                             const double2* __restrict__ Cg,
                                                             const double* __restrict__ theta,
                                                             double* __restrict__ npart) {
    constexpr int CW = 16 + ((NT + 1) & ~1);   // columns of C kept in LDS (zero past mb); even, so
                                               // the double2 arrays after th and red stay 16-byte aligned
    constexpr int NX = 4 + NT;                 // X' slots per lane
    // in mixed precision the pass over W and P (AW and AP) reads FP32 columns, the pass over X (AX) FP64
    using T0 = typename std::conditional<MIX, float2, double2>::type;
    extern __shared__ unsigned char smem_raw[];
    const int mb = bm.mb;
    const int K = bm.K;
    const int KR = max(mb + 4 * KS0, 4 * KS1);                // rows of Cs the two passes read
    double2* Cs = reinterpret_cast<double2*>(smem_raw);       // [KR][CW], zero outside K x mb
    double* th = reinterpret_cast<double*>(Cs + (size_t)KR * CW);   // [CW]
    double* red = th + CW;                                    // [4 waves][2][CW]
    double2* xw = reinterpret_cast<double2*>(red + 8 * CW);   // [4 waves][NX][64 lanes]: X' of the S chain
    int* vmap = reinterpret_cast<int*>(xw + 4 * NX * 64);     // [2K]: basis column -> V column
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int e = tid; e < KR * CW; e += 256) {
        const int k = e / CW, j = e % CW;
        Cs[e] = (k < K && j < mb) ? Cg[(size_t)k * mb + j] : mk<double2>(0.0, 0.0);
    }
    for (int q = tid; q < 2 * K; q += 256) vmap[bm.lc[q]] = bm.pc[q];
    for (int j = tid; j < CW; j += 256) th[j] = j < mb ? theta[j] : 0.0;
    for (int e = tid; e < 8 * CW; e += 256) red[e] = 0.0;
    __syncthreads();
    double* wred = red + wave * 2 * CW;   // this wave's running sums of |R'|^2 and |X'|^2 per column
    double2* xs = xw + (size_t)wave * NX * 64 + lane;   // this lane's X' slots, stride 64
    const size_t nstrip = (n + 15) / 16;
    const size_t nwaves = (size_t)gridDim.x * 4;
    // sum over the 4 lanes of a row (lk = 0..3), result in all of them
    auto rowsum = [](double v) {
        v += __shfl_xor(v, 16);
        return v + __shfl_xor(v, 32);
    };
    // B fragments of one chain of one strip, lane (li, lk): pass 0
    // S[row][mb + 4 s + lk], pass 1 S[row][4 s + lk]; okm flags the lanes and
    // steps that hold a basis column of a row < n
    struct Frag {
        T0 f0[KS0];
        double2 f1[KS1];
        unsigned okm;
    };
    auto load = [&](Frag& F, size_t st, int ch) {   // issued, not waited for
        const size_t row = st * 16 + li;
        const bool rok = row < n;
        const size_t rowc = rok ? row : n - 1;   // masked lanes load a valid element and discard it
        F.okm = 0;
#pragma unroll
        for (int s = 0; s < KS0; ++s) {
            const int kk = mb + 4 * s + lk;
            const size_t o = (size_t)vmap[ch * K + min(kk, K - 1)] * ld + rowc;
            if constexpr (MIX) F.f0[s] = V32[o];
            else F.f0[s] = V[o];
            F.okm |= (unsigned)(rok && kk < K) << s;
        }
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            const int kk = 4 * s + lk;
            F.f1[s] = V[(size_t)(ch * 3 * mb + min(kk, mb - 1)) * ld + rowc];   // X and AX are never permuted
            F.okm |= (unsigned)(rok && kk < mb) << (KS0 + s);
        }
    };
    // one chain of one strip: ch 0 (S) writes P' and keeps X' in LDS, ch 1 (AS)
    // writes AP', then X', AX', R' and adds the column norms
    auto chain = [&](const Frag& F, size_t st, int ch) {
        const size_t row = st * 16 + li;
        const bool rok = row < n;
        d4 acc[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
        double tre[NT > 0 ? NT : 1], tim[NT > 0 ? NT : 1];   // tail bands: this lane's partial sums
#pragma unroll
        for (int c = 0; c < NT; ++c) tre[c] = tim[c] = 0.0;
        // C is the same for every strip; an opaque zero offset keeps its LDS
        // reads here rather than hoisted into registers for the whole kernel
        int zo;
        asm volatile("s_mov_b32 %0, 0" : "=s"(zo));
        const double2* Cz = Cs + zo;
        auto step = [&](double br, double bi, int kr) {
            // keep each step's LDS reads in place: hoisted together they
            // would hold every step's C values in registers at once
            __builtin_amdgcn_sched_barrier(0);
            const double2 a = Cz[kr * CW + li];
            acc[0] = mfma64(a.x, br, acc[0]);
            acc[1] = mfma64(a.y, bi, acc[1]);
            acc[2] = mfma64(a.x + a.y, br + bi, acc[2]);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const double2 t = Cz[kr * CW + 16 + c];
                tre[c] = fma(br, t.x, fma(-bi, t.y, tre[c]));
                tim[c] = fma(br, t.y, fma(bi, t.x, tim[c]));
                // the sums are due here: deferred to their use, the FMAs
                // would keep every step's C values live (no instruction)
                asm volatile("" : "+v"(tre[c]), "+v"(tim[c]));
            }
        };
#pragma unroll
        for (int s = 0; s < KS0; ++s) {
            const bool ok = (F.okm >> s) & 1u;
            step(ok ? (double)F.f0[s].x : 0.0, ok ? (double)F.f0[s].y : 0.0, mb + 4 * s + lk);
        }
        // P' (S chain) or AP' (AS chain) of every band
        auto put = [&](int j, double re, double im) {   // column (ch ? 5 : 2) mb + j, row
            const size_t o = (size_t)((ch ? 5 : 2) * mb + j) * ld + row;
            if constexpr (MIX) U32[o] = make_float2((float)re, (float)im);
            else U[o] = mk<double2>(re, im);
        };
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = lk + 4 * r;
            if (rok && j < mb) put(j, acc[0][r] - acc[1][r], acc[2][r] - acc[0][r] - acc[1][r]);
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const double re = rowsum(tre[c]), im = rowsum(tim[c]);
            if (rok && 16 + c < mb && lk == (c & 3)) put(16 + c, re, im);
        }
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            const bool ok = (F.okm >> (KS0 + s)) & 1u;
            step(ok ? F.f1[s].x : 0.0, ok ? F.f1[s].y : 0.0, 4 * s + lk);
        }
        if (ch == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                xs[r * 64] = mk<double2>(acc[0][r] - acc[1][r], acc[2][r] - acc[0][r] - acc[1][r]);
#pragma unroll
            for (int c = 0; c < NT; ++c) xs[(4 + c) * 64] = mk<double2>(rowsum(tre[c]), rowsum(tim[c]));
            return;
        }
        // X', AX', R' = AX' - X' theta; column norms (sums over the 16 rows li,
        // added in strip order to the wave's running sums)
        auto finish = [&](int j, double2 x, double2 ax, bool mine) {
            double nr = 0.0, nx = 0.0;
            if (mine && rok && j < mb) {
                const double tj = th[j];
                const double2 res = mk<double2>(ax.x - tj * x.x, ax.y - tj * x.y);
                U[(size_t)j * ld + row] = x;
                U[(size_t)(3 * mb + j) * ld + row] = ax;
                const size_t o = (size_t)(mb + j) * ld + row;
                if constexpr (MIX) U32[o] = make_float2((float)res.x, (float)res.y);
                else U[o] = res;
                nr = cabs2(res);
                nx = cabs2(x);
            }
            for (int o = 8; o > 0; o >>= 1) {
                nr += __shfl_down(nr, o, 16);
                nx += __shfl_down(nx, o, 16);
            }
            if (mine && li == 0) {
                wred[j] += nr;
                wred[CW + j] += nx;
            }
        };
#pragma unroll
        for (int r = 0; r < 4; ++r)
            finish(lk + 4 * r, xs[r * 64], mk<double2>(acc[0][r] - acc[1][r], acc[2][r] - acc[0][r] - acc[1][r]),
                   true);
#pragma unroll
        for (int c = 0; c < NT; ++c)
            finish(16 + c, xs[(4 + c) * 64], mk<double2>(rowsum(tre[c]), rowsum(tim[c])), lk == (c & 3));
    };
    // Software pipeline over the chains: the AS fragments of a strip load while
    // its S chain runs, the next strip's S fragments while its AS chain runs,
    // so each wave keeps one chain's loads in flight behind its matrix work.
    // The last prefetch repeats the wave's last strip (in bounds, unused).
    // The widest instances (21 and 22 columns, and the FP64 one of up to 20
    // columns at full basis) cannot hold two chains' fragments beside their
    // accumulators without spilling: they load each chain just before it runs.
    constexpr bool PIPE = NT < 5 && (MIX || KS0 < 10);
    size_t st = (size_t)blockIdx.x * 4 + wave;
    if constexpr (PIPE) {
        Frag FA, FB;
        if (st < nstrip) load(FA, st, 0);
        for (; st < nstrip; st += nwaves) {
            load(FB, st, 1);
            chain(FA, st, 0);
            load(FA, st + nwaves < nstrip ? st + nwaves : st, 0);
            chain(FB, st, 1);
        }
    } else {
        Frag F;
        for (; st < nstrip; st += nwaves) {
            load(F, st, 0);
            chain(F, st, 0);
            load(F, st, 1);
            chain(F, st, 1);
        }
    }
    // sums over the 4 waves in order
    __syncthreads();
    if (tid < 2 * mb) {
        const int which = tid / mb, j = tid % mb;
        double t = 0.0;
        for (int w = 0; w < 4; ++w) t += red[(w * 2 + which) * CW + j];
        npart[(size_t)blockIdx.x * 2 * mb + tid] = t;
    }
}

template <int KS0, int KS1, int NT>
static hipError_t update_wave(const void* V, const void* V32, void* U, void* U32, size_t ld, size_t n,
                              const BasisMap& bm, const void* C, const double* theta, int nparts, double* npart,
                              hipStream_t s) {
    constexpr int CW = 16 + ((NT + 1) & ~1), NX = 4 + NT;   // as in the kernel
    const int K = bm.K, mb = bm.mb;
    if (mb > CW || (K - mb + 3) / 4 > KS0 || (mb + 3) / 4 > KS1 || K > BASIS_KMAX || !n) return hipErrorInvalidValue;
    if ((V32 == nullptr) != (U32 == nullptr)) return hipErrorInvalidValue;
    const size_t lds = (size_t)std::max(mb + 4 * KS0, 4 * KS1) * CW * sizeof(double2) +
                       (size_t)9 * CW * sizeof(double) + (size_t)4 * NX * 64 * sizeof(double2) +
                       (size_t)2 * K * sizeof(int);
    auto launch = [&](auto kern) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nparts), dim3(256), lds, s, (const double2*)V, (const float2*)V32,
                           (double2*)U, (float2*)U32, ld, n, bm, (const double2*)C, theta, npart);
        return hipGetLastError();
    };
    return V32 ? launch(update_wave_kernel<KS0, KS1, NT, true>) : launch(update_wave_kernel<KS0, KS1, NT, false>);
}

hipError_t launch_update_mfma(const void* V, const void* V32, void* U, void* U32, size_t ld, size_t n,
                              const BasisMap& bm, const void* C, const double* theta, int nparts, double* npart,
                              double* norms, hipStream_t s, int rows, bool sum) {
    const int mb = bm.mb;
    const int nk0 = (bm.K - mb + 3) / 4;   // k-steps over the W and P columns
    hipError_t e;
#define UPW(KS0, KS1, NT) update_wave<KS0, KS1, NT>(V, V32, U, U32, ld, n, bm, C, theta, nparts, npart, s)
#define UPB(MJ, RB) update_mj<MJ, RB>(V, V32, U, U32, ld, n, bm, C, theta, nparts, npart, s)
    if (mb < 1 || mb > 22) return hipErrorInvalidValue;
    if (rows == 0 && mb <= 16)
        e = nk0 <= 2 ? UPW(2, 4, 0) : nk0 <= 4 ? UPW(4, 4, 0) : nk0 <= 6 ? UPW(6, 4, 0) : UPW(8, 4, 0);
    else if (rows == 0 && mb <= 20)
        e = nk0 <= 2   ? UPW(2, 5, 4)
            : nk0 <= 4 ? UPW(4, 5, 4)
            : nk0 <= 6 ? UPW(6, 5, 4)
            : nk0 <= 8 ? UPW(8, 5, 4)
                       : UPW(10, 5, 4);
    else if (rows == 0 && mb <= 21)
        e = nk0 <= 4 ? UPW(4, 6, 5) : nk0 <= 8 ? UPW(8, 6, 5) : UPW(11, 6, 5);
    else if (rows == 0)
        e = nk0 <= 4 ? UPW(4, 6, 6) : nk0 <= 8 ? UPW(8, 6, 6) : UPW(11, 6, 6);
    else if (mb <= 16)
        e = rows == 16 ? UPB(1, 16) : UPB(1, 32);
    else
        e = rows == 16 ? UPB(2, 16) : UPB(2, 32);
#undef UPW
#undef UPB
    if (e != hipSuccess || !sum) return e;
    return launch_reduce(npart, nparts, 2 * mb, norms, s);
}

}  // namespace mfd
