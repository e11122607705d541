// HIP kernels of the multigrid hot path and setup, for gfx950 (wave64).
//
// Memory-bound kernels (BSR SpMV, block-Jacobi sweeps, transfers, vector ops)
// use the sliced row-interleaved layout described in kernels.h: a wavefront
// owns floor(64/nb) consecutive block rows, one lane per scalar row, so every
// load of matrix values by a wavefront is one contiguous run of L values.
// Workgroups are 4 wavefronts; workgroup ids are remapped so that each of the
// 8 XCDs (dispatched round-robin) processes one contiguous range of slices,
// which keeps neighbouring x blocks in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>

#include "kernels.h"

namespace amgdg {

constexpr int WG = 256;
constexpr int WAVES_PER_WG = WG / 64;

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    const int q = nblk >> 3, rmd = nblk & 7;
    const int x = bid & 7, j = bid >> 3;
    return x * q + (x < rmd ? x : rmd) + j;
}

// The same runs, each walked from its end when rev is set (XCD x holds the
// q + (x < rmd) workgroups x, x + 8, ...; j counts them).
__device__ __forceinline__ int xcd_remap_dir(int bid, int nblk, int rev) {
    const int q = nblk >> 3, rmd = nblk & 7;
    const int x = bid & 7, j = bid >> 3;
    const int len = q + (x < rmd ? 1 : 0);
    return x * q + (x < rmd ? x : rmd) + (rev ? len - 1 - j : j);
}

static inline unsigned grid_for(int64_t n, int per = WG) { return unsigned((n + per - 1) / per); }

// ============================================================ BSR kernels

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
};
template <>
struct Vec16<float> {
    using type = float4;
};

// Makes this wavefront's LDS writes visible to its own later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// r[c] -= sum_t vals[t] * x(t)[c] over the flattened (slot, column) values of
// this lane's row; the x blocks of the slice are first staged in LDS (xs, one
// row of tpad * M values per block row of the slice) by the br lanes of the
// block row, lane i taking the block columns i, i + br, ...
// CHUNKED (one column): rows too long for their x blocks to be staged in LDS
// at once (coarse operators whose rows span much of the level) stage them
// A.tpad values at a time (the launcher sets tpad to the chunk length, a
// multiple of VW); the products run in the same order, so the result is the
// same as with one staging.

template <typename T, int M, bool CHUNKED = false>
__device__ __forceinline__ void sell_row(const Sell<T>& A, int slice, int lane, int lc, int g, int i,
                                         const T* __restrict__ x, int ld, T* xs, T (&r)[M], T sign) {
    constexpr int VW = 16 / int(sizeof(T));
    using V = typename Vec16<T>::type;
    const int L = A.L, bc = A.bc, G = A.G, TP = A.tpad;
    const int K = A.K[slice];
    const int Tn = K * bc;
    const int TQ = (Tn + VW - 1) / VW;
    const int32_t* __restrict__ cp = A.cols + A.coff[slice] + g;
    const V* __restrict__ vp = reinterpret_cast<const V*>(A.vals + A.voff[slice]) + lc;
    if (CHUNKED) {
        static_assert(!CHUNKED || M == 1, "the chunked form takes one column");
        T* xr = xs + g * TP;
        for (int c0 = 0; c0 < TQ * VW; c0 += TP) {
            const int cn = min(TP, TQ * VW - c0);
            if (lane < L)
                for (int t = c0 + i; t < c0 + cn; t += A.br) {
                    T v = T(0);
                    if (t < Tn) {
                        const int kk = t / bc;
                        v = x[(int64_t(cp[kk * G]) * bc + (t - kk * bc)) * ld];
                    }
                    xr[t - c0] = v;
                }
            wave_lds_sync();
            const int q1 = (c0 + cn) / VW;
#pragma unroll 4
            for (int q = c0 / VW; q < q1; ++q) {
                T a[VW];
                *reinterpret_cast<V*>(a) = vp[q * L];
#pragma unroll
                for (int u = 0; u < VW; ++u) r[0] += sign * a[u] * xr[q * VW + u - c0];
            }
            wave_lds_sync();
        }
        return;
    }
    T* xr = xs + g * TP * M;
    // the first PRE value vectors do not depend on the staging: load them first
    // (one or two columns only, to keep the register count down)
    constexpr int PRE = M <= 2 ? 4 : 0;
    V pre[PRE > 0 ? PRE : 1];
#pragma unroll
    for (int q = 0; q < PRE; ++q)
        if (q < TQ) pre[q] = vp[q * L];
    // rows of M values move as 16-byte vectors when the stride and the base allow
    const bool vx = M % VW == 0 && ld % VW == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (lane < L) {
        // lane i stages columns i, i + br, ... of every block (one pass when bc <= br)
        for (int j = i; j < bc; j += A.br) {
            // unrolled so that several blocks' column and x loads are in flight at once
#pragma unroll 4
            for (int kk = 0; kk < K; ++kk) {
                const T* __restrict__ src = x + (int64_t(cp[kk * G]) * bc + j) * ld;
                T* dst = xr + (kk * bc + j) * M;
                if (vx) {
#pragma unroll
                    for (int q = 0; q < M / VW; ++q) reinterpret_cast<V*>(dst)[q] = reinterpret_cast<const V*>(src)[q];
                } else {
#pragma unroll
                    for (int c = 0; c < M; ++c) dst[c] = src[c];
                }
            }
        }
        for (int t = Tn + i; t < TQ * VW; t += A.br)
#pragma unroll
            for (int c = 0; c < M; ++c) xr[t * M + c] = T(0);
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
        if (q < TQ) {
            T a[VW];
            *reinterpret_cast<V*>(a) = pre[q];
#pragma unroll
            for (int u = 0; u < VW; ++u)
#pragma unroll
                for (int c = 0; c < M; ++c) r[c] += sign * a[u] * xr[(q * VW + u) * M + c];
        }
    }
#pragma unroll 4
    for (int q = PRE; q < TQ; ++q) {
        T a[VW];
        *reinterpret_cast<V*>(a) = vp[q * L];
#pragma unroll
        for (int u = 0; u < VW; ++u)
#pragma unroll
            for (int c = 0; c < M; ++c) r[c] += sign * a[u] * xr[(q * VW + u) * M + c];
    }
}

template <typename T, int M, int MODE, bool ROWS, bool CHUNKED = false>
__global__ __launch_bounds__(WG) void k_sweep(Sell<T> A, const T* __restrict__ dinv, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, T omega,
                                               const int32_t* __restrict__ colmask, int ld, T* __restrict__ y2) {
    constexpr bool HAS_B = (MODE == SWEEP || MODE == SWEEP0);
    constexpr bool HAS_A = (MODE != SWEEP0);
    constexpr int VW = 16 / int(sizeof(T));
    using V = typename Vec16<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_WG + wave;
    if (slice >= A.n_slices) return;
    const int L = A.L, br = A.br, G = A.G, BP = A.brpad;
    const int lc = lane < L ? lane : L - 1;
    const int g = lc / br;
    const int i = lc - g * br;
    const int64_t brow = ROWS ? int64_t(A.rows[int64_t(slice) * G + g]) : int64_t(slice) * G + g;
    const bool own = lane < L && brow < A.n_brow;
    const int64_t row = brow * br + i;
    T* xs = reinterpret_cast<T*>(smem_raw) + int64_t(wave) * G * (A.tpad + BP) * M;
    T* rs = xs + G * A.tpad * M;

    // the first DPRE vectors of this lane's D^{-1} row do not depend on the
    // residual: load them first (one or two columns only)
    const V* __restrict__ dp = reinterpret_cast<const V*>(dinv + int64_t(slice) * BP * L) + lc;
    constexpr int DPRE = M <= 2 ? 4 : 0;
    V dpre[DPRE > 0 ? DPRE : 1];
#pragma unroll
    for (int q = 0; q < DPRE; ++q)
        if (q < BP / VW) dpre[q] = dp[q * L];
    T r[M];
#pragma unroll
    for (int c = 0; c < M; ++c) r[c] = T(0);
    if (HAS_B && own) {
#pragma unroll
        for (int c = 0; c < M; ++c) r[c] = b[row * ld + c];
    }
    if (HAS_A) sell_row<T, M, CHUNKED>(A, slice, lane, lc, g, i, x, ld, xs, r, T(-1));
    // residual of the block row through LDS, then row i of D^{-1}
    T* rr = rs + g * BP * M;
    if (lane < L) {
#pragma unroll
        for (int c = 0; c < M; ++c) rr[i * M + c] = r[c];
        for (int t = br + i; t < BP; t += br)
#pragma unroll
            for (int c = 0; c < M; ++c) rr[t * M + c] = T(0);
    }
    wave_lds_sync();
    T o[M];
#pragma unroll
    for (int c = 0; c < M; ++c) o[c] = T(0);
#pragma unroll
    for (int jq = 0; jq < DPRE; ++jq) {
        if (jq < BP / VW) {
            T d[VW];
            *reinterpret_cast<V*>(d) = dpre[jq];
#pragma unroll
            for (int u = 0; u < VW; ++u)
#pragma unroll
                for (int c = 0; c < M; ++c) o[c] += d[u] * rr[(jq * VW + u) * M + c];
        }
    }
#pragma unroll 4
    for (int jq = DPRE; jq < BP / VW; ++jq) {
        T d[VW];
        *reinterpret_cast<V*>(d) = dp[jq * L];
#pragma unroll
        for (int u = 0; u < VW; ++u)
#pragma unroll
            for (int c = 0; c < M; ++c) o[c] += d[u] * rr[(jq * VW + u) * M + c];
    }
    if (!own) return;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        T v;
        if (MODE == SWEEP) v = x[row * ld + c] + omega * o[c];
        else if (MODE == SWEEP0) v = omega * o[c];
        else if (MODE == RELAX) v = colmask[c] ? x[row * ld + c] + omega * o[c] : x[row * ld + c];
        else v = -o[c];  // DINVA: r = -A x
        y[row * ld + c] = v;
        if (MODE == SWEEP0 && y2) y2[row * ld + c] = o[c];
    }
}

template <typename T, int M, int MODE, bool ROWS, bool CHUNKED = false>
__global__ __launch_bounds__(WG) void k_spmv(Sell<T> A, const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ y, int ldx, int ldy, T omega, T* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wg = xcd_remap_dir(blockIdx.x, gridDim.x, A.rev);
    const int slice = wg * WAVES_PER_WG + wave;
    const bool live = slice < A.n_slices;
    if (!live && MODE != AX_DOT) return;  // AX_DOT: every wave reaches the workgroup barrier
    const int L = A.L, br = A.br, G = A.G;
    const int lc = lane < L ? lane : L - 1;
    const int g = lc / br;
    const int i = lc - g * br;
    const int64_t brow = !live ? int64_t(A.n_brow)
                                 : ROWS ? int64_t(A.rows[int64_t(slice) * G + g]) : int64_t(slice) * G + g;
    const bool own = live && lane < L && brow < A.n_brow;
    const int64_t row = brow * br + i;
    T* xs = reinterpret_cast<T*>(smem_raw) + int64_t(wave) * G * A.tpad * M;
    // the epilogue's own-row operands are loaded first, so their latency
    // overlaps the row's product instead of following it
    constexpr bool PB = (MODE == B_MINUS || MODE == B_PLUS || MODE == S_SWEEP || MODE == S_SWEEP_R);
    constexpr bool PX = (MODE == S_SWEEP || MODE == S_SWEEP_R || MODE == AX_DOT);
    const bool px = PX || A.unit;  // the own x entries (unit: the implied diagonal blocks)
    T bo[PB ? M : 1], xo[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (PB) bo[c] = own ? b[row * ldy + c] : T(0);
        xo[c] = (px && own) ? x[row * ldx + c] : T(0);
    }
    T acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = T(0);
    if (live) sell_row<T, M, CHUNKED>(A, slice, lane, lc, g, i, x, ldx, xs, acc, T(1));
    if (A.unit)
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] += xo[c];
    if (MODE == AX_DOT) {
        // the workgroup's partial of x . y per column: lanes of each wave by an
        // xor tree, then the four waves in order
        __shared__ T red[WAVES_PER_WG][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T v = own ? xo[c] * acc[c] : T(0);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) red[wave][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < M)
            part[int64_t(threadIdx.x) * gridDim.x + wg] =
                (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    }
    if (!own) return;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        T v = acc[c];
        if (MODE == B_MINUS) v = bo[PB ? c : 0] - v;
        else if (MODE == B_PLUS) v = bo[PB ? c : 0] + v;
        else if (MODE == S_SWEEP) v = xo[c] + omega * (bo[PB ? c : 0] - v);
        else if (MODE == S_SWEEP_R) {
            const T e = bo[PB ? c : 0] - v;
            part[row * ldy + c] = e;  // y2: the residual the sweep starts from
            v = xo[c] + omega * e;
        }
        y[row * ldy + c] = v;
    }
}

// the row-mapped instance only for slices whose rows were reordered
#define SELL_LAUNCH(KERNEL, MD, ...)                                                                   \
    if (A.rows) hipLaunchKernelGGL((KERNEL<T, M, MD, true, CHUNKED>), grid, block, lds, st, __VA_ARGS__); \
    else hipLaunchKernelGGL((KERNEL<T, M, MD, false, CHUNKED>), grid, block, lds, st, __VA_ARGS__)

template <typename T, int M, bool CHUNKED = false>
static hipError_t sweep_m(int mode, const Sell<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega,
                          const int32_t* mask, int ld, hipStream_t st, T* y2) {
    dim3 grid(grid_for(A.n_slices, WAVES_PER_WG)), block(WG);
    if (A.n_slices == 0) return hipSuccess;
    const size_t lds = size_t(WAVES_PER_WG) * A.G * (A.tpad + A.brpad) * M * sizeof(T);
    switch (mode) {
        case SWEEP: SELL_LAUNCH(k_sweep, SWEEP, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case SWEEP0: SELL_LAUNCH(k_sweep, SWEEP0, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case RELAX: SELL_LAUNCH(k_sweep, RELAX, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case DINVA: SELL_LAUNCH(k_sweep, DINVA, A, dinv, x, b, y, omega, mask, ld, y2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int M, bool CHUNKED = false>
static hipError_t spmv_m(int mode, const Sell<T>& A, const T* x, const T* b, T* y, int ldx, int ldy,
                         hipStream_t st, T omega, T* part = nullptr) {
    dim3 grid(grid_for(A.n_slices, WAVES_PER_WG)), block(WG);
    if (A.n_slices == 0) return hipSuccess;
    const size_t lds = size_t(WAVES_PER_WG) * A.G * A.tpad * M * sizeof(T);
    switch (mode) {
        case AX: SELL_LAUNCH(k_spmv, AX, A, x, b, y, ldx, ldy, omega, part); break;
        case B_MINUS: SELL_LAUNCH(k_spmv, B_MINUS, A, x, b, y, ldx, ldy, omega, part); break;
        case B_PLUS: SELL_LAUNCH(k_spmv, B_PLUS, A, x, b, y, ldx, ldy, omega, part); break;
        case S_SWEEP: SELL_LAUNCH(k_spmv, S_SWEEP, A, x, b, y, ldx, ldy, omega, part); break;
        case S_SWEEP_R: SELL_LAUNCH(k_spmv, S_SWEEP_R, A, x, b, y, ldx, ldy, omega, part); break;
        case AX_DOT: SELL_LAUNCH(k_spmv, AX_DOT, A, x, b, y, ldx, ldy, omega, part); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// LDS one workgroup may allocate on the current device (160 KB on gfx950),
// read once per device.  Launch shapes are chosen within 64 KB, which keeps
// several workgroups resident per CU; only a launch that cannot fit 64 KB even
// at one block row per wavefront and one column (coarse operators whose rows
// span most of the level) uses more, up to this limit.
static size_t lds_limit() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int a = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || a < 65536)
            a = 65536;
        cache[dev].store(a, std::memory_order_relaxed);
        v = a;
    }
    return size_t(v);
}

// Columns are processed in chunks (each a separate launch): the LDS staging
// buffers grow with the chunk width, so it is capped at 4 (FP64) / 8 (FP32).
// and kept within 64 KB of LDS per workgroup.
// `want` (1, 2, 4 or 8; 0: the default 4 FP64 / 8 FP32) bounds the chunk width; the
// chunk width does not change the arithmetic of any column.
template <typename T>
static int sell_chunk(int rem, const Sell<T>& A, bool with_dinv, int want) {
    int cap = want > 0 ? want : (sizeof(T) == 8 ? 4 : 8);
    const size_t per_col = size_t(WAVES_PER_WG) * A.G * (A.tpad + (with_dinv ? A.brpad : 0)) * sizeof(T);
    while (cap > 1 && per_col * cap > 65536) cap = cap == 8 ? 4 : cap - 1;
    const int w = rem >= 8 ? 8 : rem >= 4 ? 4 : rem;
    return w <= cap ? w : (cap >= 4 ? 4 : cap >= 2 ? 2 : 1);
}

// LDS budget of a staged launch per workgroup (several workgroups stay resident per CU)
constexpr size_t STAGE_LDS = 65536;

// The sliced matrix as a chunked launch sees it: tpad becomes the chunk of x
// staged at a time, the longest multiple of VW for which a workgroup's staging
// (and D^{-1} residuals, with_dinv) takes at most 64 KB.
template <typename T>
static Sell<T> chunked_view(const Sell<T>& A, bool with_dinv) {
    constexpr int VW = 16 / int(sizeof(T));
    Sell<T> c = A;
    const int64_t per_row = int64_t(STAGE_LDS) / (int64_t(WAVES_PER_WG) * std::max(A.G, 1) * int64_t(sizeof(T)));
    const int64_t chunk = (per_row - (with_dinv ? A.brpad : 0)) / VW * VW;
    c.tpad = int32_t(std::max<int64_t>(VW, std::min<int64_t>(chunk, A.tpad)));
    return c;
}

int sell_rows_per_wave(int br, int bc, int max_row_blocks) {
    const size_t need = size_t((int64_t(max_row_blocks) * bc + 1) / 2 * 2 + (br + 1) / 2 * 2) * sizeof(double);
    int G = 64 / br;
    while (G > 1 && size_t(WAVES_PER_WG) * G * need > STAGE_LDS) --G;
    // lowered so far that half the lanes or more would idle: one block row per
    // wavefront, which the split-row kernels serve on all 64 lanes (br <= 16)
    if (G < 64 / br && G * br <= 32 && br <= 16) G = 1;
    return G;
}

// Operators of at most this many block rows at one block row per wavefront take
// the split kernels' workgroup-per-row form (WGR).
constexpr int SPLIT_WG_SLICES = 4096;

// The sweeps with D^{-1} (sliced layout) at one block row per wavefront, the
// row's product split over four groups of 16 lanes as in k_spmv_split (with WGR
// over a workgroup's 16 groups, for operators of few block rows); the block
// row's residual then goes through LDS to the br lanes that apply their row of
// D^{-1}.  One column per launch at every batch width.
template <typename T, int MODE, bool ROWS, bool WGR>
__global__ __launch_bounds__(WG) void k_sweep_split(Sell<T> A, const T* __restrict__ dinv, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y, T omega,
                                                     const int32_t* __restrict__ colmask, int ld,
                                                     T* __restrict__ y2) {
    constexpr bool HAS_B = (MODE == SWEEP || MODE == SWEEP0);
    constexpr bool HAS_A = (MODE != SWEEP0);
    constexpr int VW = 16 / int(sizeof(T));
    constexpr int NG = WGR ? 4 * WAVES_PER_WG : 4;
    using V = typename Vec16<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red[WGR ? WAVES_PER_WG : 1][16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = WGR ? xcd_remap(blockIdx.x, gridDim.x) : xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_WG + wave;
    if (slice >= A.n_slices) return;  // the whole wavefront (WGR: the whole workgroup)
    const int br = A.br, bc = A.bc, L = A.L, BP = A.brpad;  // G == 1, so L == br
    const int q = WGR ? wave * 4 + (lane >> 4) : lane >> 4, i = lane & 15;
    const int64_t brow = ROWS ? int64_t(A.rows[slice]) : int64_t(slice);
    const bool mine = q == 0 && i < br;
    const bool own = mine && brow < A.n_brow;
    const int64_t row = brow * br + i;
    T* xs = reinterpret_cast<T*>(smem_raw) + (WGR ? 0 : int64_t(wave) * (A.tpad + BP));
    T* rr = xs + A.tpad;
    T acc = T(0);
    if (HAS_A) {
        const int K = A.K[slice];
        const int Tn = K * bc, TQ = (Tn + VW - 1) / VW;
        const int32_t* __restrict__ cp = A.cols + A.coff[slice];
        for (int t = WGR ? int(threadIdx.x) : lane; t < TQ * VW; t += WGR ? WG : 64) {
            T v = T(0);
            if (t < Tn) {
                const int kk = t / bc;
                v = x[(int64_t(cp[kk]) * bc + (t - kk * bc)) * ld];
            }
            xs[t] = v;
        }
        if (WGR) __syncthreads();
        else wave_lds_sync();
        if (i < L) {
            const V* __restrict__ vp = reinterpret_cast<const V*>(A.vals + A.voff[slice]) + i;
#pragma unroll 4
            for (int v = q; v < TQ; v += NG) {
                T a[VW];
                *reinterpret_cast<V*>(a) = vp[int64_t(v) * L];
#pragma unroll
                for (int u = 0; u < VW; ++u) acc += a[u] * xs[v * VW + u];
            }
        }
        acc += __shfl_xor(acc, 16);
        acc += __shfl_xor(acc, 32);
        if (WGR) {
            if (lane < 16) red[wave][lane] = acc;
            __syncthreads();
            acc = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
        }
    }
    if (WGR && wave != 0) return;  // the D^{-1} stage runs on the first wavefront
    // residual of the block row through LDS (zero-padded to brpad), then row i of D^{-1}
    if (q == 0 && i < BP) {
        T r = T(0);
        if (own) r = (HAS_B ? b[row * ld] : T(0)) - acc;
        rr[i] = r;
    }
    wave_lds_sync();
    if (!own) return;
    const V* __restrict__ dp = reinterpret_cast<const V*>(dinv + int64_t(slice) * BP * L) + i;
    T o = T(0);
#pragma unroll 4
    for (int jq = 0; jq < BP / VW; ++jq) {
        T d[VW];
        *reinterpret_cast<V*>(d) = dp[jq * L];
#pragma unroll
        for (int u = 0; u < VW; ++u) o += d[u] * rr[jq * VW + u];
    }
    T v;
    if (MODE == SWEEP) v = x[row * ld] + omega * o;
    else if (MODE == SWEEP0) v = omega * o;
    else if (MODE == RELAX) v = colmask[0] ? x[row * ld] + omega * o : x[row * ld];
    else v = -o;  // DINVA: r = -A x
    y[row * ld] = v;
    if (MODE == SWEEP0 && y2) y2[row * ld] = o;
}

template <typename T>
static hipError_t sweep_split(int mode, const Sell<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega,
                              int m, const int32_t* colmask, hipStream_t st, T* y2) {
    const bool wgr = A.n_slices <= SPLIT_WG_SLICES;  // one workgroup per block row
    const size_t lds = size_t(wgr ? 1 : WAVES_PER_WG) * (A.tpad + A.brpad) * sizeof(T);
    if (lds > lds_limit()) return hipErrorInvalidConfiguration;
    if (A.n_slices == 0) return hipSuccess;
    const dim3 grid{unsigned(wgr ? A.n_slices : grid_for(A.n_slices, WAVES_PER_WG)), 1u, 1u},
        block{unsigned(WG), 1u, 1u};
    for (int c = 0; c < m; ++c) {
        const T* xc = x ? x + c : nullptr;
        const T* bcol = b ? b + c : nullptr;
        const int32_t* mc = colmask ? colmask + c : nullptr;
        T* yc = y + c;
        T* y2c = y2 ? y2 + c : nullptr;
#define SPLIT_LAUNCH_W(MD, W)                                                                                 \
    if (A.rows)                                                                                               \
        hipLaunchKernelGGL((k_sweep_split<T, MD, true, W>), grid, block, lds, st, A, dinv, xc, bcol, yc, omega, mc, \
                           m, y2c);                                                                           \
    else                                                                                                      \
        hipLaunchKernelGGL((k_sweep_split<T, MD, false, W>), grid, block, lds, st, A, dinv, xc, bcol, yc, omega,    \
                           mc, m, y2c)
#define SPLIT_LAUNCH(MD)           \
    if (wgr) {                     \
        SPLIT_LAUNCH_W(MD, true);  \
    } else {                       \
        SPLIT_LAUNCH_W(MD, false); \
    }
        switch (mode) {
            case SWEEP: SPLIT_LAUNCH(SWEEP); break;
            case SWEEP0: SPLIT_LAUNCH(SWEEP0); break;
            case RELAX: SPLIT_LAUNCH(RELAX); break;
            case DINVA: SPLIT_LAUNCH(DINVA); break;
            default: return hipErrorInvalidValue;
        }
#undef SPLIT_LAUNCH
#undef SPLIT_LAUNCH_W
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_sweep(int mode, const Sell<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                        const int32_t* colmask, hipStream_t st, int cap, T* y2) {
    // Launches whose staging of one column exceeds the LDS a workgroup may
    // take (coarse operators with rows across most of the level) stage x in
    // chunks instead, one column per launch.
    const bool fits1 = size_t(WAVES_PER_WG) * A.G * (A.tpad + A.brpad) * sizeof(T) <= lds_limit();
    if (A.G == 1 && A.br <= 16 && size_t(WAVES_PER_WG) * (A.tpad + A.brpad) * sizeof(T) <= lds_limit())
        return sweep_split(mode, A, dinv, x, b, y, omega, m, colmask, st, y2);
    if (!fits1) {
        // x staging of one column does not fit: chunked staging, one column per launch
        const Sell<T> Ac = chunked_view(A, true);
        for (int c = 0; c < m; ++c) {
            const hipError_t e = sweep_m<T, 1, true>(mode, Ac, dinv, x ? x + c : nullptr, b ? b + c : nullptr, y + c,
                                                     omega, colmask ? colmask + c : nullptr, m, st,
                                                     y2 ? y2 + c : nullptr);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    int c0 = 0;
    while (c0 < m) {
        const int w = sell_chunk<T>(m - c0, A, true, cap);
        if (size_t(WAVES_PER_WG) * A.G * (A.tpad + A.brpad) * w * sizeof(T) > lds_limit())
            return hipErrorInvalidConfiguration;
        const T* xc = x ? x + c0 : nullptr;
        const T* bc = b ? b + c0 : nullptr;
        const int32_t* mc = colmask ? colmask + c0 : nullptr;
        T* y2c = y2 ? y2 + c0 : nullptr;
        hipError_t e;
        switch (w) {
            case 8: e = sweep_m<T, 8>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 4: e = sweep_m<T, 4>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 3: e = sweep_m<T, 3>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 2: e = sweep_m<T, 2>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            default: e = sweep_m<T, 1>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
        }
        if (e != hipSuccess) return e;
        c0 += w;
    }
    return hipSuccess;
}

// Long rows at one block row per wavefront (G = 1 with br <= 16, where the
// row's x staging does not fit more): the sliced kernel would walk the row's
// values with br lanes and leave the rest idle.  Here the four groups of 16
// lanes take every fourth value vector of the row, so a wavefront still reads
// one contiguous run per step, and two xor-shuffles add the groups' partial
// sums.  With WGR (operators of few block rows, SPLIT_WG_SLICES or fewer, as
// the hexahedral hierarchy's coarse levels) a whole workgroup takes one block
// row: its 16 groups take every sixteenth vector, the staging is shared, and
// the four wavefronts' sums are added in order through LDS, so four times as
// many wavefronts stream the operator.  One column per launch; every batch
// width takes this kernel, so a column's rounding does not depend on the width.
template <typename T, int MODE, bool ROWS, bool WGR>
__global__ __launch_bounds__(WG) void k_spmv_split(Sell<T> A, const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, int ldx, int ldy, T omega,
                                                    T* __restrict__ y2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red[WGR ? WAVES_PER_WG : 1][16];
    constexpr int VW = 16 / int(sizeof(T));
    constexpr int NG = WGR ? 4 * WAVES_PER_WG : 4;  // groups of 16 lanes per block row
    using V = typename Vec16<T>::type;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slice = WGR ? xcd_remap(blockIdx.x, gridDim.x) : xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_WG + wave;
    if (slice >= A.n_slices) return;  // the whole wavefront (WGR: the whole workgroup)
    const int br = A.br, bc = A.bc, L = A.L;  // G == 1, so L == br
    const int q = WGR ? wave * 4 + (lane >> 4) : lane >> 4, i = lane & 15;
    const int64_t brow = ROWS ? int64_t(A.rows[slice]) : int64_t(slice);
    const bool own = q == 0 && i < br && brow < A.n_brow;
    const int64_t row = brow * br + i;
    T* xs = reinterpret_cast<T*>(smem_raw) + (WGR ? 0 : int64_t(wave) * A.tpad);
    const int K = A.K[slice];
    const int Tn = K * bc, TQ = (Tn + VW - 1) / VW;
    const int32_t* __restrict__ cp = A.cols + A.coff[slice];
    for (int t = WGR ? int(threadIdx.x) : lane; t < TQ * VW; t += WGR ? WG : 64) {
        T v = T(0);
        if (t < Tn) {
            const int kk = t / bc;
            v = x[(int64_t(cp[kk]) * bc + (t - kk * bc)) * ldx];
        }
        xs[t] = v;
    }
    if (WGR) __syncthreads();
    else wave_lds_sync();
    T acc = T(0);
    if (i < L) {
        const V* __restrict__ vp = reinterpret_cast<const V*>(A.vals + A.voff[slice]) + i;
#pragma unroll 4
        for (int v = q; v < TQ; v += NG) {
            T a[VW];
            *reinterpret_cast<V*>(a) = vp[int64_t(v) * L];
#pragma unroll
            for (int u = 0; u < VW; ++u) acc += a[u] * xs[v * VW + u];
        }
    }
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (WGR) {
        if (lane < 16) red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0) acc = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    }
    if (!own) return;
    if (A.unit) acc += x[row * ldx];
    T val = acc;
    if (MODE == B_MINUS) val = b[row * ldy] - acc;
    else if (MODE == B_PLUS) val = b[row * ldy] + acc;
    else if (MODE == S_SWEEP) val = x[row * ldx] + omega * (b[row * ldy] - acc);
    else if (MODE == S_SWEEP_R) {
        const T e = b[row * ldy] - acc;
        y2[row * ldy] = e;
        val = x[row * ldx] + omega * e;
    }
    y[row * ldy] = val;
}

template <typename T>
static bool spmv_split_ok(int mode, const Sell<T>& A) {
    return A.G == 1 && A.br <= 16 &&
           (mode == AX || mode == B_MINUS || mode == B_PLUS || mode == S_SWEEP || mode == S_SWEEP_R);
}

template <typename T>
static hipError_t spmv_split(int mode, const Sell<T>& A, const T* x, const T* b, T* y, int m, hipStream_t st,
                             T omega, T* y2) {
    const bool wgr = A.n_slices <= SPLIT_WG_SLICES;  // one workgroup per block row
    const size_t lds = size_t(wgr ? 1 : WAVES_PER_WG) * A.tpad * sizeof(T);
    if (lds > lds_limit()) return hipErrorInvalidConfiguration;
    if (A.n_slices == 0) return hipSuccess;
    const dim3 grid{unsigned(wgr ? A.n_slices : grid_for(A.n_slices, WAVES_PER_WG)), 1u, 1u},
        block{unsigned(WG), 1u, 1u};
    for (int c = 0; c < m; ++c) {
        const T* xc = x + c;
        const T* bcol = b ? b + c : nullptr;
        T* yc = y + c;
        T* y2c = y2 ? y2 + c : nullptr;
#define SPLIT_LAUNCH_W(MD, W)                                                                                   \
    if (A.rows)                                                                                                 \
        hipLaunchKernelGGL((k_spmv_split<T, MD, true, W>), grid, block, lds, st, A, xc, bcol, yc, m, m, omega, y2c); \
    else hipLaunchKernelGGL((k_spmv_split<T, MD, false, W>), grid, block, lds, st, A, xc, bcol, yc, m, m, omega, y2c)
#define SPLIT_LAUNCH(MD)           \
    if (wgr) {                     \
        SPLIT_LAUNCH_W(MD, true);  \
    } else {                       \
        SPLIT_LAUNCH_W(MD, false); \
    }
        switch (mode) {
            case AX: SPLIT_LAUNCH(AX); break;
            case B_MINUS: SPLIT_LAUNCH(B_MINUS); break;
            case B_PLUS: SPLIT_LAUNCH(B_PLUS); break;
            case S_SWEEP: SPLIT_LAUNCH(S_SWEEP); break;
            case S_SWEEP_R: SPLIT_LAUNCH(S_SWEEP_R); break;
            default: return hipErrorInvalidValue;
        }
#undef SPLIT_LAUNCH
#undef SPLIT_LAUNCH_W
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_spmv(int mode, const Sell<T>& A, const T* x, const T* b, T* y, int m, hipStream_t st, int cap,
                       T omega, T* y2) {
    if ((mode == S_SWEEP_R) != (y2 != nullptr)) return hipErrorInvalidValue;
    if (spmv_split_ok(mode, A) && size_t(WAVES_PER_WG) * A.tpad * sizeof(T) <= lds_limit())
        return spmv_split(mode, A, x, b, y, m, st, omega, y2);
    if (size_t(WAVES_PER_WG) * A.G * A.tpad * sizeof(T) > lds_limit()) {
        // x staging of one column does not fit: chunked staging, one column per launch
        const Sell<T> Ac = chunked_view(A, false);
        for (int c = 0; c < m; ++c) {
            const hipError_t e =
                spmv_m<T, 1, true>(mode, Ac, x + c, b ? b + c : nullptr, y + c, m, m, st, omega, y2 ? y2 + c : nullptr);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    int c0 = 0;
    while (c0 < m) {
        const int w = sell_chunk<T>(m - c0, A, false, cap);
        if (size_t(WAVES_PER_WG) * A.G * A.tpad * w * sizeof(T) > lds_limit()) return hipErrorInvalidConfiguration;
        const T* bc = b ? b + c0 : nullptr;
        T* y2c = y2 ? y2 + c0 : nullptr;
        hipError_t e;
        switch (w) {
            case 8: e = spmv_m<T, 8>(mode, A, x + c0, bc, y + c0, m, m, st, omega, y2c); break;
            case 4: e = spmv_m<T, 4>(mode, A, x + c0, bc, y + c0, m, m, st, omega, y2c); break;
            case 3: e = spmv_m<T, 3>(mode, A, x + c0, bc, y + c0, m, m, st, omega, y2c); break;
            case 2: e = spmv_m<T, 2>(mode, A, x + c0, bc, y + c0, m, m, st, omega, y2c); break;
            default: e = spmv_m<T, 1>(mode, A, x + c0, bc, y + c0, m, m, st, omega, y2c); break;
        }
        if (e != hipSuccess) return e;
        c0 += w;
    }
    return hipSuccess;
}

template hipError_t launch_sweep<double>(int, const Sell<double>&, const double*, const double*, const double*,
                                         double*, double, int, const int32_t*, hipStream_t, int, double*);
template hipError_t launch_sweep<float>(int, const Sell<float>&, const float*, const float*, const float*, float*,
                                        float, int, const int32_t*, hipStream_t, int, float*);
template hipError_t launch_spmv<double>(int, const Sell<double>&, const double*, const double*, double*, int,
                                        hipStream_t, int, double, double*);
template hipError_t launch_spmv<float>(int, const Sell<float>&, const float*, const float*, float*, int,
                                       hipStream_t, int, float, float*);

// ============================================================ block-CSR kernels (small blocks)

// acc[i][c] = sum over the blocks of block row `brow` handled by this lane of
// A_blk[i][j] * x[col*bc + j][c]; then summed over the P lanes of the group.
template <typename T, int M, int BR>
__device__ __forceinline__ void bcsr_row(const Bcsr<T>& A, int64_t brow, bool valid, int p, const T* __restrict__ x,
                                         int ld, T (&acc)[BR][M]) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int c = 0; c < M; ++c) acc[i][c] = T(0);
    // the M values of an x row are read as 16-byte vectors when the row stride
    // and the base keep them aligned (the same values, so the same sums)
    constexpr int VW = 16 / int(sizeof(T));
    using V = typename Vec16<T>::type;
    const bool vx = M % VW == 0 && ld % VW == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (valid) {
        const int bc = A.bc;
        const int e = A.rp[brow + 1];
        for (int blk = A.rp[brow] + p; blk < e; blk += A.P) {
            const int64_t cb = int64_t(A.ci[blk]) * bc;
            const T* __restrict__ a = A.vals + int64_t(blk) * BR * bc;
            // unrolled so that several columns' loads are in flight at once
#pragma unroll 4
            for (int j = 0; j < bc; ++j) {
                T xv[M];
                const T* __restrict__ xr = x + (cb + j) * ld;
                if (vx) {
#pragma unroll
                    for (int q = 0; q < M / VW; ++q) *reinterpret_cast<V*>(xv + q * VW) = reinterpret_cast<const V*>(xr)[q];
                } else {
#pragma unroll
                    for (int c = 0; c < M; ++c) xv[c] = xr[c];
                }
#pragma unroll
                for (int i = 0; i < BR; ++i) {
                    const T av = a[i * bc + j];
#pragma unroll
                    for (int c = 0; c < M; ++c) acc[i][c] += av * xv[c];
                }
            }
        }
    }
    for (int off = A.P >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int c = 0; c < M; ++c) acc[i][c] += __shfl_xor(acc[i][c], off);
    }
}

template <typename T, int M, int MODE, int BR>
__global__ __launch_bounds__(WG) void k_bsweep(Bcsr<T> A, const T* __restrict__ dinv, const T* __restrict__ x,
                                                const T* __restrict__ b, T* __restrict__ y, T omega,
                                                const int32_t* __restrict__ colmask, int ld, T* __restrict__ y2) {
    constexpr bool HAS_B = (MODE == SWEEP || MODE == SWEEP0);
    constexpr bool HAS_A = (MODE != SWEEP0);
    const int gpw = 64 / A.P;
    const int64_t wv = int64_t(xcd_remap(blockIdx.x, gridDim.x)) * WAVES_PER_WG + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = lane / A.P, p = lane - (lane / A.P) * A.P;
    const int64_t brow = wv * gpw + g;
    const bool valid = brow < A.n_brow;
    // the epilogue's row of D^{-1} and the block row's b are loaded before the
    // block loop, so their latency overlaps it
    const bool mine = valid && p < BR;
    T dv[BR], bv[HAS_B ? BR : 1][M];
#pragma unroll
    for (int j = 0; j < BR; ++j) {
        dv[j] = mine ? dinv[(brow * BR + p) * BR + j] : T(0);
#pragma unroll
        for (int c = 0; c < M; ++c)
            if (HAS_B) bv[j][c] = mine ? b[(brow * BR + j) * ld + c] : T(0);
    }
    T acc[BR][M];
    if (HAS_A) {
        bcsr_row<T, M, BR>(A, brow, valid, p, x, ld, acc);
    } else {
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int c = 0; c < M; ++c) acc[i][c] = T(0);
    }
    if (!valid || p >= BR) return;
    // residual of the whole block row, then row p of D^{-1} applied to it
    T o[M];
#pragma unroll
    for (int c = 0; c < M; ++c) o[c] = T(0);
#pragma unroll
    for (int j = 0; j < BR; ++j) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const T bj = HAS_B ? bv[HAS_B ? j : 0][c] : T(0);
            o[c] += dv[j] * (bj - acc[j][c]);
        }
    }
    const int64_t row = brow * BR + p;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        T v;
        if (MODE == SWEEP) v = x[row * ld + c] + omega * o[c];
        else if (MODE == SWEEP0) v = omega * o[c];
        else if (MODE == RELAX) v = colmask[c] ? x[row * ld + c] + omega * o[c] : x[row * ld + c];
        else v = -o[c];
        y[row * ld + c] = v;
        if (MODE == SWEEP0 && y2) y2[row * ld + c] = o[c];
    }
}

template <typename T, int M, int MODE, int BR>
__global__ __launch_bounds__(WG) void k_bspmv(Bcsr<T> A, const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, int ld, T omega, const T* __restrict__ dinv,
                                               T* __restrict__ y2) {
    const int gpw = 64 / A.P;
    const int64_t wv = int64_t(xcd_remap(blockIdx.x, gridDim.x)) * WAVES_PER_WG + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = lane / A.P, p = lane - (lane / A.P) * A.P;
    const int64_t brow = wv * gpw + g;
    const bool valid = brow < A.n_brow;
    const int64_t row = brow * BR + p;
    // the epilogue's own-row operands are loaded first, so their latency
    // overlaps the block loop instead of following the reduction
    constexpr bool PB = (MODE == B_MINUS || MODE == B_PLUS || MODE == S_SWEEP || MODE == S_SWEEP_R);
    constexpr bool PX = (MODE == S_SWEEP || MODE == S_SWEEP_R);
    const bool px = PX || A.unit;
    T bo[PB ? M : 1], xo[M];
    constexpr bool PD = (MODE == AX_DSCALE);
    T dv[PD ? BR : 1];
    {
        const bool mine = valid && p < BR;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            if (PB) bo[c] = mine ? b[row * ld + c] : T(0);
            xo[c] = (px && mine) ? x[row * ld + c] : T(0);
        }
#pragma unroll
        for (int j = 0; j < BR; ++j)
            if (PD) dv[PD ? j : 0] = mine ? dinv[(brow * BR + p) * BR + j] : T(0);
    }
    T acc[BR][M];
    bcsr_row<T, M, BR>(A, brow, valid, p, x, ld, acc);
    if (!valid || p >= BR) return;
    if (A.unit)
#pragma unroll
        for (int i = 0; i < BR; ++i)
            if (i == p)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[i][c] += xo[c];
    if (MODE == AX_DSCALE) {
        // row p of D'^{-1} (the output rows' own block) applied to the block row's
        // product: the operations of a first sweep whose right-hand side is A x
        T o[M];
#pragma unroll
        for (int c = 0; c < M; ++c) o[c] = T(0);
#pragma unroll
        for (int j = 0; j < BR; ++j) {
#pragma unroll
            for (int c = 0; c < M; ++c) o[c] += dv[PD ? j : 0] * acc[j][c];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            y[row * ld + c] = omega * o[c];
            y2[row * ld + c] = o[c];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < BR; ++i) {
        if (i != p) continue;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T v = acc[i][c];
            if (MODE == B_MINUS) v = bo[PB ? c : 0] - v;
            else if (MODE == B_PLUS) v = bo[PB ? c : 0] + v;
            else if (MODE == S_SWEEP) v = xo[c] + omega * (bo[PB ? c : 0] - v);
            else if (MODE == S_SWEEP_R) {
                const T e = bo[PB ? c : 0] - v;
                y2[row * ld + c] = e;
                v = xo[c] + omega * e;
            }
            y[row * ld + c] = v;
        }
    }
}

// Block rows of many blocks (Bcsr::P = 128 or 256): one wavefront (128) or one
// workgroup (256) per block row; its lanes take the row's entries e = (block q,
// column j) in order, e = t0, t0 + stride, ..., so that neighbouring lanes read
// neighbouring values of a block row and the x entries of one block column.
// The lanes' partial sums are added by an xor butterfly, then over the
// workgroup's wavefronts in order; lane p < BR of the first wavefront writes
// row p.  The summation order depends on the row's length only.
template <typename T, int M, int MODE, int BR>
__global__ __launch_bounds__(WG) void k_bspmv_wide(Bcsr<T> A, const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, int ld, T omega,
                                                    const T* __restrict__ dinv, T* __restrict__ y2) {
    __shared__ T red[WAVES_PER_WG][BR * M];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const bool whole = A.P == 256;  // one workgroup per block row
    const int64_t brow = whole ? int64_t(wg) : int64_t(wg) * WAVES_PER_WG + wave;
    if (brow >= A.n_brow) return;  // the whole wavefront (P = 128) or workgroup (P = 256)
    const int bc = A.bc;
    const int beg = A.rp[brow], end = A.rp[brow + 1];
    const int E = (end - beg) * bc;
    const int stride = whole ? 64 * WAVES_PER_WG : 64;
    const int t0 = (whole ? wave * 64 : 0) + lane;
    // the epilogue's own-row operands first
    constexpr bool PB = (MODE == B_MINUS || MODE == S_SWEEP || MODE == S_SWEEP_R);
    constexpr bool PX = (MODE == S_SWEEP || MODE == S_SWEEP_R);
    const bool writer = lane < BR && (!whole || wave == 0);
    const int64_t row = brow * BR + lane;
    const bool px = PX || A.unit;
    T bo[PB ? M : 1], xo[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (PB) bo[c] = writer ? b[row * ld + c] : T(0);
        xo[c] = (px && writer) ? x[row * ld + c] : T(0);
    }
    constexpr bool PD = (MODE == AX_DSCALE);
    T dv[PD ? BR : 1];
#pragma unroll
    for (int j = 0; j < BR; ++j)
        if (PD) dv[PD ? j : 0] = writer ? dinv[(brow * BR + lane) * BR + j] : T(0);
    T acc[BR][M];
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int c = 0; c < M; ++c) acc[i][c] = T(0);
    // U of a lane's entries per step: their index, value and x loads are all
    // issued before the products (each lane still adds its entries in order)
    constexpr int U = (M * BR <= 8) ? 4 : 2;
    for (int e0 = t0; e0 < E; e0 += U * stride) {
        int blk[U], jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * stride;
            const int q = e < E ? e / bc : 0;
            blk[u] = beg + q;
            jj[u] = e < E ? e - q * bc : 0;
        }
        int32_t col[U];
#pragma unroll
        for (int u = 0; u < U; ++u) col[u] = A.ci[blk[u]];
        T av[U][BR], xv[U][M];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T* __restrict__ a = A.vals + int64_t(blk[u]) * BR * bc + jj[u];
#pragma unroll
            for (int i = 0; i < BR; ++i) av[u][i] = a[i * bc];
            const T* __restrict__ xr = x + (int64_t(col[u]) * bc + jj[u]) * ld;
#pragma unroll
            for (int c = 0; c < M; ++c) xv[u][c] = xr[c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e0 + u * stride >= E) break;
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[i][c] += av[u][i] * xv[u][c];
        }
    }
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) acc[i][c] += __shfl_xor(acc[i][c], o);
    if (whole) {
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int c = 0; c < M; ++c) red[wave][i * M + c] = acc[i][c];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int c = 0; c < M; ++c)
                acc[i][c] = (red[0][i * M + c] + red[1][i * M + c]) + (red[2][i * M + c] + red[3][i * M + c]);
    }
    if (!writer) return;
    const int p = lane;
    if (A.unit)
#pragma unroll
        for (int i = 0; i < BR; ++i)
            if (i == p)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[i][c] += xo[c];
    if (MODE == AX_DSCALE) {
        T o[M];
#pragma unroll
        for (int c = 0; c < M; ++c) o[c] = T(0);
#pragma unroll
        for (int jj = 0; jj < BR; ++jj) {
#pragma unroll
            for (int c = 0; c < M; ++c) o[c] += dv[PD ? jj : 0] * acc[jj][c];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            y[row * ld + c] = omega * o[c];
            y2[row * ld + c] = o[c];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < BR; ++i) {
        if (i != p) continue;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T v = acc[i][c];
            if (MODE == B_MINUS) v = bo[PB ? c : 0] - v;
            else if (MODE == S_SWEEP) v = xo[c] + omega * (bo[PB ? c : 0] - v);
            else if (MODE == S_SWEEP_R) {
                const T e = bo[PB ? c : 0] - v;
                y2[row * ld + c] = e;
                v = xo[c] + omega * e;
            }
            y[row * ld + c] = v;
        }
    }
}

static bool bspmv_wide_mode(int mode) {
    return mode == AX || mode == B_MINUS || mode == S_SWEEP || mode == S_SWEEP_R || mode == AX_DSCALE;
}

template <typename T, int M, int BR>
static hipError_t bspmv_wide_mb(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int ld, hipStream_t st,
                                T omega, const T* dinv, T* y2) {
    const int64_t wgs = A.P == 256 ? int64_t(A.n_brow) : (int64_t(A.n_brow) + WAVES_PER_WG - 1) / WAVES_PER_WG;
    if (wgs == 0) return hipSuccess;
    const dim3 grid{unsigned(wgs), 1u, 1u}, block{unsigned(WG), 1u, 1u};
#define WIDE_LAUNCH(MD) hipLaunchKernelGGL((k_bspmv_wide<T, M, MD, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2)
    switch (mode) {
        case AX: WIDE_LAUNCH(AX); break;
        case B_MINUS: WIDE_LAUNCH(B_MINUS); break;
        case S_SWEEP: WIDE_LAUNCH(S_SWEEP); break;
        case S_SWEEP_R: WIDE_LAUNCH(S_SWEEP_R); break;
        case AX_DSCALE: WIDE_LAUNCH(AX_DSCALE); break;
        default: return hipErrorInvalidValue;
    }
#undef WIDE_LAUNCH
    return hipGetLastError();
}

template <typename T, int M>
static hipError_t bspmv_wide_m(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int ld, hipStream_t st,
                               T omega, const T* dinv, T* y2) {
    switch (A.br) {
        case 1: return bspmv_wide_mb<T, M, 1>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 2: return bspmv_wide_mb<T, M, 2>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 3: return bspmv_wide_mb<T, M, 3>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 4: return bspmv_wide_mb<T, M, 4>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int M, int BR>
static hipError_t bsweep_mb(int mode, const Bcsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega,
                            const int32_t* mask, int ld, hipStream_t st, T* y2) {
    const int64_t waves = (A.n_brow + (64 / A.P) - 1) / (64 / A.P);
    if (waves == 0) return hipSuccess;
    dim3 grid(grid_for(waves, WAVES_PER_WG)), block(WG);
    switch (mode) {
        case SWEEP: hipLaunchKernelGGL((k_bsweep<T, M, SWEEP, BR>), grid, block, 0, st, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case SWEEP0: hipLaunchKernelGGL((k_bsweep<T, M, SWEEP0, BR>), grid, block, 0, st, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case RELAX: hipLaunchKernelGGL((k_bsweep<T, M, RELAX, BR>), grid, block, 0, st, A, dinv, x, b, y, omega, mask, ld, y2); break;
        case DINVA: hipLaunchKernelGGL((k_bsweep<T, M, DINVA, BR>), grid, block, 0, st, A, dinv, x, b, y, omega, mask, ld, y2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int M, int BR>
static hipError_t bspmv_mb(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int ld, hipStream_t st,
                           T omega, const T* dinv, T* y2) {
    const int64_t waves = (A.n_brow + (64 / A.P) - 1) / (64 / A.P);
    if (waves == 0) return hipSuccess;
    dim3 grid(grid_for(waves, WAVES_PER_WG)), block(WG);
    switch (mode) {
        case AX: hipLaunchKernelGGL((k_bspmv<T, M, AX, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        case B_MINUS: hipLaunchKernelGGL((k_bspmv<T, M, B_MINUS, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        case B_PLUS: hipLaunchKernelGGL((k_bspmv<T, M, B_PLUS, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        case S_SWEEP: hipLaunchKernelGGL((k_bspmv<T, M, S_SWEEP, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        case S_SWEEP_R: hipLaunchKernelGGL((k_bspmv<T, M, S_SWEEP_R, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        case AX_DSCALE: hipLaunchKernelGGL((k_bspmv<T, M, AX_DSCALE, BR>), grid, block, 0, st, A, x, b, y, ld, omega, dinv, y2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int M>
static hipError_t bsweep_m(int mode, const Bcsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega,
                           const int32_t* mask, int ld, hipStream_t st, T* y2) {
    switch (A.br) {
        case 1: return bsweep_mb<T, M, 1>(mode, A, dinv, x, b, y, omega, mask, ld, st, y2);
        case 2: return bsweep_mb<T, M, 2>(mode, A, dinv, x, b, y, omega, mask, ld, st, y2);
        case 3: return bsweep_mb<T, M, 3>(mode, A, dinv, x, b, y, omega, mask, ld, st, y2);
        case 4: return bsweep_mb<T, M, 4>(mode, A, dinv, x, b, y, omega, mask, ld, st, y2);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int M>
static hipError_t bspmv_m(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int ld, hipStream_t st,
                          T omega, const T* dinv, T* y2) {
    switch (A.br) {
        case 1: return bspmv_mb<T, M, 1>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 2: return bspmv_mb<T, M, 2>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 3: return bspmv_mb<T, M, 3>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        case 4: return bspmv_mb<T, M, 4>(mode, A, x, b, y, ld, st, omega, dinv, y2);
        default: return hipErrorInvalidValue;
    }
}

// chunk width of the block-CSR kernels: up to 16 columns per launch, bounded
// by `cap` (1, 2, 4, 8 or 16; 0: 16); it does not change any column's arithmetic
static int bcsr_chunk(int rem, int cap) {
    const int c = cap > 0 ? cap : 16;
    int w = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem;
    while (w > c) w = w == 16 ? 8 : w == 8 ? 4 : w >= 4 ? 2 : 1;
    return w;
}

template <typename T>
hipError_t launch_bsweep(int mode, const Bcsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                         const int32_t* colmask, hipStream_t st, int cap, T* y2) {
    if (A.P > 64) {
        // the sweeps with D^{-1} take whole blocks per lane (64 lanes) on any layout
        Bcsr<T> A64 = A;
        A64.P = 64;
        return launch_bsweep<T>(mode, A64, dinv, x, b, y, omega, m, colmask, st, cap, y2);
    }
    int c0 = 0;
    while (c0 < m) {
        const int w = bcsr_chunk(m - c0, cap);
        const T* xc = x ? x + c0 : nullptr;
        const T* bc = b ? b + c0 : nullptr;
        const int32_t* mc = colmask ? colmask + c0 : nullptr;
        T* y2c = y2 ? y2 + c0 : nullptr;
        hipError_t e;
        switch (w) {
            case 16: e = bsweep_m<T, 16>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 8: e = bsweep_m<T, 8>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 4: e = bsweep_m<T, 4>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 3: e = bsweep_m<T, 3>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            case 2: e = bsweep_m<T, 2>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
            default: e = bsweep_m<T, 1>(mode, A, dinv, xc, bc, y + c0, omega, mc, m, st, y2c); break;
        }
        if (e != hipSuccess) return e;
        c0 += w;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_bspmv(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int m, hipStream_t st, int cap,
                        T omega, const T* dinv, T* y2) {
    if (mode == S_SWEEP_R && !y2) return hipErrorInvalidValue;
    if (A.P > 64 && bspmv_wide_mode(mode)) {
        // entry-wise lanes: up to 8 columns per launch
        int c0 = 0;
        while (c0 < m) {
            int w = bcsr_chunk(m - c0, cap);
            w = w >= 8 ? 8 : w >= 4 ? 4 : w >= 2 ? 2 : 1;
            const T* bc = b ? b + c0 : nullptr;
            T* y2c = y2 ? y2 + c0 : nullptr;
            hipError_t e;
            switch (w) {
                case 8: e = bspmv_wide_m<T, 8>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2c); break;
                case 4: e = bspmv_wide_m<T, 4>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2c); break;
                case 2: e = bspmv_wide_m<T, 2>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2c); break;
                default: e = bspmv_wide_m<T, 1>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2c); break;
            }
            if (e != hipSuccess) return e;
            c0 += w;
        }
        return hipSuccess;
    }
    if (A.P > 64) {
        // a mode the entry-wise kernel does not take: whole blocks per lane, 64 lanes
        Bcsr<T> A64 = A;
        A64.P = 64;
        return launch_bspmv<T>(mode, A64, x, b, y, m, st, cap, omega, dinv, y2);
    }
    int c0 = 0;
    while (c0 < m) {
        const int w = bcsr_chunk(m - c0, cap);
        const T* bc = b ? b + c0 : nullptr;
        hipError_t e;
        switch (w) {
            case 16: e = bspmv_m<T, 16>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
            case 8: e = bspmv_m<T, 8>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
            case 4: e = bspmv_m<T, 4>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
            case 3: e = bspmv_m<T, 3>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
            case 2: e = bspmv_m<T, 2>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
            default: e = bspmv_m<T, 1>(mode, A, x + c0, bc, y + c0, m, st, omega, dinv, y2 ? y2 + c0 : nullptr); break;
        }
        if (e != hipSuccess) return e;
        c0 += w;
    }
    return hipSuccess;
}

template hipError_t launch_bsweep<double>(int, const Bcsr<double>&, const double*, const double*, const double*,
                                          double*, double, int, const int32_t*, hipStream_t, int, double*);
template hipError_t launch_bsweep<float>(int, const Bcsr<float>&, const float*, const float*, const float*, float*,
                                         float, int, const int32_t*, hipStream_t, int, float*);
template hipError_t launch_bspmv<double>(int, const Bcsr<double>&, const double*, const double*, double*, int,
                                         hipStream_t, int, double, const double*, double*);
template hipError_t launch_bspmv<float>(int, const Bcsr<float>&, const float*, const float*, float*, int,
                                        hipStream_t, int, float, const float*, float*);

// ============================================================ MFMA tiles
// Lane layout of the 16x16x4 matrix instructions (wave64), as measured on
// gfx950: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it receives
// D[4 (l / 16) + v][l % 16] (FP32) or D[l / 16 + 4 v][l % 16] (FP64), v = 0..3.

template <typename T>
struct Mma;
template <>
struct Mma<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mma<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// One wavefront per block row, one 16-column tile per blockIdx.y.  Block
// (brow, col) contributes A_blk (br x bc, zero-padded to 16 x 4t) times the
// x block rows col*bc .. col*bc + bc - 1 of the tile; lanes l / 16 = g take
// k = 4t + g, so each step loads 16 consecutive x values per k.  The operand
// fragments of up to U blocks are loaded before their products, and the
// epilogue's b, x and D^{-1} fragments before the block loop, so that a
// wavefront keeps several blocks' loads in flight.
template <typename T, int MODE, int U>
__global__ __launch_bounds__(WG) void k_mfma(Nbsr<T> A, const T* __restrict__ dinv, const T* __restrict__ x,
                                             const T* __restrict__ b, T* __restrict__ y, T omega, int ld,
                                             T* __restrict__ y2) {
    __shared__ T tile[WAVES_PER_WG][16][17];
    __shared__ T red[WAVES_PER_WG][16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int brow = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_WG + wave);
    if (brow >= A.n_brow) {
        // MF_AXDOT: a wavefront past the last block row adds zero to its
        // workgroup's partials (the first wavefront of a workgroup always has a row)
        if (MODE == MF_AXDOT) {
            if (lane < 16) red[wave][lane] = T(0);
            __syncthreads();
        }
        return;
    }
    const int i = lane & 15, g = lane >> 4;
    const int br = A.br, bc = A.bc;
    const int64_t col0 = int64_t(blockIdx.y) * MFMA_COLS + i;
    const int64_t r0 = int64_t(brow) * br;
    constexpr bool SW = (MODE == MF_SWEEP || MODE == MF_SWEEP0 || MODE == MF_RDINV);
    // epilogue operands first
    T bpre[4], xpre[4], dpre[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = Mma<T>::row(g, v);
        const int64_t e = (r0 + row) * ld + col0;
        bpre[v] = (MODE != MF_AX && MODE != MF_RDINV && row < br) ? b[e] : T(0);
        xpre[v] = ((MODE == MF_SWEEP || MODE == MF_SSWEEP || MODE == MF_SSWEEP_R || MODE == MF_AXDOT || A.unit) &&
                   row < br)
                      ? x[e]
                      : T(0);
    }
    if (SW) {
        const T* __restrict__ Db = dinv + int64_t(brow) * br * br;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + g;
            dpre[t] = (i < br && k < br) ? Db[i * br + k] : T(0);
        }
    }
    typename Mma<T>::acc acc = {T(0), T(0), T(0), T(0)};
    if (MODE != MF_SWEEP0) {
        const int kt = (bc + 3) >> 2;
        const int beg = A.rp[brow], end = A.rp[brow + 1];
        for (int blk = beg; blk < end; blk += U) {
            T av[U][4], xv[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool on = blk + u < end;
                const int bq = on ? blk + u : blk;
                const T* __restrict__ Ab = A.vals + int64_t(bq) * br * bc;
                const T* __restrict__ Xb = x + int64_t(A.ci[bq]) * bc * ld + col0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 4 * t + g;
                    av[u][t] = (on && t < kt && i < br && k < bc) ? Ab[i * bc + k] : T(0);
                    xv[u][t] = (on && t < kt && k < bc) ? Xb[int64_t(k) * ld] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (blk + u < end) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < kt) acc = Mma<T>::step(av[u][t], xv[u][t], acc);
                }
        }
    }
    if (!SW) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = Mma<T>::row(g, v);
            if (row < br) {
                T val = A.unit ? acc[v] + xpre[v] : acc[v];
                if (MODE == MF_BMINUS) val = bpre[v] - val;
                if (MODE == MF_BPLUS) val = bpre[v] + val;
                if (MODE == MF_SSWEEP) val = xpre[v] + omega * (bpre[v] - val);
                if (MODE == MF_SSWEEP_R) {
                    const T e = bpre[v] - val;
                    y2[(r0 + row) * ld + col0] = e;
                    val = xpre[v] + omega * e;
                }
                y[(r0 + row) * ld + col0] = val;
            }
        }
        if (MODE == MF_AXDOT) {
            // x . (A x) of column i over this block row: the lane's rows, then the
            // four lanes of column i; then the workgroup's four block rows in order
            T s = T(0);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (Mma<T>::row(g, v) < br) s += xpre[v] * (A.unit ? acc[v] + xpre[v] : acc[v]);
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (lane < 16) red[wave][lane] = s;
            __syncthreads();
            if (wave == 0 && lane < 16)
                y2[int64_t(lane) * gridDim.x + blockIdx.x] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        }
        return;
    }
    // residual tile (rows >= br are zero) through LDS into the B operand of D^{-1} R
    T(*tl)[17] = tile[wave];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = Mma<T>::row(g, v);
        tl[row][i] = (row < br) ? ((MODE == MF_SWEEP) ? bpre[v] - acc[v] : (MODE == MF_RDINV) ? acc[v] : bpre[v]) : T(0);
    }
    wave_lds_sync();
    typename Mma<T>::acc acc2 = {T(0), T(0), T(0), T(0)};
    const int kd = (br + 3) >> 2;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (t < kd) acc2 = Mma<T>::step(dpre[t], tl[4 * t + g][i], acc2);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = Mma<T>::row(g, v);
        if (row < br) {
            y[(r0 + row) * ld + col0] = xpre[v] + omega * acc2[v];
            if ((MODE == MF_SWEEP0 || MODE == MF_RDINV) && y2) y2[(r0 + row) * ld + col0] = acc2[v];
        }
    }
}

// The products without D^{-1} (MF_AX, MF_BMINUS, MF_BPLUS, MF_SSWEEP,
// MF_SSWEEP_R) and the restriction MF_RDINV (D'^{-1} of the output rows applied
// to the result tile, row by row) with their operands staged through
// wavefront-private LDS by
// 16-byte loads: a chunk of B consecutive blocks of a block row
// (mfma_v_blocks: 6 blocks of 10 x 10 or 16 of 4 x 4 at U = 4) is one
// contiguous run of values, and each block's x rows hold the tile's 16
// columns contiguously, so a wavefront
// reads them with a few vector loads instead of one 4-byte load per lane per
// operand and k step (the tiles' address processing, not HBM, limited the
// 16-column sweep).  The accumulator tile returns through LDS to row-major
// order, so the epilogue's b, x, y and y2 move 16 bytes per lane as well.  The
// products are those of k_mfma, in the same order.  On the 16-column 3D
// workload the FP32 sweep went from 1367 us to 1306-1338 us and the V-cycle
// from 12.6 ms to 12.0-12.4 ms (three runs); the address unit's busy share
// (83% of the sweep's cycles with per-lane loads) had suggested more.
// LDS per wavefront: mfma_v_lds values.
// values of LDS per wavefront: B blocks, their x rows, the 16 x 17 result tile
// and one spare vector, rounded up to whole 16-byte vectors
__host__ __device__ constexpr int mfma_v_lds(int B, int per, int xper, int VW) {
    return (B * (per + xper) + MFMA_COLS * 17 + VW + VW - 1) / VW * VW;
}

// Blocks staged per chunk: as many as the U * 16 * 16 values of operand and
// of x rows a lane's registers hold at most (NL vectors per lane each), and at
// most 64 (one column index per lane): 16 blocks of 4 x 4, 6 of 10 x 10 at U = 4.
__host__ __device__ constexpr int mfma_v_blocks(int U, int br, int bc, int VW) {
    const int nl64 = 64 * (U * NBSR_MAXB * NBSR_MAXB / (VW * 64));
    const int by_a = nl64 / (br * bc / VW);
    const int by_x = nl64 / (bc * (MFMA_COLS / VW));
    const int b = by_a < by_x ? by_a : by_x;
    return b < 1 ? 1 : b > 64 ? 64 : b;
}

template <typename T, int N>
struct ExtVec {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T, int MODE, int U>
__global__ __launch_bounds__(WG) void k_mfma_v(Nbsr<T> A, const T* __restrict__ dinv, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, T omega, int ld,
                                               T* __restrict__ y2, int B) {
    constexpr int VW = 16 / int(sizeof(T));
    using V = typename ExtVec<T, VW>::type;
    constexpr int LPR = MFMA_COLS / VW;         // lanes per 16-column row: 4 (FP32), 8 (FP64)
    constexpr int RPP = 64 / LPR;               // rows per epilogue pass: 16, 8
    constexpr int NP = (MFMA_COLS + RPP - 1) / RPP;
    constexpr int NL = U * NBSR_MAXB * NBSR_MAXB / (VW * 64);  // vector loads per lane and operand, at most
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int brow = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_WG + wave);
    if (brow >= A.n_brow) return;
    const int br = A.br, bc = A.bc;
    const int per = br * bc, xper = bc * MFMA_COLS;
    T* sA = reinterpret_cast<T*>(smem_raw) + int64_t(wave) * mfma_v_lds(B, per, xper, VW);
    T* sX = sA + B * per;
    T* sY = sX + B * xper;
    const int i = lane & 15, g = lane >> 4;
    const int64_t tile0 = int64_t(blockIdx.y) * MFMA_COLS;
    const int64_t r0 = int64_t(brow) * br;
    // epilogue operands first, row-major: lane (er, eq) holds columns eq*VW.. of rows er + p*RPP
    const int er = lane / LPR, eq = lane - (lane / LPR) * LPR;
    constexpr bool NB = (MODE == MF_BMINUS || MODE == MF_BPLUS || MODE == MF_SSWEEP || MODE == MF_SSWEEP_R);
    const bool nx = MODE == MF_SSWEEP || MODE == MF_SSWEEP_R || A.unit;
    V bo[NP], xo[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int row = er + p * RPP;
        const int64_t e = (r0 + (row < br ? row : br - 1)) * ld + tile0 + eq * VW;  // clamped: loads stay unconditional
        bo[p] = V(T(0));
        xo[p] = V(T(0));
        (void)e;
        if (NB) {
            const V t = *reinterpret_cast<const V*>(b + e);
            bo[p] = row < br ? t : V(T(0));
        }
        if (nx) {
            const V t = *reinterpret_cast<const V*>(x + e);
            xo[p] = row < br ? t : V(T(0));
        }
    }
    // MF_RDINV: row er (+ p RPP) of the output rows' D'^{-1} block (br <= 16)
    T dr[MODE == MF_RDINV ? NP : 1][MODE == MF_RDINV ? NBSR_MAXB : 1];
    if (MODE == MF_RDINV) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int row = er + p * RPP;
            const T* __restrict__ dp = dinv + (r0 + (row < br ? row : br - 1)) * br;
#pragma unroll
            for (int j = 0; j < NBSR_MAXB; ++j) dr[p][j] = j < br ? dp[j] : T(0);
        }
    }
    typename Mma<T>::acc acc = {T(0), T(0), T(0), T(0)};
    const int beg = A.rp[brow], end = A.rp[brow + 1];
    const int kt = (bc + 3) >> 2;
    for (int blk = beg; blk < end; blk += B) {
        const int nbu = min(B, end - blk);
        // lane l holds the column of the chunk's block l (B <= 64)
        const int32_t cl = A.ci[blk + (lane < nbu ? lane : nbu - 1)];
        // the chunk's blocks (contiguous) and their x rows, all loads issued first
        const V* __restrict__ ag = reinterpret_cast<const V*>(A.vals + int64_t(blk) * per);
        const int nva = nbu * per / VW, nvx = nbu * bc * LPR;
        // indices clamped to the last vector, so every load is unconditional;
        // the surplus lanes write to a spare slot after the tile
        V ra[NL], rx[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int v = lane + 64 * j;
            ra[j] = ag[v < nva ? v : nva - 1];
            const int vx = v < nvx ? v : nvx - 1;
            const int u = vx / (bc * LPR);
            const int rem = vx - u * (bc * LPR);
            const int k = rem / LPR, q = rem - (rem / LPR) * LPR;
            const int32_t c = __shfl(cl, u);
            rx[j] = *reinterpret_cast<const V*>(x + (int64_t(c) * bc + k) * ld + tile0 + q * VW);
        }
        V* const spare = reinterpret_cast<V*>(sY + MFMA_COLS * 17);
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int v = lane + 64 * j;
            *(v < nva ? reinterpret_cast<V*>(sA) + v : spare) = ra[j];
            *(v < nvx ? reinterpret_cast<V*>(sX) + v : spare) = rx[j];
        }
        wave_lds_sync();
        for (int u = 0; u < nbu; ++u) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= kt) break;
                const int k = 4 * t + g;
                const T av = (i < br && k < bc) ? sA[u * per + i * bc + k] : T(0);
                const T xv = (k < bc) ? sX[(u * bc + k) * MFMA_COLS + i] : T(0);
                acc = Mma<T>::step(av, xv, acc);
            }
        }
        wave_lds_sync();  // the next chunk overwrites sA and sX
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sY[Mma<T>::row(g, v) * 17 + i] = acc[v];
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int row = er + p * RPP;
        if (row >= br) break;
        const V bv = bo[p], xv = xo[p];
        V o, e2 = V(T(0));
        if (MODE == MF_RDINV) {
            // o = D'^{-1} (the tile's column), y = omega o, y2 = o
#pragma unroll
            for (int w = 0; w < VW; ++w) {
                T v = T(0);
#pragma unroll
                for (int j = 0; j < NBSR_MAXB; ++j)
                    if (j < br) v += dr[p][j] * sY[j * 17 + eq * VW + w];
                e2[w] = v;
                o[w] = omega * v;
            }
            const int64_t e = (r0 + row) * ld + tile0 + eq * VW;
            *reinterpret_cast<V*>(y + e) = o;
            *reinterpret_cast<V*>(y2 + e) = e2;
            continue;
        }
#pragma unroll
        for (int w = 0; w < VW; ++w) {
            T val = sY[row * 17 + eq * VW + w];
            if (A.unit) val += xv[w];
            if (MODE == MF_BMINUS) val = bv[w] - val;
            if (MODE == MF_BPLUS) val = bv[w] + val;
            if (MODE == MF_SSWEEP) val = xv[w] + omega * (bv[w] - val);
            if (MODE == MF_SSWEEP_R) {
                e2[w] = bv[w] - val;
                val = xv[w] + omega * e2[w];
            }
            o[w] = val;
        }
        const int64_t e = (r0 + row) * ld + tile0 + eq * VW;
        *reinterpret_cast<V*>(y + e) = o;
        if (MODE == MF_SSWEEP_R) *reinterpret_cast<V*>(y2 + e) = e2;
    }
}

template <typename T>
static bool mfma_v_ok(int mode, const Nbsr<T>& A, const T* x, const T* b, const T* y, int ld) {
    constexpr int VW = 16 / int(sizeof(T));
    auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    // FP32, and FP64 for blocks of at most 16 values (coarse levels of 4 x 4 blocks, whose long rows
    // the staged form takes 16 blocks at a time): in FP64 the staged form measured slower on
    // 10 x 10 blocks (the 16-column 3D sweep 2.61 ms against 2.40 ms)
    return (sizeof(T) == 4 || A.br * A.bc <= 16) &&
           (mode == MF_AX || mode == MF_BMINUS || mode == MF_BPLUS || mode == MF_SSWEEP || mode == MF_SSWEEP_R ||
            mode == MF_RDINV) &&
           (A.br * A.bc) % VW == 0 && ld % VW == 0 && al(A.vals) && al(x) && al(y) && (!b || al(b));
}

template <typename T, int U>
static hipError_t mfma_u(int mode, const Nbsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                         hipStream_t st, T* y2) {
    // U = 3 exists for the staged tiles only (a chunk of four 10 x 10 blocks, a
    // whole level-0 row of the 3D tetrahedra); the per-lane tiles take 2 there
    if constexpr (U == 3) {
        if (!mfma_v_ok<T>(mode, A, x, b, y, m)) return mfma_u<T, 2>(mode, A, dinv, x, b, y, omega, m, st, y2);
    }
    if (mfma_v_ok<T>(mode, A, x, b, y, m) &&
        ((mode != MF_SSWEEP_R && mode != MF_RDINV) || (reinterpret_cast<uintptr_t>(y2) & 15) == 0)) {
        dim3 grid(grid_for(A.n_brow, WAVES_PER_WG), m / MFMA_COLS), block(WG);
        constexpr int VW = 16 / int(sizeof(T));
        const int B = mfma_v_blocks(U, A.br, A.bc, VW);
        const size_t lds = size_t(WAVES_PER_WG) * mfma_v_lds(B, A.br * A.bc, A.bc * MFMA_COLS, VW) * sizeof(T);
        if (lds <= lds_limit()) {
#define MFV_LAUNCH(MD) hipLaunchKernelGGL((k_mfma_v<T, MD, U>), grid, block, lds, st, A, dinv, x, b, y, omega, m, y2, B)
            switch (mode) {
                case MF_AX: MFV_LAUNCH(MF_AX); break;
                case MF_BMINUS: MFV_LAUNCH(MF_BMINUS); break;
                case MF_BPLUS: MFV_LAUNCH(MF_BPLUS); break;
                case MF_SSWEEP: MFV_LAUNCH(MF_SSWEEP); break;
                case MF_RDINV: MFV_LAUNCH(MF_RDINV); break;
                default: MFV_LAUNCH(MF_SSWEEP_R); break;
            }
#undef MFV_LAUNCH
            return hipGetLastError();
        }
    }
    if constexpr (U == 3) {
        return mfma_u<T, 2>(mode, A, dinv, x, b, y, omega, m, st, y2);
    } else {
    dim3 grid(grid_for(A.n_brow, WAVES_PER_WG), m / MFMA_COLS), block(WG);
    switch (mode) {
        case MF_AX: hipLaunchKernelGGL((k_mfma<T, MF_AX, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_BMINUS: hipLaunchKernelGGL((k_mfma<T, MF_BMINUS, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_BPLUS: hipLaunchKernelGGL((k_mfma<T, MF_BPLUS, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_SWEEP: hipLaunchKernelGGL((k_mfma<T, MF_SWEEP, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_SWEEP0: hipLaunchKernelGGL((k_mfma<T, MF_SWEEP0, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_SSWEEP: hipLaunchKernelGGL((k_mfma<T, MF_SSWEEP, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_RDINV: hipLaunchKernelGGL((k_mfma<T, MF_RDINV, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2); break;
        case MF_SSWEEP_R:
            if (!y2) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_mfma<T, MF_SSWEEP_R, U>), grid, block, 0, st, A, dinv, x, b, y, omega, m, y2);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
    }
}

template <typename T>
hipError_t launch_mfma(int mode, const Nbsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                       hipStream_t st, int u, T* y2) {
    if (A.n_brow == 0) return hipSuccess;
    if (m % MFMA_COLS != 0 || A.br > NBSR_MAXB || A.bc > NBSR_MAXB) return hipErrorInvalidValue;
    switch (u) {
        case 1: return mfma_u<T, 1>(mode, A, dinv, x, b, y, omega, m, st, y2);
        case 2: return mfma_u<T, 2>(mode, A, dinv, x, b, y, omega, m, st, y2);
        case 3: return mfma_u<T, 3>(mode, A, dinv, x, b, y, omega, m, st, y2);
        default: return mfma_u<T, 4>(mode, A, dinv, x, b, y, omega, m, st, y2);
    }
}
template hipError_t launch_mfma<float>(int, const Nbsr<float>&, const float*, const float*, const float*, float*,
                                       float, int, hipStream_t, int, float*);
template hipError_t launch_mfma<double>(int, const Nbsr<double>&, const double*, const double*, const double*,
                                        double*, double, int, hipStream_t, int, double*);

// ============================================================ layout conversion

// one thread per (slot q, i, j): t = k*bc + j goes to
// vals[base + (t / VW) * L * VW + (g*br + i) * VW + t % VW]
template <typename T>
__global__ void k_to_sell_vals(const double* __restrict__ nat, const int64_t* __restrict__ src,
                               const int64_t* __restrict__ base, const int32_t* __restrict__ sk,
                               const int32_t* __restrict__ sg, int64_t n_slots, int L, int br, int bc,
                               T* __restrict__ vals) {
    constexpr int VW = 16 / int(sizeof(T));
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(br) * bc;
    if (tid >= n_slots * per) return;
    const int64_t q = tid / per;
    const int rem = int(tid - q * per);
    const int i = rem / bc, j = rem - (rem / bc) * bc;
    const int64_t s = src[q];
    if (s < 0) return;  // padding slot: the buffer was zeroed
    const int t = sk[q] * bc + j;
    vals[base[q] + int64_t(t / VW) * L * VW + int64_t(sg[q] * br + i) * VW + t % VW] = T(nat[s * per + int64_t(i) * bc + j]);
}

template <typename T>
hipError_t launch_to_sell_vals(const double* nat, const int64_t* src, const int64_t* base, const int32_t* sk,
                               const int32_t* sg, int64_t n_slots, int L, int br, int bc, T* vals, hipStream_t st) {
    const int64_t tot = n_slots * br * bc;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL((k_to_sell_vals<T>), dim3(grid_for(tot)), dim3(WG), 0, st, nat, src, base, sk, sg, n_slots, L,
                       br, bc, vals);
    return hipGetLastError();
}
template hipError_t launch_to_sell_vals<double>(const double*, const int64_t*, const int64_t*, const int32_t*,
                                                const int32_t*, int64_t, int, int, int, double*, hipStream_t);
template hipError_t launch_to_sell_vals<float>(const double*, const int64_t*, const int64_t*, const int32_t*,
                                               const int32_t*, int64_t, int, int, int, float*, hipStream_t);

template <typename T>
__global__ void k_dinv_to_sell(const double* __restrict__ dn, int64_t n_brow, int br, int G, int L, int BP,
                               T* __restrict__ ds, const int32_t* __restrict__ pos) {
    constexpr int VW = 16 / int(sizeof(T));
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(br) * br;
    if (t >= n_brow * per) return;
    const int64_t e = t / per;
    const int rem = int(t - e * per);
    const int i = rem / br, j = rem - (rem / br) * br;
    const int64_t q = pos ? int64_t(pos[e]) : e;
    const int64_t s = q / G;
    const int g = int(q - s * G);
    ds[s * BP * L + int64_t(j / VW) * L * VW + int64_t(g * br + i) * VW + j % VW] = T(dn[t]);
}

template <typename T>
hipError_t launch_dinv_to_sell(const double* dn, int64_t n_brow, int br, int G, int L, int BP, T* ds, hipStream_t st,
                               const int32_t* pos) {
    const int64_t tot = n_brow * br * br;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL((k_dinv_to_sell<T>), dim3(grid_for(tot)), dim3(WG), 0, st, dn, n_brow, br, G, L, BP, ds, pos);
    return hipGetLastError();
}
template hipError_t launch_dinv_to_sell<double>(const double*, int64_t, int, int, int, int, double*, hipStream_t,
                                                const int32_t*);
template hipError_t launch_dinv_to_sell<float>(const double*, int64_t, int, int, int, int, float*, hipStream_t,
                                               const int32_t*);

template <typename Ti, typename To>
__global__ void k_convert(const Ti* __restrict__ a, To* __restrict__ b, int64_t n) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) b[t] = To(a[t]);  // double -> float rounds to nearest even
}

template <typename Ti, typename To>
hipError_t launch_convert(const Ti* in, To* out, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<Ti, To>), dim3(grid_for(n)), dim3(WG), 0, st, in, out, n);
    return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_convert<float, float>(const float*, float*, int64_t, hipStream_t);

hipError_t launch_f64_to_f32(const double* a, float* b, int64_t n, hipStream_t st) {
    return launch_convert<double, float>(a, b, n, st);
}

// ============================================================ block inverse
// Batched Gauss-Jordan with partial pivoting (LAPACK-style pivot choice: the
// largest magnitude, the lowest row on ties).  One lane holds one row of the
// augmented block [D | I]; floor(64/nb) blocks per wavefront; nb <= 16.
constexpr int MAXB = 16;

__global__ __launch_bounds__(WG) void k_block_inverse(const double* __restrict__ Av, const int32_t* __restrict__ dpos,
                                                      int64_t n_brow, int nb, double* __restrict__ dinv,
                                                      int32_t* __restrict__ flag) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int G = 64 / nb;
    const int L = G * nb;
    const int lc = lane < L ? lane : L - 1;
    const int g = lc / nb, i = lc - g * nb;
    const int64_t blk = (int64_t(blockIdx.x) * WAVES_PER_WG + wave) * G + g;
    const bool own = lane < L && blk < n_brow;
    const int base = g * nb;
    double a[MAXB], v[MAXB];
    const double* src = own ? Av + int64_t(dpos[blk]) * nb * nb + int64_t(i) * nb : nullptr;
    double amax = 0.0;
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        a[q] = (own && q < nb) ? src[q] : 0.0;
        v[q] = (q == i) ? 1.0 : 0.0;
        amax = fmax(amax, fabs(a[q]));
    }
    for (int j = 0; j < nb; ++j) amax = fmax(amax, __shfl(amax, base + j));
    const double tol = nb * DBL_EPSILON * amax;
    bool singular = (amax == 0.0);
    for (int c = 0; c < nb; ++c) {
        double ac = 0.0;
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q == c) ac = a[q];
        // pivot row p >= c of largest |a[p][c]|
        int p = c;
        double best = -1.0;
        for (int j = c; j < nb; ++j) {
            const double val = fabs(__shfl(ac, base + j));
            if (val > best) { best = val; p = j; }
        }
        // swap rows c and p
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const double ap = __shfl(a[q], base + p), acq = __shfl(a[q], base + c);
            const double vp = __shfl(v[q], base + p), vcq = __shfl(v[q], base + c);
            if (i == c) { a[q] = ap; v[q] = vp; }
            else if (i == p) { a[q] = acq; v[q] = vcq; }
        }
        double acol = 0.0;
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q == c) acol = a[q];
        const double piv = __shfl(acol, base + c);
        if (!(fabs(piv) > tol)) singular = true;
        const double inv = 1.0 / piv;
        double rc[MAXB], vc[MAXB];
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            rc[q] = __shfl(a[q], base + c) * inv;
            vc[q] = __shfl(v[q], base + c) * inv;
        }
        if (i == c) {
#pragma unroll
            for (int q = 0; q < MAXB; ++q) { a[q] = rc[q]; v[q] = vc[q]; }
        } else {
            const double f = acol;
#pragma unroll
            for (int q = 0; q < MAXB; ++q) { a[q] -= f * rc[q]; v[q] -= f * vc[q]; }
        }
    }
    if (!own) return;
    if (singular) atomicOr(flag, 1);
    double* dst = dinv + blk * nb * nb + int64_t(i) * nb;
#pragma unroll
    for (int q = 0; q < MAXB; ++q)
        if (q < nb) dst[q] = v[q];
}

// Blocks of 17..64 rows: one wavefront per block, the block in LDS (row
// stride 65), lane i owns row i.  In-place Gauss-Jordan with the same pivot
// choice (largest magnitude, lowest row on ties): the pivot row is swapped
// into place, scaled by the pivot's reciprocal (which takes the pivot's
// position), every other row subtracts its multiple of it (its pivot-column
// entry becoming -f times the reciprocal); the row swaps are undone as column
// swaps of the inverse at the end.
constexpr int MAXB_LDS = 64;

__global__ __launch_bounds__(64) void k_block_inverse_lds(const double* __restrict__ Av,
                                                          const int32_t* __restrict__ dpos, int64_t n_brow, int nb,
                                                          double* __restrict__ dinv, int32_t* __restrict__ flag) {
    __shared__ double a[MAXB_LDS][MAXB_LDS + 1];
    __shared__ int piv[MAXB_LDS];
    const int i = threadIdx.x;
    const int64_t blk = blockIdx.x;
    if (blk >= n_brow) return;
    const double* src = Av + int64_t(dpos[blk]) * nb * nb;
    double amax = 0.0;
    if (i < nb)
        for (int q = 0; q < nb; ++q) {
            a[i][q] = src[int64_t(i) * nb + q];
            amax = fmax(amax, fabs(a[i][q]));
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    const double tol = nb * DBL_EPSILON * amax;
    bool singular = (amax == 0.0);
    wave_lds_sync();
    for (int c = 0; c < nb; ++c) {
        // pivot row p >= c of largest |a[p][c]|, lowest p on ties
        double v = (i >= c && i < nb) ? fabs(a[i][c]) : -1.0;
        int p = i;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ov = __shfl_xor(v, o);
            const int op = __shfl_xor(p, o);
            if (ov > v || (ov == v && op < p)) { v = ov; p = op; }
        }
        if (i == 0) piv[c] = p;
        if (p != c && i < nb) {
            const double t = a[c][i];
            a[c][i] = a[p][i];
            a[p][i] = t;
        }
        wave_lds_sync();
        const double pv = a[c][c];
        if (!(fabs(pv) > tol)) singular = true;
        const double inv = 1.0 / pv;
        double f = 0.0;
        if (i < nb && i != c) f = a[i][c];
        wave_lds_sync();
        if (i < nb) a[c][i] = (i == c) ? inv : a[c][i] * inv;
        wave_lds_sync();
        if (i < nb && i != c) {
            for (int q = 0; q < nb; ++q)
                a[i][q] = (q == c) ? -f * inv : a[i][q] - f * a[c][q];
        }
        wave_lds_sync();
    }
    // undo the row swaps as column swaps, last first
    for (int c = nb - 1; c >= 0; --c) {
        const int p = piv[c];
        if (p != c && i < nb) {
            const double t = a[i][c];
            a[i][c] = a[i][p];
            a[i][p] = t;
        }
    }
    if (singular && i == 0) atomicOr(flag, 1);
    if (i < nb) {
        double* dst = dinv + blk * nb * nb + int64_t(i) * nb;
        for (int q = 0; q < nb; ++q) dst[q] = a[i][q];
    }
}

hipError_t launch_block_inverse(const double* Av, const int32_t* dpos, int64_t n_brow, int nb, double* dinv,
                                int32_t* flag, hipStream_t st) {
    if (nb > MAXB && nb <= MAXB_LDS) {
        if (n_brow == 0) return hipSuccess;
        hipLaunchKernelGGL(k_block_inverse_lds, dim3(unsigned(n_brow)), dim3(64), 0, st, Av, dpos, n_brow, nb, dinv,
                           flag);
        return hipGetLastError();
    }
    if (nb < 1 || nb > MAXB) return hipErrorInvalidValue;
    const int G = 64 / nb;
    const int64_t waves = (n_brow + G - 1) / G;
    if (waves == 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_inverse, dim3(grid_for(waves, WAVES_PER_WG)), dim3(WG), 0, st, Av, dpos, n_brow, nb,
                       dinv, flag);
    return hipGetLastError();
}

// ============================================================ SVD (one-sided Jacobi)
// One wavefront per aggregate J.  The rows of J are the contiguous dofs
// [first_child[J] * nb, first_child[J+1] * nb) of B (row-major, r columns).
// Lanes hold rows lane and lane + 64 (<= 128 rows), r <= 16 columns.  Hestenes'
// one-sided Jacobi rotates column pairs until they are orthogonal to working
// precision; the singular values are the column norms and the left singular
// vectors the normalised columns.  Output: the leading s columns (descending
// singular values), each flipped so its largest-magnitude entry (lowest row on
// ties) is positive, written to Pu (row-major n x s), and all r singular values.
constexpr int SVD_MAXR = 16;
constexpr int SVD_MAXROWS = 128;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(WG) void k_svd(const double* __restrict__ B, int r, const int32_t* __restrict__ fc,
                                            int64_t n_agg, int nb, int s, double* __restrict__ Pu,
                                            double* __restrict__ sv, int32_t* __restrict__ flag) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t J = int64_t(blockIdx.x) * WAVES_PER_WG + wave;
    if (J >= n_agg) return;
    const int64_t r0 = int64_t(fc[J]) * nb;
    const int nrows = int(int64_t(fc[J + 1]) * nb - r0);
    if (nrows > SVD_MAXROWS) { if (lane == 0) atomicOr(flag, 2); return; }
    double m0[SVD_MAXR], m1[SVD_MAXR];
    const bool h0 = lane < nrows, h1 = lane + 64 < nrows;
#pragma unroll
    for (int c = 0; c < SVD_MAXR; ++c) {
        m0[c] = (h0 && c < r) ? B[(r0 + lane) * r + c] : 0.0;
        m1[c] = (h1 && c < r) ? B[(r0 + lane + 64) * r + c] : 0.0;
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < SVD_MAXR; ++p) {
#pragma unroll
            for (int q = p + 1; q < SVD_MAXR; ++q) {
                if (q >= r) continue;
                const double al = wave_sum(m0[p] * m0[p] + m1[p] * m1[p]);
                const double be = wave_sum(m0[q] * m0[q] + m1[q] * m1[q]);
                const double ga = wave_sum(m0[p] * m0[q] + m1[p] * m1[q]);
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                const double a0 = m0[p], b0 = m0[q], a1 = m1[p], b1 = m1[q];
                m0[p] = cs * a0 - sn * b0;
                m0[q] = sn * a0 + cs * b0;
                m1[p] = cs * a1 - sn * b1;
                m1[q] = sn * a1 + cs * b1;
            }
        }
        if (!rotated) break;
    }
    double sig[SVD_MAXR];
#pragma unroll
    for (int c = 0; c < SVD_MAXR; ++c) sig[c] = (c < r) ? sqrt(wave_sum(m0[c] * m0[c] + m1[c] * m1[c])) : -1.0;
#pragma unroll
    for (int c = 0; c < SVD_MAXR; ++c) {
        if (c >= r) continue;
        int rank = 0;
#pragma unroll
        for (int q = 0; q < SVD_MAXR; ++q)
            if (q < r && (sig[q] > sig[c] || (sig[q] == sig[c] && q < c))) ++rank;
        if (lane == 0) sv[J * r + rank] = sig[c];
        if (rank >= s) continue;
        if (!(sig[c] > 0.0)) { if (lane == 0) atomicOr(flag, 4); }
        const double inv = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
        const double u0 = m0[c] * inv, u1 = m1[c] * inv;
        // largest magnitude entry, lowest row on ties
        double bv = h0 ? fabs(u0) : -1.0;
        int brw = lane;
        if (h1 && fabs(u1) > bv) { bv = fabs(u1); brw = lane + 64; }
        double sgnv = (brw == lane) ? u0 : u1;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int orw = __shfl_xor(brw, o);
            const double os = __shfl_xor(sgnv, o);
            if (ov > bv || (ov == bv && orw < brw)) { bv = ov; brw = orw; sgnv = os; }
        }
        const double fl = sgnv < 0.0 ? -1.0 : 1.0;
        if (h0) Pu[(r0 + lane) * s + rank] = fl * u0;
        if (h1) Pu[(r0 + lane + 64) * s + rank] = fl * u1;
    }
}

hipError_t launch_svd(const double* B, int r, const int32_t* fc, int64_t n_agg, int nb, int s, double* Pu,
                      double* sv, int32_t* flag, hipStream_t st) {
    if (r < 1 || r > SVD_MAXR || s < 1 || s > r) return hipErrorInvalidValue;
    if (n_agg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_svd, dim3(grid_for(n_agg, WAVES_PER_WG)), dim3(WG), 0, st, B, r, fc, n_agg, nb, s, Pu, sv,
                       flag);
    return hipGetLastError();
}

// General form (up to 64 candidates, any number of rows, one coarse size per
// aggregate): one workgroup per aggregate J, the working columns in global
// memory (work + woff[J]).  The rows of J are the real dofs of its children
// (child u owns rows u*nb + [0, sz[u])), nr of them; with nr >= r the r
// columns of B_J (length nr) are orthogonalised, with nr < r the nr columns of
// B_J^T (length r) are, and the rotations are accumulated in V (nr x nr), whose
// columns are then the left singular vectors of B_J.  Column pairs follow a
// round-robin order, a round's disjoint pairs spread over the four
// wavefronts; sweeps repeat until no pair needs a rotation (at most 60).
// sJ[J] >= 0 is the number of vectors kept (eq:sik, h-step); sJ[J] < 0 asks
// for the h*-step count, the singular values above delta times the largest,
// which is written back to sJ[J].  Output: the leading sJ[J] left singular
// vectors with canonical sign in Pu (row-major, spad columns; other entries
// untouched), the r singular values of J in sv (zeros beyond the rank bound).
constexpr int SVDG_MAXR = 64;
constexpr int SVDG_SWEEPS = 60;

__global__ __launch_bounds__(WG) void k_svd_gen(const double* __restrict__ B, int r, const int32_t* __restrict__ fc,
                                                const int32_t* __restrict__ sz, int nb, int64_t n_agg,
                                                int32_t* __restrict__ sJ, double delta, int spad,
                                                double* __restrict__ work, const int64_t* __restrict__ woff,
                                                double* __restrict__ Pu, double* __restrict__ sv,
                                                int32_t* __restrict__ flag) {
    __shared__ int32_t rowof[1024];
    __shared__ double sig[SVDG_MAXR];
    __shared__ int rank_of[SVDG_MAXR];
    __shared__ int any_rot;
    __shared__ int nr_sh;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t J = blockIdx.x;
    if (J >= n_agg) return;
    // real rows of J, in child order
    if (threadIdx.x == 0) {
        int nr = 0;
        for (int32_t u = fc[J]; u < fc[J + 1]; ++u)
            for (int i = 0; i < sz[u] && nr < 1024; ++i) rowof[nr++] = u * nb + i;
        int tot = 0;
        for (int32_t u = fc[J]; u < fc[J + 1]; ++u) tot += sz[u];
        nr_sh = tot;
    }
    __syncthreads();
    const int nr = nr_sh;
    if (nr > 1024) {
        if (threadIdx.x == 0) atomicOr(flag, 2);
        return;
    }
    const bool tall = nr >= r;
    const int ncol = tall ? r : nr;       // columns rotated
    const int len = tall ? nr : r;        // their length
    double* W = work + woff[J];           // ncol columns of length len
    double* V = W + int64_t(ncol) * len;  // nr x nr (column-major) when !tall
    for (int t = threadIdx.x; t < ncol * len; t += WG) {
        const int col = t / len, e = t - (t / len) * len;
        W[t] = tall ? B[int64_t(rowof[e]) * r + col] : B[int64_t(rowof[col]) * r + e];
    }
    if (!tall)
        for (int t = threadIdx.x; t < nr * nr; t += WG) V[t] = (t / nr == t % nr) ? 1.0 : 0.0;
    __syncthreads();
    const int np = (ncol + 1) & ~1;       // players of the round-robin (one dummy when ncol is odd)
    for (int sweep = 0; sweep < SVDG_SWEEPS; ++sweep) {
        if (threadIdx.x == 0) any_rot = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pi = wave; pi < np / 2; pi += WAVES_PER_WG) {
                auto player = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + round) % (np - 1); };
                int p = player(pi), q = player(np - 1 - pi);
                if (p > q) { const int t = p; p = q; q = t; }
                if (q >= ncol) continue;  // the dummy player
                double* wp = W + int64_t(p) * len;
                double* wq = W + int64_t(q) * len;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int e = lane; e < len; e += 64) {
                    const double x = wp[e], y = wq[e];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                if (lane == 0) any_rot = 1;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int e = lane; e < len; e += 64) {
                    const double x = wp[e], y = wq[e];
                    wp[e] = cs * x - sn * y;
                    wq[e] = sn * x + cs * y;
                }
                if (!tall) {
                    double* vp = V + int64_t(p) * nr;
                    double* vq = V + int64_t(q) * nr;
                    for (int e = lane; e < nr; e += 64) {
                        const double x = vp[e], y = vq[e];
                        vp[e] = cs * x - sn * y;
                        vq[e] = sn * x + cs * y;
                    }
                }
            }
            __syncthreads();
        }
        if (!any_rot) break;
        __syncthreads();
    }
    // singular values: column norms
    for (int c = wave; c < ncol; c += WAVES_PER_WG) {
        double a = 0.0;
        for (int e = lane; e < len; e += 64) a += W[int64_t(c) * len + e] * W[int64_t(c) * len + e];
        a = wave_sum(a);
        if (lane == 0) sig[c] = sqrt(a);
    }
    __syncthreads();
    if (threadIdx.x < ncol) {
        const int c = threadIdx.x;
        int rk = 0;
        for (int q = 0; q < ncol; ++q)
            if (sig[q] > sig[c] || (sig[q] == sig[c] && q < c)) ++rk;
        rank_of[c] = rk;
        sv[J * r + rk] = sig[c];
    }
    for (int c = ncol + int(threadIdx.x); c < r; c += WG) sv[J * r + c] = 0.0;
    __syncthreads();
    __shared__ int s_keep;
    if (threadIdx.x == 0) {
        int sk = sJ[J];
        double smax = 0.0;
        for (int c = 0; c < ncol; ++c) smax = fmax(smax, sig[c]);
        if (sk < 0) {
            sk = 0;
            for (int c = 0; c < ncol; ++c)
                if (sig[c] > delta * smax) ++sk;
            sJ[J] = sk;
        }
        if (sk > spad || sk > ncol) atomicOr(flag, 2);
        s_keep = sk;
    }
    __syncthreads();
    const int sk = s_keep;
    if (sk > spad || sk > ncol) return;
    for (int c = wave; c < ncol; c += WAVES_PER_WG) {
        const int rk = rank_of[c];
        if (rk >= sk) continue;
        if (!(sig[c] > 0.0)) {
            if (lane == 0) atomicOr(flag, 4);
            continue;
        }
        // left singular vector: W_c / sigma_c (tall) or column c of V
        const double inv = 1.0 / sig[c];
        const double* src = tall ? W + int64_t(c) * len : V + int64_t(c) * nr;
        const double scl = tall ? inv : 1.0;
        double bv = -1.0, sg = 0.0;
        int brw = 1 << 30;
        for (int e = lane; e < nr; e += 64) {
            const double u = src[e] * scl;
            if (fabs(u) > bv) { bv = fabs(u); brw = e; sg = u; }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int orw = __shfl_xor(brw, o);
            const double os = __shfl_xor(sg, o);
            if (ov > bv || (ov == bv && orw < brw)) { bv = ov; brw = orw; sg = os; }
        }
        const double fl = sg < 0.0 ? -1.0 : 1.0;
        for (int e = lane; e < nr; e += 64) Pu[int64_t(rowof[e]) * spad + rk] = fl * src[e] * scl;
    }
}

hipError_t launch_svd_gen(const double* B, int r, const int32_t* fc, const int32_t* sz, int nb, int64_t n_agg,
                          int32_t* sJ, double delta, int spad, double* work, const int64_t* woff, double* Pu,
                          double* sv, int32_t* flag, hipStream_t st) {
    if (r < 1 || r > SVDG_MAXR || spad < 1) return hipErrorInvalidValue;
    if (n_agg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_svd_gen, dim3(unsigned(n_agg)), dim3(WG), 0, st, B, r, fc, sz, nb, n_agg, sJ, delta, spad,
                       work, woff, Pu, sv, flag);
    return hipGetLastError();
}

// ============================================================ T, R, A T, Galerkin
// Small dense block products driven by host-built index lists (symbolic phase).
// One thread per (output block, output row); the s columns of the output row
// are formed in chunks of 16 accumulators.

// W_t = sum_{a in Tm(t)} A_a * P~[col(a)]   (nb x s);  T_t = [J==agg(e)] P~[e] - omega D_e^{-1} W_t
__global__ void k_T_W(const double* __restrict__ Av, const int32_t* __restrict__ A_ci, const int32_t* __restrict__ Tm_ptr,
                      const int32_t* __restrict__ Tm_a, int64_t nT, int nb, int s, const double* __restrict__ Pu,
                      double* __restrict__ W) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nT * nb) return;
    const int64_t t = tid / nb;
    const int i = int(tid - t * nb);
    for (int l0 = 0; l0 < s; l0 += MAXB) {
        double acc[MAXB];
#pragma unroll
        for (int l = 0; l < MAXB; ++l) acc[l] = 0.0;
        for (int32_t q = Tm_ptr[t]; q < Tm_ptr[t + 1]; ++q) {
            const int32_t a = Tm_a[q];
            const double* Ar = Av + int64_t(a) * nb * nb + int64_t(i) * nb;
            const double* Pc = Pu + int64_t(A_ci[a]) * nb * s + l0;
            for (int j = 0; j < nb; ++j) {
                const double av = Ar[j];
#pragma unroll
                for (int l = 0; l < MAXB; ++l)
                    if (l0 + l < s) acc[l] += av * Pc[j * s + l];
            }
        }
#pragma unroll
        for (int l = 0; l < MAXB; ++l)
            if (l0 + l < s) W[(t * nb + i) * s + l0 + l] = acc[l];
    }
}

__global__ void k_T_final(const int32_t* __restrict__ T_row, const int32_t* __restrict__ T_ci,
                          const int32_t* __restrict__ agg, int64_t nT, int nb, int s, const double* __restrict__ Pu,
                          const double* __restrict__ dinv, double omega, const double* __restrict__ W,
                          double* __restrict__ Tv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nT * nb) return;
    const int64_t t = tid / nb;
    const int i = int(tid - t * nb);
    const int64_t e = T_row[t];
    const bool own = T_ci[t] == agg[e];
    const double* Dr = dinv + e * nb * nb + int64_t(i) * nb;
    const double* Wt = W + t * nb * s;
    for (int l0 = 0; l0 < s; l0 += MAXB) {
        double acc[MAXB];
#pragma unroll
        for (int l = 0; l < MAXB; ++l) acc[l] = 0.0;
        for (int j = 0; j < nb; ++j) {
            const double d = Dr[j];
#pragma unroll
            for (int l = 0; l < MAXB; ++l)
                if (l0 + l < s) acc[l] += d * Wt[j * s + l0 + l];
        }
#pragma unroll
        for (int l = 0; l < MAXB; ++l)
            if (l0 + l < s)
                Tv[(t * nb + i) * s + l0 + l] = (own ? Pu[(e * nb + i) * s + l0 + l] : 0.0) - omega * acc[l];
    }
}

hipError_t launch_T_build(const double* Av, const int32_t* A_ci, const int32_t* T_row, const int32_t* T_ci,
                          const int32_t* Tm_ptr, const int32_t* Tm_a, const int32_t* agg, int64_t nT, int nb, int s,
                          const double* Pu, const double* dinv, double omega, double* W, double* Tv, hipStream_t st) {
    if (s < 1) return hipErrorInvalidValue;
    if (nT == 0) return hipSuccess;
    hipLaunchKernelGGL(k_T_W, dim3(grid_for(nT * nb)), dim3(WG), 0, st, Av, A_ci, Tm_ptr, Tm_a, nT, nb, s, Pu, W);
    hipLaunchKernelGGL(k_T_final, dim3(grid_for(nT * nb)), dim3(WG), 0, st, T_row, T_ci, agg, nT, nb, s, Pu, dinv,
                       omega, W, Tv);
    return hipGetLastError();
}

__global__ void k_R_from_T(const double* __restrict__ Tv, const int32_t* __restrict__ R_t, int64_t nR, int nb, int s,
                           double* __restrict__ Rv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(nb) * s;
    if (tid >= nR * per) return;
    const int64_t rb = tid / per;
    const int rem = int(tid - rb * per);
    const int l = rem / nb, j = rem - (rem / nb) * nb;  // R block is s x nb: (l, j)
    Rv[tid] = Tv[int64_t(R_t[rb]) * per + int64_t(j) * s + l];
}

hipError_t launch_R_from_T(const double* Tv, const int32_t* R_t, int64_t nR, int nb, int s, double* Rv,
                           hipStream_t st) {
    const int64_t tot = nR * nb * s;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_R_from_T, dim3(grid_for(tot)), dim3(WG), 0, st, Tv, R_t, nR, nb, s, Rv);
    return hipGetLastError();
}

// S = D^{-1} A: block (row, blk) of S is D^{-1}_row A_blk; one thread per
// entry (i, j) of one block row's blocks.
__global__ void k_row_scale(const double* __restrict__ Av, const int32_t* __restrict__ rp, int64_t n_brow, int nb,
                            const double* __restrict__ dinv, double* __restrict__ Sv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(nb) * nb;
    if (tid >= n_brow * per) return;
    const int64_t row = tid / per;
    const int rem = int(tid - row * per);
    const int i = rem / nb, j = rem - (rem / nb) * nb;
    const double* __restrict__ Dr = dinv + row * per + int64_t(i) * nb;
    for (int32_t blk = rp[row]; blk < rp[row + 1]; ++blk) {
        const double* __restrict__ Ab = Av + int64_t(blk) * per;
        double acc = 0.0;
        for (int k = 0; k < nb; ++k) acc += Dr[k] * Ab[int64_t(k) * nb + j];
        Sv[int64_t(blk) * per + int64_t(i) * nb + j] = acc;
    }
}

hipError_t launch_row_scale(const double* Av, const int32_t* rp, int64_t n_brow, int nb, const double* dinv,
                            double* Sv, hipStream_t st) {
    const int64_t tot = n_brow * nb * nb;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_scale, dim3(grid_for(tot)), dim3(WG), 0, st, Av, rp, n_brow, nb, dinv, Sv);
    return hipGetLastError();
}

__global__ void k_gather_blocks(const double* __restrict__ vals, const int32_t* __restrict__ src, int64_t n, int per,
                                double* __restrict__ out) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= n * per) return;
    const int64_t b = tid / per;
    out[tid] = vals[int64_t(src[b]) * per + (tid - b * per)];
}

hipError_t launch_gather_blocks(const double* vals, const int32_t* src, int64_t n, int per, double* out,
                                hipStream_t st) {
    if (n * per == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_blocks, dim3(grid_for(n * per)), dim3(WG), 0, st, vals, src, n, per, out);
    return hipGetLastError();
}

// RD = R D: block (J, col) of RD is R_blk (s x nb) times the diagonal block of
// A in block row col, found at A_diag[col]; one thread per entry.
__global__ void k_right_diag(const double* __restrict__ Rv, const int32_t* __restrict__ R_ci, int64_t nR, int nb,
                             int s, const double* __restrict__ Av, const int32_t* __restrict__ A_diag,
                             double* __restrict__ RDv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(s) * nb;
    if (tid >= nR * per) return;
    const int64_t rb = tid / per;
    const int rem = int(tid - rb * per);
    const int l = rem / nb, j = rem - (rem / nb) * nb;
    const double* __restrict__ Rr = Rv + rb * per + int64_t(l) * nb;
    const double* __restrict__ D = Av + int64_t(A_diag[R_ci[rb]]) * nb * nb;
    double acc = 0.0;
    for (int k = 0; k < nb; ++k) acc += Rr[k] * D[int64_t(k) * nb + j];
    RDv[tid] = acc;
}

hipError_t launch_right_diag(const double* Rv, const int32_t* R_ci, int64_t nR, int nb, int s, const double* Av,
                             const int32_t* A_diag, double* RDv, hipStream_t st) {
    const int64_t tot = nR * nb * s;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_right_diag, dim3(grid_for(tot)), dim3(WG), 0, st, Rv, R_ci, nR, nb, s, Av, A_diag, RDv);
    return hipGetLastError();
}

// AT_u = sum over pairs (a, t) of A_a (nb x nb) * T_t (nb x s)
__global__ void k_AT(const double* __restrict__ Av, const double* __restrict__ Tv, const int64_t* __restrict__ pp,
                     const int32_t* __restrict__ pa, const int32_t* __restrict__ pt, int64_t nAT, int nb, int s,
                     double* __restrict__ ATv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nAT * nb) return;
    const int64_t u = tid / nb;
    const int i = int(tid - u * nb);
    for (int l0 = 0; l0 < s; l0 += MAXB) {
        double acc[MAXB];
#pragma unroll
        for (int l = 0; l < MAXB; ++l) acc[l] = 0.0;
        for (int64_t q = pp[u]; q < pp[u + 1]; ++q) {
            const double* Ar = Av + int64_t(pa[q]) * nb * nb + int64_t(i) * nb;
            const double* Tt = Tv + int64_t(pt[q]) * nb * s + l0;
            for (int j = 0; j < nb; ++j) {
                const double av = Ar[j];
#pragma unroll
                for (int l = 0; l < MAXB; ++l)
                    if (l0 + l < s) acc[l] += av * Tt[j * s + l];
            }
        }
#pragma unroll
        for (int l = 0; l < MAXB; ++l)
            if (l0 + l < s) ATv[(u * nb + i) * s + l0 + l] = acc[l];
    }
}

hipError_t launch_AT(const double* Av, const double* Tv, const int64_t* pp, const int32_t* pa, const int32_t* pt,
                     int64_t nAT, int nb, int s, double* ATv, hipStream_t st) {
    if (s < 1) return hipErrorInvalidValue;
    if (nAT == 0) return hipSuccess;
    hipLaunchKernelGGL(k_AT, dim3(grid_for(nAT * nb)), dim3(WG), 0, st, Av, Tv, pp, pa, pt, nAT, nb, s, ATv);
    return hipGetLastError();
}

// C_v = sum over pairs (t, u) of T_t^T (s x nb) * AT_u (nb x s)
__global__ void k_galerkin(const double* __restrict__ Tv, const double* __restrict__ ATv,
                           const int64_t* __restrict__ pp, const int32_t* __restrict__ pt,
                           const int32_t* __restrict__ pu, int64_t nC, int nb, int s, double* __restrict__ Cv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nC * s) return;
    const int64_t v = tid / s;
    const int i = int(tid - v * s);
    for (int l0 = 0; l0 < s; l0 += MAXB) {
        double acc[MAXB];
#pragma unroll
        for (int l = 0; l < MAXB; ++l) acc[l] = 0.0;
        for (int64_t q = pp[v]; q < pp[v + 1]; ++q) {
            const double* Tt = Tv + int64_t(pt[q]) * nb * s;
            const double* Au = ATv + int64_t(pu[q]) * nb * s + l0;
            for (int j = 0; j < nb; ++j) {
                const double tv = Tt[j * s + i];
#pragma unroll
                for (int l = 0; l < MAXB; ++l)
                    if (l0 + l < s) acc[l] += tv * Au[j * s + l];
            }
        }
#pragma unroll
        for (int l = 0; l < MAXB; ++l)
            if (l0 + l < s) Cv[(v * s + i) * s + l0 + l] = acc[l];
    }
}

hipError_t launch_galerkin(const double* Tv, const double* ATv, const int64_t* pp, const int32_t* pt,
                           const int32_t* pu, int64_t nC, int nb, int s, double* Cv, hipStream_t st) {
    if (s < 1) return hipErrorInvalidValue;
    if (nC == 0) return hipSuccess;
    hipLaunchKernelGGL(k_galerkin, dim3(grid_for(nC * s)), dim3(WG), 0, st, Tv, ATv, pp, pt, pu, nC, nb, s, Cv);
    return hipGetLastError();
}

// M_v = sum over pairs q of w_q R_{pr[q]} (s x nb) * A_{pa[q]} (nb x nb); one
// thread per row i of an M block, nb outputs in chunks of MAXB
__global__ void k_restrict_resid(const double* __restrict__ Rv, const double* __restrict__ Av,
                                 const int32_t* __restrict__ R_ci, const int32_t* __restrict__ M_ci,
                                 const int64_t* __restrict__ pp, const int32_t* __restrict__ pr,
                                 const int32_t* __restrict__ pa, int64_t nM, int nb, int s, double omega,
                                 double* __restrict__ Mv) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nM * s) return;
    const int64_t v = tid / s;
    const int i = int(tid - v * s);
    const int32_t col = M_ci[v];
    for (int j0 = 0; j0 < nb; j0 += MAXB) {
        double acc[MAXB];
#pragma unroll
        for (int j = 0; j < MAXB; ++j) acc[j] = 0.0;
        for (int64_t q = pp[v]; q < pp[v + 1]; ++q) {
            const double w = (R_ci[pr[q]] == col) ? 1.0 - omega : -omega;
            const double* Rr = Rv + int64_t(pr[q]) * s * nb + int64_t(i) * nb;
            const double* Ab = Av + int64_t(pa[q]) * nb * nb + j0;
            for (int l = 0; l < nb; ++l) {
                const double rv = w * Rr[l];
#pragma unroll
                for (int j = 0; j < MAXB; ++j)
                    if (j0 + j < nb) acc[j] += rv * Ab[int64_t(l) * nb + j];
            }
        }
#pragma unroll
        for (int j = 0; j < MAXB; ++j)
            if (j0 + j < nb) Mv[(v * s + i) * nb + j0 + j] = acc[j];
    }
}

hipError_t launch_restrict_resid(const double* Rv, const double* Av, const int32_t* R_ci, const int32_t* M_ci,
                                 const int64_t* pp, const int32_t* pr, const int32_t* pa, int64_t nM, int nb, int s,
                                 double omega, double* Mv, hipStream_t st) {
    if (s < 1 || nb < 1) return hipErrorInvalidValue;
    if (nM == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict_resid, dim3(grid_for(nM * s)), dim3(WG), 0, st, Rv, Av, R_ci, M_ci, pp, pr, pa, nM,
                       nb, s, omega, Mv);
    return hipGetLastError();
}

// Units of a coarse level whose s_J is below the level's block size carry
// zero rows and columns in their padding; a unit diagonal there keeps the
// diagonal blocks invertible while the padding stays zero in every vector.
__global__ void k_pad_diag(double* __restrict__ Av, const int32_t* __restrict__ diag_pos, int64_t n_brow, int nb,
                           const int32_t* __restrict__ sz) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= n_brow * nb) return;
    const int64_t u = tid / nb;
    const int i = int(tid - u * nb);
    if (i >= sz[u]) Av[int64_t(diag_pos[u]) * nb * nb + int64_t(i) * nb + i] = 1.0;
}

hipError_t launch_pad_diag(double* Av, const int32_t* diag_pos, int64_t n_brow, int nb, const int32_t* sz,
                           hipStream_t st) {
    if (n_brow * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_diag, dim3(grid_for(n_brow * nb)), dim3(WG), 0, st, Av, diag_pos, n_brow, nb, sz);
    return hipGetLastError();
}

// ============================================================ block-diagonal updates
// The block-Jacobi steps of a level whose operator is applied matrix-free
// (q = A_k u formed by another chain of products): one thread per (row, column)
//   BD_SWEEP  y = x + omega (c - D^{-1} q)   (c = D^{-1} b)
//   BD_RESID  y = c - D^{-1} q               (the residual D^{-1} (b - A u))
//   BD_START  y = omega D^{-1} q, y2 = D^{-1} q   (the first sweep, q = b)
// with D^{-1} natural (n_units x nb x nb); FP32 operands accumulate in FP32.
template <typename T, int MODE>
__global__ __launch_bounds__(WG) void k_bdiag(const T* __restrict__ dinv, const T* __restrict__ q,
                                              const T* __restrict__ c, const T* __restrict__ x, T* __restrict__ y,
                                              T* __restrict__ y2, T omega, int64_t n_units, int nb, int m) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = n_units * nb;
    if (tid >= n * m) return;
    const int64_t row = tid / m;
    const int col = int(tid - row * m);
    const int64_t u = row / nb;
    const int i = int(row - u * nb);
    const T* __restrict__ Dr = dinv + (u * nb + i) * nb;
    const T* __restrict__ qu = q + u * nb * m + col;
    T acc = T(0);
    for (int j = 0; j < nb; ++j) acc += Dr[j] * qu[int64_t(j) * m];
    if (MODE == BD_SWEEP) y[tid] = x[tid] + omega * (c[tid] - acc);
    else if (MODE == BD_RESID) y[tid] = c[tid] - acc;
    else {
        y[tid] = omega * acc;
        y2[tid] = acc;
    }
}

template <typename T>
hipError_t launch_bdiag(int mode, const T* dinv, const T* q, const T* c, const T* x, T* y, T* y2, T omega,
                        int64_t n_units, int nb, int m, hipStream_t st) {
    const int64_t tot = n_units * nb * m;
    if (tot == 0) return hipSuccess;
    const dim3 g(grid_for(tot)), b(WG);
    switch (mode) {
        case BD_SWEEP: hipLaunchKernelGGL((k_bdiag<T, BD_SWEEP>), g, b, 0, st, dinv, q, c, x, y, y2, omega, n_units, nb, m); break;
        case BD_RESID: hipLaunchKernelGGL((k_bdiag<T, BD_RESID>), g, b, 0, st, dinv, q, c, x, y, y2, omega, n_units, nb, m); break;
        case BD_START: hipLaunchKernelGGL((k_bdiag<T, BD_START>), g, b, 0, st, dinv, q, c, x, y, y2, omega, n_units, nb, m); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_bdiag<double>(int, const double*, const double*, const double*, const double*, double*,
                                         double*, double, int64_t, int, int, hipStream_t);
template hipError_t launch_bdiag<float>(int, const float*, const float*, const float*, const float*, float*, float*,
                                        float, int64_t, int, int, hipStream_t);

// ============================================================ coarsest level
__global__ void k_dense_from_bsr(const double* __restrict__ vals, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, int64_t n_brow, int nb, double* __restrict__ dense) {
    const int64_t nnz = rp[n_brow];
    const int64_t per = int64_t(nb) * nb;
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= nnz * per) return;
    const int64_t blk = tid / per;
    const int rem = int(tid - blk * per);
    const int i = rem / nb, j = rem - (rem / nb) * nb;
    // block row by binary search
    int64_t lo = 0, hi = n_brow;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (rp[mid] <= blk) lo = mid; else hi = mid;
    }
    const int64_t n = n_brow * nb;
    dense[(lo * nb + i) * n + int64_t(ci[blk]) * nb + j] = vals[tid];
}

hipError_t launch_dense_from_bsr(const double* vals, const int32_t* rp, const int32_t* ci, int64_t n_brow, int nb,
                                 int64_t nnzb, double* dense, hipStream_t st) {
    const int64_t n = n_brow * nb;
    hipError_t e = hipMemsetAsync(dense, 0, sizeof(double) * n * n, st);
    if (e != hipSuccess) return e;
    const int64_t tot = nnzb * nb * nb;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_from_bsr, dim3(grid_for(tot)), dim3(WG), 0, st, vals, rp, ci, n_brow, nb, dense);
    return hipGetLastError();
}

__global__ void k_absmax_part(const double* __restrict__ a, int64_t n, double* __restrict__ out) {
    __shared__ double sh[WG];
    double m = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG) m = fmax(m, fabs(a[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ void k_absmax_final(const double* __restrict__ part, int np, double* __restrict__ out) {
    __shared__ double sh[WG];
    double m = 0.0;
    for (int i = threadIdx.x; i < np; i += WG) m = fmax(m, part[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

hipError_t launch_absmax(const double* a, int64_t n, double* out, hipStream_t st) {
    // out must hold 1 + DOT_PARTS doubles: out[0] result, out[1..] partials
    const int np = int(std::min<int64_t>(DOT_PARTS, std::max<int64_t>(1, (n + WG - 1) / WG)));
    hipLaunchKernelGGL(k_absmax_part, dim3(np), dim3(WG), 0, st, a, n, out + 1);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(WG), 0, st, out + 1, np, out);
    return hipGetLastError();
}

// In-place Gauss-Jordan inversion with row pivoting, one elimination step per
// call: (1) one workgroup picks the pivot row (largest |a[i][c]|, i >= c, lowest
// row on ties), swaps it into row c and saves row c and column c; (2) the rank-1
// update of every entry.  After all steps the row interchanges are undone as
// column interchanges in reverse order.
__global__ void k_gj_pivot(double* __restrict__ a, int64_t n, int64_t c, int32_t* __restrict__ piv,
                           int32_t* __restrict__ flag, const double* __restrict__ amax, double tol_scale,
                           double* __restrict__ rowc, double* __restrict__ colc) {
    __shared__ double bv[1024];
    __shared__ int64_t bi[1024];
    const int t = threadIdx.x;
    double best = -1.0;
    int64_t bidx = c;
    for (int64_t i = c + t; i < n; i += blockDim.x) {
        const double v = fabs(a[i * n + c]);
        if (v > best) { best = v; bidx = i; }
    }
    bv[t] = best;
    bi[t] = bidx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) {
            if (bv[t + o] > bv[t] || (bv[t + o] == bv[t] && bi[t + o] < bi[t])) { bv[t] = bv[t + o]; bi[t] = bi[t + o]; }
        }
        __syncthreads();
    }
    const int64_t p = bi[0];
    if (t == 0) {
        piv[c] = int32_t(p);
        if (!(bv[0] > tol_scale * amax[0])) atomicOr(flag, 1);
    }
    if (p != c)
        for (int64_t j = t; j < n; j += blockDim.x) {
            const double tmp = a[c * n + j];
            a[c * n + j] = a[p * n + j];
            a[p * n + j] = tmp;
        }
    __syncthreads();
    for (int64_t j = t; j < n; j += blockDim.x) {
        rowc[j] = a[c * n + j];
        colc[j] = a[j * n + c];
    }
}

__global__ void k_gj_update(double* __restrict__ a, int64_t n, int64_t c, const double* __restrict__ rowc,
                            const double* __restrict__ colc) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= n * n) return;
    const int64_t i = tid / n, j = tid - (tid / n) * n;
    const double pv = rowc[c];
    double v;
    if (i != c && j != c) v = a[tid] - colc[i] * rowc[j] / pv;
    else if (i == c && j != c) v = rowc[j] / pv;
    else if (i != c) v = -colc[i] / pv;
    else v = 1.0 / pv;
    a[tid] = v;
}

__global__ void k_gj_unpermute(double* __restrict__ a, int64_t n, const int32_t* __restrict__ piv) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* row = a + i * n;
    for (int64_t c = n - 1; c >= 0; --c) {
        const int64_t p = piv[c];
        if (p != c) {
            const double tmp = row[c];
            row[c] = row[p];
            row[p] = tmp;
        }
    }
}

hipError_t launch_gj_invert(double* a, int64_t n, int32_t* piv, int32_t* flag, const double* amax, double tol_scale,
                            double* rowc, double* colc, hipStream_t st) {
    for (int64_t c = 0; c < n; ++c) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, a, n, c, piv, flag, amax, tol_scale, rowc, colc);
        hipLaunchKernelGGL(k_gj_update, dim3(grid_for(n * n)), dim3(WG), 0, st, a, n, c, rowc, colc);
    }
    hipLaunchKernelGGL(k_gj_unpermute, dim3(grid_for(n)), dim3(WG), 0, st, a, n, piv);
    return hipGetLastError();
}

// ============================================================ random streams
// SplitMix64 (Steele, Lea & Flood 2014): output i of the stream seeded with s is
// mix(s + (i+1) * 0x9E3779B97F4A7C15); uniform double = (z >> 11) * 2^-53.
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t z) { return double(z >> 11) * 0x1.0p-53; }

// x[u*nb + i] = 2 U(seed, (perm ? perm[u] : u) * nb + i) - 1
__global__ void k_uniform(uint64_t seed, const int64_t* __restrict__ perm, int64_t n_units, int nb, double* __restrict__ x) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_units * nb) return;
    const int64_t u = t / nb;
    const int i = int(t - u * nb);
    const int64_t e = perm ? perm[u] : u;
    x[t] = 2.0 * u01(splitmix(seed, uint64_t(e * nb + i))) - 1.0;
}

hipError_t launch_uniform(uint64_t seed, const int64_t* perm, int64_t n_units, int nb, double* x, hipStream_t st) {
    if (n_units * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform, dim3(grid_for(n_units * nb)), dim3(WG), 0, st, seed, perm, n_units, nb, x);
    return hipGetLastError();
}

// padded level: x[u*nb + i] = 2 U(seed, roff[u] + i) - 1 for i < sz[u], 0 in the padding
__global__ void k_uniform_padded(uint64_t seed, const int64_t* __restrict__ roff, const int32_t* __restrict__ sz,
                                 int64_t n_units, int nb, double* __restrict__ x) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_units * nb) return;
    const int64_t u = t / nb;
    const int i = int(t - u * nb);
    x[t] = i < sz[u] ? 2.0 * u01(splitmix(seed, uint64_t(roff[u] + i))) - 1.0 : 0.0;
}

hipError_t launch_uniform_padded(uint64_t seed, const int64_t* roff, const int32_t* sz, int64_t n_units, int nb,
                                 double* x, hipStream_t st) {
    if (n_units * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform_padded, dim3(grid_for(n_units * nb)), dim3(WG), 0, st, seed, roff, sz, n_units, nb,
                       x);
    return hipGetLastError();
}

// Box-Muller normals: stream index k = (caller dof) * r + c; pair k/2 uses
// u1 = 1 - U(2*(k/2)), u2 = U(2*(k/2)+1); even k -> R cos(2 pi u2), odd -> R sin.
__global__ void k_normal(uint64_t seed, const int64_t* __restrict__ perm, int64_t n_units, int nb, int r,
                         double* __restrict__ x) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_units * nb * r) return;
    const int64_t row = t / r;
    const int c = int(t - row * r);
    const int64_t u = row / nb;
    const int i = int(row - u * nb);
    const int64_t e = perm ? perm[u] : u;
    const uint64_t k = uint64_t((e * nb + i) * r + c);
    const uint64_t pr = k >> 1;
    const double u1 = 1.0 - u01(splitmix(seed, 2 * pr));
    const double u2 = u01(splitmix(seed, 2 * pr + 1));
    const double R = sqrt(-2.0 * log(u1));
    x[t] = (k & 1) ? R * sin(2.0 * M_PI * u2) : R * cos(2.0 * M_PI * u2);
}

hipError_t launch_normal(uint64_t seed, const int64_t* perm, int64_t n_units, int nb, int r, double* x, hipStream_t st) {
    const int64_t tot = n_units * nb * r;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_normal, dim3(grid_for(tot)), dim3(WG), 0, st, seed, perm, n_units, nb, r, x);
    return hipGetLastError();
}

// ============================================================ reductions
// Deterministic two-pass dot products: a fixed grid of partial sums (grid-stride
// loop, LDS tree), then one workgroup sums the partials in a fixed order.
template <typename T, int M>
__global__ __launch_bounds__(WG) void k_dot_part(const T* __restrict__ a, const T* __restrict__ b, int64_t n, int ld,
                                                 double* __restrict__ part) {
    __shared__ double sh[WG];
    double s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG) {
#pragma unroll
        for (int c = 0; c < M; ++c) s[c] += double(a[i * ld + c]) * double(b[i * ld + c]);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        sh[threadIdx.x] = s[c];
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[int64_t(c) * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(WG) void k_sum_parts(const double* __restrict__ part, int np, int m, double* __restrict__ out) {
    __shared__ double sh[WG];
    for (int c = 0; c < m; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < np; i += WG) s += part[int64_t(c) * np + i];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = sh[0];
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n, int m, double* part, double* out, hipStream_t st) {
    // part must hold DOT_PARTS * m doubles
    const int np = int(std::min<int64_t>(DOT_PARTS, std::max<int64_t>(1, (n + WG - 1) / WG)));
    int c0 = 0;
    while (c0 < m) {
        const int rem = m - c0;
        const int w = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem;
        double* pc = part + int64_t(c0) * np;
        switch (w) {
            case 16: hipLaunchKernelGGL((k_dot_part<T, 16>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
            case 8: hipLaunchKernelGGL((k_dot_part<T, 8>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
            case 4: hipLaunchKernelGGL((k_dot_part<T, 4>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
            case 3: hipLaunchKernelGGL((k_dot_part<T, 3>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
            case 2: hipLaunchKernelGGL((k_dot_part<T, 2>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
            default: hipLaunchKernelGGL((k_dot_part<T, 1>), dim3(np), dim3(WG), 0, st, a + c0, b + c0, n, m, pc); break;
        }
        c0 += w;
    }
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(WG), 0, st, part, np, m, out);
    return hipGetLastError();
}
template hipError_t launch_dot<double>(const double*, const double*, int64_t, int, double*, double*, hipStream_t);
template hipError_t launch_dot<float>(const float*, const float*, int64_t, int, double*, double*, hipStream_t);

// ============================================================ Krylov vector ops
__global__ void k_axpby_dev(const double* __restrict__ x, double* __restrict__ y, int64_t n, int m,
                            const double* __restrict__ alpha, double sa, double by) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * m) return;
    const int c = int(t % m);
    const double a = (alpha ? alpha[c] : 1.0) * sa;
    y[t] = a * x[t] + by * y[t];
}

hipError_t launch_axpby_dev(const double* x, double* y, int64_t n, int m, const double* alpha, double sa, double by,
                            hipStream_t st) {
    if (n * m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby_dev, dim3(grid_for(n * m)), dim3(WG), 0, st, x, y, n, m, alpha, sa, by);
    return hipGetLastError();
}

// ------------------------------------------------------------ fused Krylov steps

// Each workgroup writes its partial sums s[c] to part[c * gridDim.x + block];
// k_finalize sums them in a fixed order (the kernel boundary orders the two, so
// no device-scope fence is needed inside the streaming kernels).
template <int M>
__device__ __forceinline__ void block_partials(double (&s)[M], double* __restrict__ part) {
    __shared__ double sh[WG];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        sh[threadIdx.x] = s[c];
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[int64_t(c) * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

// out1[c] = sum_i part[c*np + i] for c < split, out2[c - split] for c >= split;
// flag[c] |= 2 if sum c is not finite (flag may be NULL).
__global__ __launch_bounds__(WG) void k_finalize(const double* __restrict__ part, int np, int mt,
                                                 double* __restrict__ out1, int split, double* __restrict__ out2,
                                                 int32_t* __restrict__ flag, const uint32_t* __restrict__ msrc = nullptr,
                                                 uint32_t* __restrict__ mdst = nullptr, int mwords = 0) {
    __shared__ double sh[WG];
    for (int c = 0; c < mt; ++c) {
        // thread t adds the partials t + WG k in four interleaved sums (k mod 4),
        // so four loads are in flight; the order is fixed by np alone
        const double* __restrict__ pc = part + int64_t(c) * np;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = threadIdx.x;
        for (; i + 3 * WG < np; i += 4 * WG) {
            a0 += pc[i];
            a1 += pc[i + WG];
            a2 += pc[i + 2 * WG];
            a3 += pc[i + 3 * WG];
        }
        if (i < np) a0 += pc[i];
        if (i + WG < np) a1 += pc[i + WG];
        if (i + 2 * WG < np) a2 += pc[i + 2 * WG];
        const double v = (a0 + a1) + (a2 + a3);
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (c < split) out1[c] = sh[0];
            else out2[c - split] = sh[0];
            if (flag && !isfinite(sh[0])) atomicOr(flag + c, 2);
        }
        __syncthreads();
    }
    // optional mirror of a status record into pinned host memory: agent-scope
    // loads see this kernel's sums, system-scope stores write through to the host
    if (mdst) {
        __syncthreads();
        for (int w = threadIdx.x; w < mwords; w += WG)
            __hip_atomic_store(mdst + w, __hip_atomic_load(msrc + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// part2[c * G2 + k] = sum over j of part[c * np + k + G2 j] (thread t takes j = t,
// t + WG, ..., then a tree over the workgroup): the order is fixed by np and G2
__global__ __launch_bounds__(WG) void k_part_stride(const double* __restrict__ part, int np, int ncol,
                                                     double* __restrict__ part2) {
    __shared__ double sh[WG];
    const int G2 = gridDim.x;
    for (int c = 0; c < ncol; ++c) {
        double s = 0.0;
        for (int64_t j = threadIdx.x; blockIdx.x + G2 * j < np; j += WG) s += part[int64_t(c) * np + blockIdx.x + G2 * j];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part2[int64_t(c) * G2 + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

int64_t mfma_dot_parts(int64_t n_brow) { return int64_t(grid_for(n_brow, WAVES_PER_WG)) * MFMA_COLS; }

hipError_t launch_mfma_dot(const Nbsr<double>& A, const double* x, double* y, int m, double* part, double* part2,
                           double* xy, hipStream_t st, int u) {
    if (m % MFMA_COLS != 0 || A.br > NBSR_MAXB || A.bc > NBSR_MAXB) return hipErrorInvalidValue;
    if (A.n_brow == 0) return hipSuccess;
    const unsigned nwg = grid_for(A.n_brow, WAVES_PER_WG);
    const unsigned g2 = unsigned(std::min<int64_t>(KRY_BLOCKS, nwg));
    for (int c0 = 0; c0 < m; c0 += MFMA_COLS) {
        const dim3 grid{nwg, 1u, 1u}, block{unsigned(WG), 1u, 1u};
        switch (u) {
            case 1:
                hipLaunchKernelGGL((k_mfma<double, MF_AXDOT, 1>), grid, block, 0, st, A, nullptr, x + c0, nullptr, y + c0,
                                   0.0, m, part);
                break;
            case 2:
                hipLaunchKernelGGL((k_mfma<double, MF_AXDOT, 2>), grid, block, 0, st, A, nullptr, x + c0, nullptr, y + c0,
                                   0.0, m, part);
                break;
            default:
                hipLaunchKernelGGL((k_mfma<double, MF_AXDOT, 4>), grid, block, 0, st, A, nullptr, x + c0, nullptr, y + c0,
                                   0.0, m, part);
                break;
        }
        hipLaunchKernelGGL(k_part_stride, dim3(g2), dim3(WG), 0, st, part, int(nwg), MFMA_COLS, part2);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, part2, int(g2), MFMA_COLS, xy + c0, MFMA_COLS,
                           static_cast<double*>(nullptr), static_cast<int32_t*>(nullptr));
    }
    return hipGetLastError();
}

static inline unsigned kry_grid(int64_t n) {
    return unsigned(std::min<int64_t>(KRY_BLOCKS, std::max<int64_t>(1, (n + WG - 1) / WG)));
}

template <int M>
__global__ __launch_bounds__(WG) void k_dot_part2(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                                  int ld, double* part) {
    double s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c] = 0.0;
#pragma unroll 2
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG)
#pragma unroll
        for (int c = 0; c < M; ++c) s[c] += a[i * ld + c] * b[i * ld + c];
    block_partials<M>(s, part);
}

// The CG update of one grid-stride pass.  In place (INPLACE: the residual r_out
// is read and written through one pointer, r_in unused) or out of place; every
// pointer that is accessed is restrict, so the loads of a row's M columns are
// not held behind the previous column's stores.
template <int M, bool INPLACE>
__device__ __forceinline__ void cg_update_body(double* __restrict__ x, const double* __restrict__ r_in,
                                               double* __restrict__ r_out, const double* __restrict__ p,
                                               const double* __restrict__ q, float* __restrict__ r32, int64_t n,
                                               int ld, const double* __restrict__ rz, const double* __restrict__ pq,
                                               const int32_t* __restrict__ active, double* __restrict__ part,
                                               int32_t* __restrict__ flag) {
    double al[M], s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        s[c] = 0.0;
        al[c] = 0.0;
        if (active[c]) {
            const double d = pq[c];
            al[c] = rz[c] / d;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                if (!(d > 0.0)) atomicOr(flag + c, 1);
                if (!isfinite(al[c])) atomicOr(flag + c, 2);
            }
            if (!isfinite(al[c])) al[c] = 0.0;
        }
    }
#pragma unroll 2
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG) {
        const int64_t e0 = i * ld;
        double xv[M], pv[M], rv[M], qv[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            xv[c] = x[e0 + c];
            pv[c] = p[e0 + c];
            rv[c] = INPLACE ? r_out[e0 + c] : r_in[e0 + c];
            qv[c] = q[e0 + c];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            x[e0 + c] = xv[c] + al[c] * pv[c];
            const double v = rv[c] - al[c] * qv[c];
            r_out[e0 + c] = v;
            if (r32) r32[e0 + c] = float(v);
            s[c] += v * v;
        }
    }
    block_partials<M>(s, part);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_update_ip(double* x, double* r, const double* p, const double* q,
                                                     float* r32, int64_t n, int ld, const double* rz,
                                                     const double* pq, const int32_t* active, double* part,
                                                     int32_t* flag) {
    cg_update_body<M, true>(x, nullptr, r, p, q, r32, n, ld, rz, pq, active, part, flag);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_update_oop(double* x, const double* r_in, double* r_out, const double* p,
                                                      const double* q, float* r32, int64_t n, int ld,
                                                      const double* rz, const double* pq, const int32_t* active,
                                                      double* part, int32_t* flag) {
    cg_update_body<M, false>(x, r_in, r_out, p, q, r32, n, ld, rz, pq, active, part, flag);
}

template <int M>
__global__ __launch_bounds__(WG) void k_zdots(const float* __restrict__ z32, double* __restrict__ z,
                                              const double* __restrict__ r, const double* __restrict__ r_old,
                                              int64_t n, int ld, double* __restrict__ part) {
    constexpr int M2 = 2 * M;
    double s[M2];
#pragma unroll
    for (int c = 0; c < M2; ++c) s[c] = 0.0;
#pragma unroll 2
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG) {
        const int64_t e0 = i * ld;
        double zv[M], rv[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            zv[c] = z32 ? double(z32[e0 + c]) : z[e0 + c];
            rv[c] = r[e0 + c];
        }
        if (z32 && z) {
#pragma unroll
            for (int c = 0; c < M; ++c) z[e0 + c] = zv[c];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) s[c] += rv[c] * zv[c];
        if (r_old) {
#pragma unroll
            for (int c = 0; c < M; ++c) s[M + c] += zv[c] * r_old[e0 + c];
        }
    }
    block_partials<M2>(s, part);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_dir(double* __restrict__ p, const double* __restrict__ z, int64_t n, int ld,
                                               const double* __restrict__ rzn, const double* __restrict__ zro,
                                               const double* __restrict__ rzo, const int32_t* __restrict__ active,
                                               const float* __restrict__ z32) {
    double be[M];
#pragma unroll
    for (int c = 0; c < M; ++c) be[c] = active[c] ? (rzn[c] - (zro ? zro[c] : 0.0)) / rzo[c] : 0.0;
#pragma unroll 2
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int64_t e = i * ld + c;
            p[e] = (z32 ? double(z32[e]) : z[e]) + be[c] * p[e];
        }
}

// ---- coalesced forms (ld == M, M divides 64) ----
// A wavefront handles the 64 consecutive rows that its threads own in the
// per-row kernels (thread t: rows t + k * stride), in two sub-chunks of 32
// rows.  Lane l updates the values j * 64 + l of the sub-chunk's 32 * M
// contiguous values, all in column l % M, with coalesced accesses; the
// operands of the sums go through LDS to the owner lane of each row, which adds
// them in column order with the same multiply-adds as the per-row kernels.
// Every partial sum, and so every result, is bit-identical to theirs.
constexpr int CO_ROWS = 32;

template <int M, bool INPLACE>
__device__ __forceinline__ void cg_update_co_body(double* __restrict__ x, const double* __restrict__ r_in,
                                                     double* __restrict__ r_out, const double* __restrict__ p,
                                                     const double* __restrict__ q, float* __restrict__ r32,
                                                     int64_t n, const double* __restrict__ rz,
                                                     const double* __restrict__ pq,
                                                     const int32_t* __restrict__ active, double* __restrict__ part,
                                                     int32_t* __restrict__ flag) {
    __shared__ double buf[WAVES_PER_WG][CO_ROWS][M + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cl = lane % M;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < M; ++c)
            if (active[c]) {
                const double d = pq[c];
                if (!(d > 0.0)) atomicOr(flag + c, 1);
                if (!isfinite(rz[c] / d)) atomicOr(flag + c, 2);
            }
    }
    double alc = 0.0;
    if (active[cl]) {
        alc = rz[cl] / pq[cl];
        if (!isfinite(alc)) alc = 0.0;
    }
    double s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c] = 0.0;
    constexpr int PER = (CO_ROWS * M + 63) / 64;
    const int64_t stride = int64_t(gridDim.x) * WG;
    for (int64_t row0 = int64_t(blockIdx.x) * WG + wv * 64; row0 < n; row0 += stride) {
        for (int h = 0; h < 64 / CO_ROWS; ++h) {
            const int64_t rb = row0 + CO_ROWS * h;
            if (rb >= n) break;
            const int64_t lim = min(n - rb, int64_t(CO_ROWS)) * M;
            const int64_t base = rb * M;
            // all loads first (index clamped into the sub-chunk), then the stores
            double xv[PER], pv[PER], qv[PER], rv[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int el = j * 64 + lane;
                const int64_t e = base + (el < lim ? el : 0);
                xv[j] = x[e];
                pv[j] = p[e];
                qv[j] = q[e];
                rv[j] = INPLACE ? r_out[e] : r_in[e];
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int el = j * 64 + lane;
                if (el < lim) {
                    const int64_t e = base + el;
                    x[e] = xv[j] + alc * pv[j];
                    const double v = rv[j] - alc * qv[j];
                    r_out[e] = v;
                    if (r32) r32[e] = float(v);
                    buf[wv][el / M][el % M] = v;
                }
            }
            wave_lds_sync();
            const int ro = lane - CO_ROWS * h;
            if (ro >= 0 && ro < CO_ROWS && rb + ro < n) {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    const double v = buf[wv][ro][c];
                    s[c] += v * v;
                }
            }
            wave_lds_sync();
        }
    }
    block_partials<M>(s, part);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_update_co_ip(double* x, double* r, const double* p, const double* q,
                                                        float* r32, int64_t n, const double* rz, const double* pq,
                                                        const int32_t* active, double* part, int32_t* flag) {
    cg_update_co_body<M, true>(x, nullptr, r, p, q, r32, n, rz, pq, active, part, flag);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_update_co_oop(double* x, const double* r_in, double* r_out,
                                                         const double* p, const double* q, float* r32, int64_t n,
                                                         const double* rz, const double* pq, const int32_t* active,
                                                         double* part, int32_t* flag) {
    cg_update_co_body<M, false>(x, r_in, r_out, p, q, r32, n, rz, pq, active, part, flag);
}

// 16-row sub-chunks keep the LDS of the three-operand and two-operand sums small
// enough for several workgroups per CU
constexpr int ZR = 16;

template <int M, bool Z32, bool ROLD>
__device__ __forceinline__ void zdots_co_body(const float* __restrict__ z32, double* __restrict__ z,
                                              const double* __restrict__ r, const double* __restrict__ r_old,
                                              int64_t n, double* __restrict__ part) {
    constexpr int M2 = 2 * M;
    __shared__ double buf[WAVES_PER_WG][3][ZR][M + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double s[M2];
#pragma unroll
    for (int c = 0; c < M2; ++c) s[c] = 0.0;
    constexpr int PER = (ZR * M + 63) / 64;
    const int64_t stride = int64_t(gridDim.x) * WG;
    for (int64_t row0 = int64_t(blockIdx.x) * WG + wv * 64; row0 < n; row0 += stride) {
        for (int h = 0; h < 64 / ZR; ++h) {
            const int64_t rb = row0 + ZR * h;
            if (rb >= n) break;
            const int64_t lim = min(n - rb, int64_t(ZR)) * M;
            const int64_t base = rb * M;
            double zv[PER], rv[PER], ov[PER];
            float fz[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int el = j * 64 + lane;
                const int64_t e = base + (el < lim ? el : 0);
                if (Z32) fz[j] = z32[e];
                else zv[j] = z[e];
                rv[j] = r[e];
                ov[j] = ROLD ? r_old[e] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if (Z32) zv[j] = double(fz[j]);
                const int el = j * 64 + lane;
                if (el < lim) {
                    if (Z32 && z) z[base + el] = zv[j];
                    buf[wv][0][el / M][el % M] = zv[j];
                    buf[wv][1][el / M][el % M] = rv[j];
                    buf[wv][2][el / M][el % M] = ov[j];
                }
            }
            wave_lds_sync();
            const int ro = lane - ZR * h;
            if (ro >= 0 && ro < ZR && rb + ro < n) {
#pragma unroll
                for (int c = 0; c < M; ++c) s[c] += buf[wv][1][ro][c] * buf[wv][0][ro][c];
                if (ROLD) {
#pragma unroll
                    for (int c = 0; c < M; ++c) s[M + c] += buf[wv][0][ro][c] * buf[wv][2][ro][c];
                }
            }
            wave_lds_sync();
        }
    }
    block_partials<M2>(s, part);
}

#define ZDOTS_CO_KERNEL(NAME, Z, R)                                                                    \
    template <int M>                                                                                 \
    __global__ __launch_bounds__(WG) void NAME(const float* z32, double* z, const double* r,          \
                                               const double* r_old, int64_t n, double* part) {        \
        zdots_co_body<M, Z, R>(z32, z, r, r_old, n, part);                                           \
    }
ZDOTS_CO_KERNEL(k_zdots_co_ff, false, false)
ZDOTS_CO_KERNEL(k_zdots_co_ft, false, true)
ZDOTS_CO_KERNEL(k_zdots_co_tf, true, false)
ZDOTS_CO_KERNEL(k_zdots_co_tt, true, true)
#undef ZDOTS_CO_KERNEL

template <int M>
__global__ __launch_bounds__(WG) void k_dot_co(const double* __restrict__ a, const double* __restrict__ b,
                                               int64_t n, double* __restrict__ part) {
    __shared__ double buf[WAVES_PER_WG][2][ZR][M + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c] = 0.0;
    constexpr int PER = (ZR * M + 63) / 64;
    const int64_t stride = int64_t(gridDim.x) * WG;
    for (int64_t row0 = int64_t(blockIdx.x) * WG + wv * 64; row0 < n; row0 += stride) {
        for (int h = 0; h < 64 / ZR; ++h) {
            const int64_t rb = row0 + ZR * h;
            if (rb >= n) break;
            const int64_t lim = min(n - rb, int64_t(ZR)) * M;
            const int64_t base = rb * M;
            double av[PER], bv[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int el = j * 64 + lane;
                const int64_t e = base + (el < lim ? el : 0);
                av[j] = a[e];
                bv[j] = b[e];
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int el = j * 64 + lane;
                if (el < lim) {
                    buf[wv][0][el / M][el % M] = av[j];
                    buf[wv][1][el / M][el % M] = bv[j];
                }
            }
            wave_lds_sync();
            const int ro = lane - ZR * h;
            if (ro >= 0 && ro < ZR && rb + ro < n) {
#pragma unroll
                for (int c = 0; c < M; ++c) s[c] += buf[wv][0][ro][c] * buf[wv][1][ro][c];
            }
            wave_lds_sync();
        }
    }
    block_partials<M>(s, part);
}

template <int M>
__global__ __launch_bounds__(WG) void k_cg_dir_co(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                                                  const double* __restrict__ rzn, const double* __restrict__ zro,
                                                  const double* __restrict__ rzo,
                                                  const int32_t* __restrict__ active,
                                                  const float* __restrict__ z32) {
    const int cl = (threadIdx.x & 63) % M;
    const double be = active[cl] ? (rzn[cl] - (zro ? zro[cl] : 0.0)) / rzo[cl] : 0.0;
    const int64_t tot = n * M;
    for (int64_t e = int64_t(blockIdx.x) * WG + threadIdx.x; e < tot; e += int64_t(gridDim.x) * WG)
        p[e] = (z32 ? double(z32[e]) : z[e]) + be * p[e];
}

#define CO_DISPATCH(w, KERNEL, ...)                                                                    \
    switch (w) {                                                                                     \
        case 16: hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__); break;                                \
        case 8: hipLaunchKernelGGL((KERNEL<8>), __VA_ARGS__); break;                                  \
        case 4: hipLaunchKernelGGL((KERNEL<4>), __VA_ARGS__); break;                                  \
        case 2: hipLaunchKernelGGL((KERNEL<2>), __VA_ARGS__); break;                                  \
        default: hipLaunchKernelGGL((KERNEL<1>), __VA_ARGS__); break;                                 \
    }

// the coalesced forms apply when one chunk covers all m > 1 columns and m divides 64
// (at one column the per-row forms are coalesced already)
static inline bool co_ok(int m, int w) { return w == m && m > 1 && 64 % m == 0; }

template <typename F>
static hipError_t for_chunks(int m, F&& f) {
    int c0 = 0;
    while (c0 < m) {
        const int rem = m - c0;
        const int w = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem;
        hipError_t e = f(c0, w);
        if (e != hipSuccess) return e;
        c0 += w;
    }
    return hipSuccess;
}

#define KRY_DISPATCH(w, KERNEL, ...)                                                                   \
    switch (w) {                                                                                     \
        case 16: hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__); break;                                \
        case 8: hipLaunchKernelGGL((KERNEL<8>), __VA_ARGS__); break;                                  \
        case 4: hipLaunchKernelGGL((KERNEL<4>), __VA_ARGS__); break;                                  \
        case 3: hipLaunchKernelGGL((KERNEL<3>), __VA_ARGS__); break;                                  \
        case 2: hipLaunchKernelGGL((KERNEL<2>), __VA_ARGS__); break;                                  \
        default: hipLaunchKernelGGL((KERNEL<1>), __VA_ARGS__); break;                                 \
    }

hipError_t launch_dot_tail(const double* a, const double* b, int64_t n, int m, double* part, double* out,
                           hipStream_t st) {
    const unsigned g = kry_grid(n);
    return for_chunks(m, [&](int c0, int w) {
        if (co_ok(m, w)) {
            CO_DISPATCH(w, k_dot_co, dim3(g), dim3(WG), 0, st, a, b, n, part)
        } else {
            KRY_DISPATCH(w, k_dot_part2, dim3(g), dim3(WG), 0, st, a + c0, b + c0, n, m, part)
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, part, int(g), w, out + c0, w,
                           static_cast<double*>(nullptr), static_cast<int32_t*>(nullptr));
        return hipGetLastError();
    });
}

hipError_t launch_spmv_dot(const Sell<double>& A, const double* x, double* y, int m, double* part, double* xy,
                           hipStream_t st, int cap) {
    int c0 = 0;
    while (c0 < m) {
        const int w = sell_chunk<double>(m - c0, A, false, cap);
        if (size_t(WAVES_PER_WG) * A.G * A.tpad * w * sizeof(double) > lds_limit())
            return hipErrorInvalidConfiguration;
        hipError_t e;
        switch (w) {
            case 8: e = spmv_m<double, 8>(AX_DOT, A, x + c0, nullptr, y + c0, m, m, st, 0.0, part); break;
            case 4: e = spmv_m<double, 4>(AX_DOT, A, x + c0, nullptr, y + c0, m, m, st, 0.0, part); break;
            case 3: e = spmv_m<double, 3>(AX_DOT, A, x + c0, nullptr, y + c0, m, m, st, 0.0, part); break;
            case 2: e = spmv_m<double, 2>(AX_DOT, A, x + c0, nullptr, y + c0, m, m, st, 0.0, part); break;
            default: e = spmv_m<double, 1>(AX_DOT, A, x + c0, nullptr, y + c0, m, m, st, 0.0, part); break;
        }
        if (e != hipSuccess) return e;
        if (A.n_slices > 0)
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, part, int(grid_for(A.n_slices, WAVES_PER_WG)), w,
                               xy + c0, w, static_cast<double*>(nullptr), static_cast<int32_t*>(nullptr));
        c0 += w;
    }
    return hipGetLastError();
}

hipError_t launch_cg_update(double* x, const double* r_in, double* r_out, const double* p, const double* q,
                            float* r32, int64_t n, int m, const double* rz, const double* pq,
                            const int32_t* active, double* part, double* rr, int32_t* flag, hipStream_t st,
                            const double* stat, double* stat_host, int stat_len) {
    const unsigned g = kry_grid(n);
    return for_chunks(m, [&](int c0, int w) {
        const bool last = c0 + w == m && stat_host;
        if (co_ok(m, w) && r_in == r_out) {
            CO_DISPATCH(w, k_cg_update_co_ip, dim3(g), dim3(WG), 0, st, x, r_out, p, q, r32, n, rz, pq, active, part,
                        flag)
        } else if (co_ok(m, w)) {
            CO_DISPATCH(w, k_cg_update_co_oop, dim3(g), dim3(WG), 0, st, x, r_in, r_out, p, q, r32, n, rz, pq, active,
                        part, flag)
        } else if (r_in == r_out) {
            KRY_DISPATCH(w, k_cg_update_ip, dim3(g), dim3(WG), 0, st, x + c0, r_out + c0, p + c0, q + c0,
                         r32 ? r32 + c0 : nullptr, n, m, rz + c0, pq + c0, active + c0, part, flag + c0)
        } else {
            KRY_DISPATCH(w, k_cg_update_oop, dim3(g), dim3(WG), 0, st, x + c0, r_in + c0, r_out + c0, p + c0, q + c0,
                         r32 ? r32 + c0 : nullptr, n, m, rz + c0, pq + c0, active + c0, part, flag + c0)
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, part, int(g), w, rr + c0, w,
                           static_cast<double*>(nullptr), flag + c0,
                           last ? reinterpret_cast<const uint32_t*>(stat) : nullptr,
                           last ? reinterpret_cast<uint32_t*>(stat_host) : nullptr, last ? 2 * stat_len : 0);
        return hipGetLastError();
    });
}

hipError_t launch_zdots(const float* z32, double* z, const double* r, const double* r_old, int64_t n, int m,
                        double* part, double* rz, double* zro, hipStream_t st) {
    const unsigned g = kry_grid(n);
    return for_chunks(m, [&](int c0, int w) {
        if (co_ok(m, w)) {
            if (z32 && r_old) CO_DISPATCH(w, k_zdots_co_tt, dim3(g), dim3(WG), 0, st, z32, z, r, r_old, n, part)
            else if (z32) CO_DISPATCH(w, k_zdots_co_tf, dim3(g), dim3(WG), 0, st, z32, z, r, r_old, n, part)
            else if (r_old) CO_DISPATCH(w, k_zdots_co_ft, dim3(g), dim3(WG), 0, st, z32, z, r, r_old, n, part)
            else CO_DISPATCH(w, k_zdots_co_ff, dim3(g), dim3(WG), 0, st, z32, z, r, r_old, n, part)
        } else {
            KRY_DISPATCH(w, k_zdots, dim3(g), dim3(WG), 0, st, z32 ? z32 + c0 : nullptr, z ? z + c0 : nullptr, r + c0,
                         r_old ? r_old + c0 : nullptr, n, m, part)
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, part, int(g), r_old ? 2 * w : w, rz + c0, w,
                           zro ? zro + c0 : static_cast<double*>(nullptr), static_cast<int32_t*>(nullptr));
        return hipGetLastError();
    });
}

hipError_t launch_cg_dir(double* p, const double* z, int64_t n, int m, const double* rz_new, const double* zro,
                         const double* rz_old, const int32_t* active, hipStream_t st, const float* z32) {
    const unsigned g = kry_grid(n);
    return for_chunks(m, [&](int c0, int w) {
        if (co_ok(m, w)) {
            CO_DISPATCH(w, k_cg_dir_co, dim3(g), dim3(WG), 0, st, p, z, n, rz_new, zro, rz_old, active, z32)
        } else {
            KRY_DISPATCH(w, k_cg_dir, dim3(g), dim3(WG), 0, st, p + c0, z ? z + c0 : nullptr, n, m, rz_new + c0,
                         zro ? zro + c0 : nullptr, rz_old + c0, active + c0, z32 ? z32 + c0 : nullptr)
        }
        return hipGetLastError();
    });
}

__global__ void k_copy_cols(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int m,
                            const int32_t* __restrict__ mask) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * m) return;
    if (mask[t % m]) dst[t] = src[t];
}

hipError_t launch_copy_cols(const double* src, double* dst, int64_t n, int m, const int32_t* mask, hipStream_t st) {
    if (n * m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_cols, dim3(grid_for(n * m)), dim3(WG), 0, st, src, dst, n, m, mask);
    return hipGetLastError();
}

// dense y = A x, one workgroup per row: its 256 threads stride the columns,
// each keeping 4 loads of the row (and of x) in flight, and the four waves'
// partial sums are added in a fixed order through LDS.  A and the sums are
// FP64; x and y are of type V (FP32 vectors are widened on load and the
// result rounded once on store).
template <typename V, int M>
__global__ __launch_bounds__(WG) void k_gemv(const double* __restrict__ A, const V* __restrict__ x,
                                             V* __restrict__ y, int64_t n, int ld) {
    constexpr int U = 4;
    __shared__ double red[WAVES_PER_WG][M];
    const int64_t row = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = 0.0;
    const double* __restrict__ Ar = A + row * n;
    for (int64_t j0 = t; j0 < n; j0 += int64_t(WG) * U) {
        double a[U], xv[U][M];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + int64_t(u) * WG;
            a[u] = j < n ? Ar[j] : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) xv[u][c] = j < n ? double(x[j * ld + c]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + int64_t(u) * WG < n)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[c] += a[u] * xv[u][c];
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if (t < M) y[row * ld + t] = V((red[0][t] + red[1][t]) + (red[2][t] + red[3][t]));
}

template <typename V>
hipError_t launch_gemv(const double* Ainv, const V* x, V* y, int64_t n, int m, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 grid{unsigned(n), 1u, 1u};
    int c0 = 0;
    while (c0 < m) {
        const int rem = m - c0;
        const int w = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem;
        switch (w) {
            case 16: hipLaunchKernelGGL((k_gemv<V, 16>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
            case 8: hipLaunchKernelGGL((k_gemv<V, 8>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
            case 4: hipLaunchKernelGGL((k_gemv<V, 4>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
            case 3: hipLaunchKernelGGL((k_gemv<V, 3>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
            case 2: hipLaunchKernelGGL((k_gemv<V, 2>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
            default: hipLaunchKernelGGL((k_gemv<V, 1>), grid, dim3(WG), 0, st, Ainv, x + c0, y + c0, n, m); break;
        }
        c0 += w;
    }
    return hipGetLastError();
}
template hipError_t launch_gemv<double>(const double*, const double*, double*, int64_t, int, hipStream_t);
template hipError_t launch_gemv<float>(const double*, const float*, float*, int64_t, int, hipStream_t);

// Admission of one right-hand side into column c of a batch (row-major n x ld
// arrays): b is gathered from the caller's array (stride ldb, rows reordered by
// perm when perm != NULL) into kb and r; x takes x0 the same way, or 0; p and q
// are zeroed; the column's error flag is cleared.
__global__ void k_admit(const double* __restrict__ b, int64_t ldb, const double* __restrict__ x0, int64_t ldx,
                        const int64_t* __restrict__ perm, int64_t n_units, int nb, double* __restrict__ kb,
                        double* __restrict__ kx, double* __restrict__ r, double* __restrict__ p,
                        double* __restrict__ q, int ld, int c, int32_t* __restrict__ flag) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) flag[c] = 0;
    if (i >= n_units * nb) return;
    int64_t src = i;
    if (perm) {
        const int64_t u = i / nb;
        src = perm[u] * nb + (i - u * nb);
    }
    const int64_t e = i * ld + c;
    const double bv = b[src * ldb];
    kb[e] = bv;
    r[e] = bv;
    kx[e] = x0 ? x0[src * ldx] : 0.0;
    p[e] = 0.0;
    q[e] = 0.0;
}

hipError_t launch_admit(const double* b, int64_t ldb, const double* x0, int64_t ldx, const int64_t* perm,
                        int64_t n_units, int nb, double* kb, double* kx, double* r, double* p, double* q, int ld,
                        int c, int32_t* flag, hipStream_t st) {
    const int64_t n = std::max<int64_t>(n_units * nb, 1);
    hipLaunchKernelGGL(k_admit, dim3(grid_for(n)), dim3(WG), 0, st, b, ldb, x0, ldx, perm, n_units, nb, kb, kx, r, p,
                       q, ld, c, flag);
    return hipGetLastError();
}

// out[row(i) * ldo] = in[i * ldi] with row(i) the caller row of internal row i
// (identity when perm == NULL): one column out of a batch.
__global__ void k_scatter_col(const double* __restrict__ in, int64_t ldi, double* __restrict__ out, int64_t ldo,
                              const int64_t* __restrict__ perm, int64_t n_units, int nb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_units * nb) return;
    int64_t dst = i;
    if (perm) {
        const int64_t u = i / nb;
        dst = perm[u] * nb + (i - u * nb);
    }
    out[dst * ldo] = in[i * ldi];
}

hipError_t launch_scatter_col(const double* in, int64_t ldi, double* out, int64_t ldo, const int64_t* perm,
                              int64_t n_units, int nb, hipStream_t st) {
    const int64_t n = n_units * nb;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_col, dim3(grid_for(n)), dim3(WG), 0, st, in, ldi, out, ldo, perm, n_units, nb);
    return hipGetLastError();
}

// level-0 reordering between caller element order and internal order
template <typename Ti, typename To>
__global__ void k_permute(const Ti* __restrict__ in, To* __restrict__ out, const int64_t* __restrict__ perm,
                          int64_t n_units, int per_unit, int gather) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_units * per_unit) return;
    const int64_t u = t / per_unit;
    const int64_t w = t - u * per_unit;
    const int64_t ext = perm[u] * per_unit + w;
    if (gather) out[t] = To(in[ext]);
    else out[ext] = To(in[t]);
}

template <typename Ti, typename To>
hipError_t launch_permute(const Ti* in, To* out, const int64_t* perm, int64_t n_units, int nb, int m, int gather,
                          hipStream_t st) {
    const int64_t tot = n_units * nb * m;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL((k_permute<Ti, To>), dim3(grid_for(tot)), dim3(WG), 0, st, in, out, perm, n_units, nb * m,
                       gather);
    return hipGetLastError();
}
template hipError_t launch_permute<double, double>(const double*, double*, const int64_t*, int64_t, int, int, int, hipStream_t);
template hipError_t launch_permute<double, float>(const double*, float*, const int64_t*, int64_t, int, int, int, hipStream_t);
template hipError_t launch_permute<float, double>(const float*, double*, const int64_t*, int64_t, int, int, int, hipStream_t);
template hipError_t launch_permute<float, float>(const float*, float*, const int64_t*, int64_t, int, int, int, hipStream_t);

__global__ void k_scale_inv_norm(double* __restrict__ x, int64_t n, const double* __restrict__ nrm2) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) x[t] = x[t] / sqrt(nrm2[0]);
}

hipError_t launch_scale_by_inv_norm(double* x, int64_t n, const double* nrm2, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_inv_norm, dim3(grid_for(n)), dim3(WG), 0, st, x, n, nrm2);
    return hipGetLastError();
}

// h[j] = V[j] . w ; grid (parts, nv), fixed order
__global__ __launch_bounds__(WG) void k_multidot_part(const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w, int64_t n, double* __restrict__ part) {
    __shared__ double sh[WG];
    const int j = blockIdx.y;
    const double* v = V + int64_t(j) * ldv;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * WG + threadIdx.x; i < n; i += int64_t(gridDim.x) * WG) s += v[i] * w[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = sh[0];
}

hipError_t launch_multidot(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* part,
                           double* out, hipStream_t st) {
    // part must hold 256 * nv doubles
    const int np = int(std::min<int64_t>(256, std::max<int64_t>(1, (n + WG - 1) / WG)));
    hipLaunchKernelGGL(k_multidot_part, dim3(np, nv), dim3(WG), 0, st, V, ldv, w, n, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(WG), 0, st, part, np, nv, out);
    return hipGetLastError();
}

__global__ void k_multi_axpy(const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
                             double* __restrict__ w, int64_t n, double sign) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += V[int64_t(j) * ldv + i] * h[j];
    w[i] += sign * s;
}

hipError_t launch_multi_axpy(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n, double sign,
                             hipStream_t st) {
    if (n == 0 || nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n)), dim3(WG), 0, st, V, ldv, nv, h, w, n, sign);
    return hipGetLastError();
}

}  // namespace amgdg
