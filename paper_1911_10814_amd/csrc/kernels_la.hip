// Bandwidth-bound linear-algebra kernels for gfx950 (64-lane wavefronts):
// block-sparse SpMV family, rank-one outlet terms, CGS2 pieces with the
// Hessenberg/Givens update on the device, Chebyshev/aggregation V-cycle
// pieces, and the per-step set-up numerics.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ns {

namespace {

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

// The dispatcher hands workgroup b to XCD (b mod 8).  xcd_block() maps it to a
// logical block so that each XCD processes one contiguous range of rows; its
// own L2 then holds the x entries those rows gather instead of every XCD
// fetching all of x.  A bijection on [0, gridDim.x).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block() {
    const int64_t b = blockIdx.x, nb = gridDim.x;
    const int64_t x = b % kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

inline unsigned red_grid(int64_t n) {
    int64_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (g < 1) g = 1;
    if (g > kMaxRedBlocks) g = kMaxRedBlocks;
    return (unsigned)g;
}

template <typename T>
__device__ inline T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block (256 threads = 4 waves); result valid in thread 0.
template <typename T>
__device__ inline T block_sum(T v, T* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) lds[w] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) r = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return r;
}

__device__ inline int lower_bound_dev(const int32_t* a, int lo, int hi, int key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace

// ---------------------------------------------------------------------------
// SpMV: W lanes per block row, lanes stride over the row's blocks (consecutive
// lanes read consecutive blocks of every value plane: coalesced), x gathered
// through L2, butterfly reduction of the BR partial sums inside the group.
// ---------------------------------------------------------------------------

// Kernel timing: events that the next launch of a timed kernel class records
// at its own start and end (hipExtLaunchKernelGGL), so the measured duration
// has no dispatch gap of a separate event record in it.
namespace {
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
}
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    g_ev_start = start;
    g_ev_stop = stop;
}
bool launch_events_pending() { return g_ev_start != nullptr; }

template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
    if (g_ev_start) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, g_ev_start, g_ev_stop, 0, args...);
        g_ev_start = g_ev_stop = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    }
}

// A timed class of several launches in sequence: the first records the start
// event at its own start, the last the stop event at its own end.
template <typename K, typename... Args>
void launch_span(K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t st, bool first, bool last,
                 Args... args) {
    hipEvent_t e0 = first ? g_ev_start : nullptr, e1 = last ? g_ev_stop : nullptr;
    if (e0 || e1) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, e0, e1, 0, args...);
        if (first) g_ev_start = nullptr;
        if (last) g_ev_stop = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
    }
}

// A lane's walk over its row's blocks k = kb + lane + m W, U blocks per trip:
// every load of a trip (column indices, value planes, then the gathers that
// depend on the columns) is issued before any is used, and all lanes of a
// row take the same trips (no divergent remainder).  A block at or past the
// row end repeats the trip's first (an address already being fetched) and
// adds nothing.  Blocks are accumulated in the order of k either way.
template <int U>
__device__ inline void trip_blocks(int k0, int ke, int W, int (&kk)[U], bool (&on)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + u * W;
        on[u] = k < ke;
        kk[u] = on[u] ? k : k0;
    }
}

template <typename T, int BR, int BC, int W, int U>
__global__ __launch_bounds__(kBlock) void k_spmv(BlockOp<T> M, const T* __restrict__ x, T* __restrict__ y, T alpha,
                                                 const T* __restrict__ z, T beta, const T* __restrict__ rscale,
                                                 RankOne<T> ro, FirstStep<T> fs) {
    const int64_t tid = (M.xcd ? xcd_block() : (int64_t)blockIdx.x) * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < M.n;
    // The row bounds, then the epilogue's own-row operands: loads only (no
    // arithmetic or branch on a loaded value before the row loop), so they
    // are all in flight together and the loop waits once; the rank-one
    // term's dependent loads follow the loop.
    int kb = 0, ke = 0;
    if (valid) {
        if (M.ell) {
            kb = row * M.ell;
            ke = kb + M.ell;
        } else {
            kb = M.rp[row];
            ke = M.rp[row + 1];
        }
    }
    const bool out_lane = valid && lane < BR;
    const int64_t i = (int64_t)BR * row + lane;
    T dxi = 0, xii = 0, zi = 0, rsi = 1, fdv = 0;
    int sl = -1;
    if (out_lane) {
        if (M.dextra) {
            dxi = M.dextra[i];
            xii = x[i];
        }
        if (z) zi = z[i];
        if (rscale) rsi = rscale[i];
        if (fs.x) fdv = fs.dinv[i];
        if (ro.slot_of) sl = ro.slot_of[row];
    }
    T acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0;
    // the column source (16-bit offsets from the row, or 32-bit columns) is
    // chosen once, outside the walk, so that a trip's loads issue together
    auto walk = [&](auto column) {
        for (int k0 = kb + lane; k0 < ke; k0 += U * W) {
            int kk[U];
            bool on[U];
            trip_blocks<U>(k0, ke, W, kk, on);
            int j[U];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = column(kk[u]);
            T v[U][BR * BC];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < BR; ++r)
#pragma unroll
                    for (int c = 0; c < BC; ++c) v[u][r * BC + c] = M.v[r * M.rs + c * M.cs + kk[u]];
            T xj[U][BC];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < BC; ++c) xj[u][c] = x[(int64_t)BC * j[u] + c];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < BR; ++r)
#pragma unroll
                    for (int c = 0; c < BC; ++c) acc[r] += v[u][r * BC + c] * (on[u] ? xj[u][c] : T(0));
        }
    };
    if (M.dcol)
        walk([&](int k) { return row + (int)M.dcol[k]; });
    else
        walk([&](int k) { return M.col[k]; });
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < BR; ++r) acc[r] += __shfl_xor(acc[r], off, W);
    if (!out_lane) return;
    T s = acc[0];
#pragma unroll
    for (int r = 1; r < BR; ++r)
        if (lane == r) s = acc[r];
    {
        // each extra term is rounded before it is added
#pragma clang fp contract(off)
        if (M.dextra) s += dxi * xii;
        if (ro.slot_of) {
            T r1 = 0;
            if (sl >= 0) r1 = ro.s[ro.oid[sl]] * ro.aval[3 * (int64_t)sl + lane];
            s += r1;
        }
    }
    T out = alpha * s;
    if (z) out += beta * zi;
    if (rscale) out *= rsi;
    y[i] = out;
    if (fs.x) {
        const T di = (fs.coef[0] * fdv) * out;
        fs.x[i] = di;
        fs.d[i] = di;
    }
}

template <typename T, int BR, int BC>
void spmv_w(const BlockOp<T>& M, const T* x, T* y, T alpha, const T* z, T beta, const T* rscale,
            const RankOne<T>& r1, const FirstStep<T>& fs, hipStream_t st) {
    switch (M.lanes) {
        case 64:
            launch_timed(k_spmv<T, BR, BC, 64, 1>, dim3(grid_for((int64_t)M.n * 64)), dim3(kBlock), st, M, x, y,
                         alpha, z, beta, rscale, r1, fs);
            break;
        case 32:
            launch_timed(k_spmv<T, BR, BC, 32, 1>, dim3(grid_for((int64_t)M.n * 32)), dim3(kBlock), st, M, x, y,
                         alpha, z, beta, rscale, r1, fs);
            break;
        case 4:
            if (M.unroll == 4)
                launch_timed(k_spmv<T, BR, BC, 4, 8>, dim3(grid_for((int64_t)M.n * 4)), dim3(kBlock), st, M, x, y,
                             alpha, z, beta, rscale, r1, fs);
            else
                launch_timed(k_spmv<T, BR, BC, 4, 4>, dim3(grid_for((int64_t)M.n * 4)), dim3(kBlock), st, M, x, y,
                             alpha, z, beta, rscale, r1, fs);
            break;
        case 8:
            if (M.unroll == 4)
                launch_timed(k_spmv<T, BR, BC, 8, 4>, dim3(grid_for((int64_t)M.n * 8)), dim3(kBlock), st, M, x, y,
                             alpha, z, beta, rscale, r1, fs);
            else
                launch_timed(k_spmv<T, BR, BC, 8, 2>, dim3(grid_for((int64_t)M.n * 8)), dim3(kBlock), st, M, x, y,
                             alpha, z, beta, rscale, r1, fs);
            break;
        default:
            launch_timed(k_spmv<T, BR, BC, 16, 1>, dim3(grid_for((int64_t)M.n * 16)), dim3(kBlock), st, M, x, y,
                         alpha, z, beta, rscale, r1, fs);
    }
}

template <typename T>
void spmv(int br, int bc, const BlockOp<T>& M, const T* x, T* y, T alpha, const T* z, T beta, const T* rscale,
          const RankOne<T>* ro, hipStream_t st, const FirstStep<T>* fsp) {
    RankOne<T> r1 = ro ? *ro : RankOne<T>{};
    FirstStep<T> fs = fsp ? *fsp : FirstStep<T>{};
    if (M.n <= 0) return;
    if (M.ell && !M.dcol) throw std::runtime_error("spmv: fixed-width rows need their column offsets");
    if (br == 3 && bc == 3)
        spmv_w<T, 3, 3>(M, x, y, alpha, z, beta, rscale, r1, fs, st);
    else if (br == 3 && bc == 1)
        spmv_w<T, 3, 1>(M, x, y, alpha, z, beta, rscale, r1, fs, st);
    else if (br == 1 && bc == 3)
        spmv_w<T, 1, 3>(M, x, y, alpha, z, beta, rscale, r1, fs, st);
    else
        spmv_w<T, 1, 1>(M, x, y, alpha, z, beta, rscale, r1, fs, st);
}

// Full field-split 4x4 operator (outer Arnoldi and true residual).
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_spmv_full(int n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col, const T* __restrict__ V,
                                                      int64_t nnzb, const T* __restrict__ x, T* __restrict__ y,
                                                      T alpha, const T* __restrict__ z, T beta, RankOne<T> ro,
                                                      int ell, const int16_t* __restrict__ dcol) {
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < n;
    const T* xp = x + 3 * (int64_t)n;
    // own-row epilogue operands, loaded ahead of the row loop
    const int64_t i = lane < 3 ? 3 * (int64_t)row + lane : 3 * (int64_t)n + row;
    T zi = 0, r1 = 0;
    if (valid && lane < 4) {
        if (z) zi = z[i];
        if (lane < 3 && ro.slot_of) {
            const int sl = ro.slot_of[row];
            if (sl >= 0) r1 = ro.s[ro.oid[sl]] * ro.aval[3 * (int64_t)sl + lane];
        }
    }
    T acc[4] = {0, 0, 0, 0};
    if (valid) {
        const int k0 = ell ? row * ell : rp[row];
        const int k1 = ell ? k0 + ell : rp[row + 1];
        for (int k = k0 + lane; k < k1; k += W) {
            const int j = ell ? row + dcol[k] : col[k];
            T xj[4] = {x[3 * (int64_t)j], x[3 * (int64_t)j + 1], x[3 * (int64_t)j + 2], xp[j]};
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r] += V[(4 * r + c) * nnzb + k] * xj[c];
        }
    }
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += __shfl_xor(acc[r], off, W);
    if (!valid || lane >= 4) return;
    T s = acc[0];
    if (lane == 1) s = acc[1];
    if (lane == 2) s = acc[2];
    if (lane == 3) s = acc[3];
    if (lane < 3 && ro.slot_of) s += r1;
    T out = alpha * s;
    if (z) out += beta * zi;
    y[i] = out;
}

template <typename T>
void spmv_full(int n, const int32_t* rp, const int32_t* col, const T* V, int64_t nnzb, const T* x, T* y, T alpha,
               const T* z, T beta, const RankOne<T>* ro, hipStream_t st, int ell, const int16_t* dcol_ell) {
    RankOne<T> r1 = ro ? *ro : RankOne<T>{};
    if (ell && !dcol_ell) throw std::runtime_error("spmv_full: fixed-width rows need their column offsets");
    launch_timed(k_spmv_full<T, 16>, dim3(grid_for((int64_t)n * 16)), dim3(kBlock), st, n, rp, col, V, nnzb, x, y,
                 alpha, z, beta, r1, ell, dcol_ell);
}

// Fixed-width row layout: thread (row, l) copies slot l of the row from every
// plane, writing zero past the row's end.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_to_ell(int n, int ell, const int32_t* __restrict__ rp,
                                                   const Tin* __restrict__ src, int64_t nnzb, int planes,
                                                   Tout* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t total = (int64_t)n * ell;
    if (t >= total) return;
    const int row = (int)(t / ell);
    const int l = (int)(t - (int64_t)row * ell);
    const int k = rp[row] + l;
    const bool in = k < rp[row + 1];
    for (int p = 0; p < planes; ++p) dst[p * total + t] = in ? (Tout)src[p * nnzb + k] : Tout(0);
}

template <typename Tin, typename Tout>
void to_ell(int n, int ell, const int32_t* rp, const Tin* src, int64_t nnzb, int planes, Tout* dst, hipStream_t st) {
    const int64_t total = (int64_t)n * ell;
    if (total <= 0) return;
    hipLaunchKernelGGL((k_to_ell<Tin, Tout>), dim3(grid_for(total)), dim3(kBlock), 0, st, n, ell, rp, src, nnzb,
                       planes, dst);
}
template void to_ell<double, float>(int, int, const int32_t*, const double*, int64_t, int, float*, hipStream_t);

// s[k] = c[k] * sum over outlet k's slots of a . x   (one block per outlet)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_outlet_dot(const int32_t* optr, const int32_t* onode, const T* aval,
                                                       const T* c, const T* x, T* s) {
    __shared__ T lds[4];
    const int k = blockIdx.x;
    const int end = optr[k + 1];
    T acc = 0;
    // four slots per trip, all loads issued before the first sum; the slots
    // are still added one by one in the order of sl
    int sl = optr[k] + threadIdx.x;
    for (; sl + 3 * kBlock < end; sl += 4 * kBlock) {
        int64_t nd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) nd[u] = onode[sl + u * kBlock];
        T a[4][3], xv[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) a[u][c] = aval[3 * (int64_t)(sl + u * kBlock) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) xv[u][c] = x[3 * nd[u] + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += a[u][0] * xv[u][0] + a[u][1] * xv[u][1] + a[u][2] * xv[u][2];
    }
    for (; sl < end; sl += kBlock) {
        const int64_t nd = onode[sl];
        acc += aval[3 * (int64_t)sl] * x[3 * nd] + aval[3 * (int64_t)sl + 1] * x[3 * nd + 1] +
               aval[3 * (int64_t)sl + 2] * x[3 * nd + 2];
    }
    T tot = block_sum(acc, lds);
    if (threadIdx.x == 0) s[k] = (c ? c[k] : T(1)) * tot;
}

template <typename T>
void outlet_dot(int n_out, const int32_t* optr, const int32_t* onode, const T* aval, const T* c, const T* x, T* s,
                hipStream_t st) {
    if (n_out <= 0) return;
    hipLaunchKernelGGL((k_outlet_dot<T>), dim3(n_out), dim3(kBlock), 0, st, optr, onode, aval, c, x, s);
}

// ---------------------------------------------------------------------------
// BLAS-1
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_axpby(int64_t n, T a, const T* x, T b, const T* y, T* out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = a * x[i] + (y ? b * y[i] : T(0));
}
template <typename T>
void axpby(int64_t n, T a, const T* x, T b, const T* y, T* out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_axpby<T>), dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n, a, x, b,
                       y, out);
}

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t n, const Tin* x, Tout* y) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = (Tout)x[i];
}
template <typename Tin, typename Tout>
void convert(int64_t n, const Tin* x, Tout* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n,
                       x, y);
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T* y) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) y[i] = v;
}
template <typename T>
void fill(int64_t n, T val, T* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_fill<T>), dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n, val, y);
}

template <typename T>
__global__ void k_mul(int64_t n, const T* a, const T* x, T* y) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = a[i] * x[i];
}
template <typename T>
void mul(int64_t n, const T* a, const T* x, T* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_mul<T>), dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n, a, x, y);
}

// ---------------------------------------------------------------------------
// CGS2 pieces, without device-scope fences: a kernel writes per-block partial
// sums and the NEXT kernel (after the kernel boundary made them visible)
// reduces them in every block in a fixed order (deterministic).
//   multidot:    partials of V_i . w (i < k) and w . w -> red1[i][G]
//   orth_dot:    h1 = reduce(red1); w -= V h1; partials of V_i . w -> red2
//   orth_update: h2 = reduce(red2); w -= V h2; partials of ||w||^2 -> red3
//   finish:      ||w||^2 = reduce(red3); block 0 updates the Hessenberg
//                column and Givens rotation; every block scales w by 1/||w||
// All four use the same G blocks of kCgsBlock threads, each thread owning
// the same 16-byte packs of w in every kernel.
// ---------------------------------------------------------------------------

constexpr int kDotGroup = 16;
constexpr int kCgsBlock = 512;
constexpr int kCgsWaves = kCgsBlock / 64;

// 16-byte packs (4 floats or 2 doubles): the Krylov basis rows are padded to
// a multiple of 64 elements and 256-byte aligned, so every pack load is one
// aligned 128-bit access; elements at or beyond n read as zero.
template <typename T>
struct alignas(16) Pk {
    static constexpr int W = 16 / sizeof(T);
    T e[W];
};

template <typename T>
__device__ inline Pk<T> ld_pk(const T* __restrict__ p, int64_t q, int64_t n) {
    constexpr int W = Pk<T>::W;
    Pk<T> v = reinterpret_cast<const Pk<T>*>(p)[q];
    if ((q + 1) * W > n) {
#pragma unroll
        for (int e = 0; e < W; ++e)
            if (q * W + e >= n) v.e[e] = T(0);
    }
    return v;
}
// A run of pack loads issued back to back (no branch between them), the
// tail of the last pack of the vectors zeroed afterwards: raw loads, then
// pk_tail on each.
template <typename T>
__device__ inline Pk<T> ld_pk_raw(const T* __restrict__ p, int64_t q) {
    return reinterpret_cast<const Pk<T>*>(p)[q];
}
template <typename T>
__device__ inline void pk_tail(Pk<T>& v, int64_t q, int64_t n) {
#pragma unroll
    for (int e = 0; e < Pk<T>::W; ++e)
        if (q * Pk<T>::W + e >= n) v.e[e] = T(0);
}
template <typename T>
__device__ inline T pk_dot(const Pk<T>& a, const Pk<T>& b) {
    T s = 0;
#pragma unroll
    for (int e = 0; e < Pk<T>::W; ++e) s += a.e[e] * b.e[e];
    return s;
}

template <typename T>
__host__ __device__ inline int64_t n_packs(int64_t n) {
    return (n + Pk<T>::W - 1) / Pk<T>::W;
}

// Blocks of every CGS2 kernel for a vector of length n: about one pack per
// thread, at most kCgsMaxBlocks partial sums per reduced value (two blocks of
// 512 threads per CU; measured on the 4e6-node contraction-expansion against
// 256, 1024 and 2048 blocks: 298 against 318, 311 and 370 us per Arnoldi step
// of the A-solves, 1207 against 1319, 1360 and 1651 us on the S_hat solve's
// long bases).  The partials fit the reduction buffer: (2k + 2) kCgsMaxBlocks
// values for k <= mmax basis vectors.
constexpr int64_t kCgsMaxBlocks = 512;
static_assert(2 * kCgsMaxBlocks <= kMaxRedBlocks, "CGS2 partials exceed the reduction buffer");
template <typename T>
inline unsigned cgs_grid(int64_t n) {
    const int64_t g = (n_packs<T>(n) + kCgsBlock - 1) / kCgsBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, kCgsMaxBlocks));
}

// every block: out_lds[i] = sum_b red[i*G + b] for i < nv (one wave per
// value); a lane's first kRedLoads partials are all loaded before any is
// added, and every lane adds its partials in order of b
constexpr int kRedLoads = 8;
static_assert(kCgsMaxBlocks <= 64 * kRedLoads, "CGS2 partials: one round of loads per lane");
template <typename T>
__device__ inline void block_reduce_partials(const T* __restrict__ red, int nv, unsigned G, T* out_lds) {
    const int nw = blockDim.x >> 6;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wv; i < nv; i += nw) {
        T p[kRedLoads];
#pragma unroll
        for (int u = 0; u < kRedLoads; ++u) {
            const unsigned b = lane + 64u * u;
            p[u] = b < G ? red[(int64_t)i * G + b] : T(0);
        }
        T s = 0;
#pragma unroll
        for (int u = 0; u < kRedLoads; ++u) s += p[u];
        for (unsigned b = lane + 64u * kRedLoads; b < G; b += 64) s += red[(int64_t)i * G + b];
        s = wave_sum(s);
        if (lane == 0) out_lds[i] = s;
    }
    __syncthreads();
}

// Block sums of K per-thread accumulators (kCgsBlock threads) written as
// partials red[g * gridDim.x + blockIdx.x] for g < cnt; one barrier.
template <typename T, int K>
__device__ inline void block_partials(const T (&acc)[K], int cnt, T* lds, T* __restrict__ red) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int g = 0; g < K; ++g) {
        if (g >= cnt) break;
        const T s = wave_sum(acc[g]);
        if (lane == 0) lds[wv * K + g] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        T s = 0;
#pragma unroll
        for (int w = 0; w < kCgsWaves; ++w) s += lds[w * K + threadIdx.x];
        red[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
}

// Givens update of Hessenberg column j (FP64, one thread).
__device__ void givens_step(const GivensArgs& a, double hn2) {
    const int j = a.j, ld = a.ldh;
    double* Hc = a.H + (int64_t)j * ld;
    for (int i = 0; i <= j; ++i) Hc[i] = a.h1[i] + a.h2[i];
    const double hn = sqrt(hn2);
    const double wpre = sqrt(a.h1[j + 1]);
    Hc[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = a.cs[i] * Hc[i] + a.sn[i] * Hc[i + 1];
        Hc[i + 1] = -a.sn[i] * Hc[i] + a.cs[i] * Hc[i + 1];
        Hc[i] = t;
    }
    const double rho = hypot(Hc[j], Hc[j + 1]);
    if (rho == 0.0) {
        a.cs[j] = 1.0;
        a.sn[j] = 0.0;
    } else {
        a.cs[j] = Hc[j] / rho;
        a.sn[j] = Hc[j + 1] / rho;
    }
    Hc[j] = rho;
    Hc[j + 1] = 0.0;
    a.g[j + 1] = -a.sn[j] * a.g[j];
    a.g[j] = a.cs[j] * a.g[j];
    const bool bd = !(hn > 1e-14 * wpre);
    a.status[0] = fabs(a.g[j + 1]);
    a.status[1] = bd ? 1.0 : 0.0;
    a.status[2] = bd ? 0.0 : 1.0 / hn;
    a.status[3] = wpre;
    if (a.hstatus) {
        a.hstatus[0] = a.status[0];
        a.hstatus[1] = a.status[1];
    }
    if (a.hseq) __hip_atomic_store(a.hseq, a.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

inline unsigned orth_grid(int64_t n) {
    int64_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

// Pass-1 dot products: partials of V_i . w (i < k) and of w . w (i = k),
// kDotGroup values per blockIdx.y.
template <typename T>
__global__ __launch_bounds__(kCgsBlock) void k_multidot(int64_t n, int k, const T* __restrict__ V, int64_t ldv,
                                                        const T* __restrict__ w, T* __restrict__ red) {
    __shared__ T lds[kCgsWaves * kDotGroup];
    const int i0 = blockIdx.y * kDotGroup;
    const int64_t np = n_packs<T>(n);
    T acc[kDotGroup];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) acc[g] = 0;
    for (int64_t q = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x; q < np; q += (int64_t)gridDim.x * kCgsBlock) {
        // every pack of the group is loaded before the first is used
        Pk<T> wp = ld_pk_raw(w, q);
        Pk<T> v[kDotGroup];
#pragma unroll
        for (int g = 0; g < kDotGroup; ++g)
            if (i0 + g < k) v[g] = ld_pk_raw(V + (int64_t)(i0 + g) * ldv, q);
        if ((q + 1) * Pk<T>::W > n) {
            pk_tail(wp, q, n);
#pragma unroll
            for (int g = 0; g < kDotGroup; ++g) pk_tail(v[g], q, n);
        }
#pragma unroll
        for (int g = 0; g < kDotGroup; ++g) {
            const int i = i0 + g;
            if (i < k) acc[g] += pk_dot(v[g], wp);
            else if (i == k) acc[g] += pk_dot(wp, wp);
        }
    }
    block_partials<T, kDotGroup>(acc, min(kDotGroup, k + 1 - i0), lds, red + (int64_t)i0 * gridDim.x);
}

// w -= sum_{i<k} V_i hs_i over this block's packs; returns the sum of the
// squares of the updated entries this thread owns.
constexpr int kSubLoads = 8;
template <typename T>
__device__ inline T orth_subtract(int64_t n, int k, const T* __restrict__ V, int64_t ldv, const T* hs,
                                  T* __restrict__ w) {
    const int64_t np = n_packs<T>(n);
    T sq = 0;
    for (int64_t q = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x; q < np; q += (int64_t)gridDim.x * kCgsBlock) {
        Pk<T> s;
#pragma unroll
        for (int e = 0; e < Pk<T>::W; ++e) s.e[e] = 0;
        // kSubLoads packs in flight at a time, added in the order of i
        for (int i0 = 0; i0 < k; i0 += kSubLoads) {
            Pk<T> v[kSubLoads];
#pragma unroll
            for (int u = 0; u < kSubLoads; ++u)
                if (i0 + u < k) v[u] = ld_pk_raw(V + (int64_t)(i0 + u) * ldv, q);
            if ((q + 1) * Pk<T>::W > n) {
#pragma unroll
                for (int u = 0; u < kSubLoads; ++u) pk_tail(v[u], q, n);
            }
#pragma unroll
            for (int u = 0; u < kSubLoads; ++u)
                if (i0 + u < k) {
                    const T h = hs[i0 + u];
#pragma unroll
                    for (int e = 0; e < Pk<T>::W; ++e) s.e[e] += v[u].e[e] * h;
                }
        }
        Pk<T> wp = ld_pk(w, q, n);
#pragma unroll
        for (int e = 0; e < Pk<T>::W; ++e) {
            wp.e[e] -= s.e[e];
            sq += wp.e[e] * wp.e[e];
        }
        reinterpret_cast<Pk<T>*>(w)[q] = wp;
    }
    return sq;
}

// Pass-1 update fused with the pass-2 dot products: h1 = reduce(red1);
// w -= V h1 over this block's packs, then partials of V_i . w over the same
// packs (written by this block, so no grid synchronisation is needed) into
// red2[i][blockIdx.x].
template <typename T>
__global__ __launch_bounds__(kCgsBlock) void k_orth_dot(int64_t n, int k, const T* __restrict__ V, int64_t ldv,
                                                        const T* __restrict__ red1, unsigned G1,
                                                        double* __restrict__ h1, T* __restrict__ w,
                                                        T* __restrict__ red2) {
    extern __shared__ char smem[];
    T* hs = reinterpret_cast<T*>(smem);
    __shared__ T lds[kCgsWaves * kDotGroup];
    block_reduce_partials<T>(red1, k + 1, G1, hs);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i <= k; i += kCgsBlock) h1[i] = (double)hs[i];
    const int64_t np = n_packs<T>(n);
    if (k <= kOrthFuseMax) {
        // Short bases (the A-level solves): each thread keeps its packs of
        // V_0..V_{k-1} in registers, so the update and the pass-2 dots read V
        // once; the sums are the same, in the same order, as the two-pass form.
        T acc[kOrthFuseMax];
#pragma unroll
        for (int i = 0; i < kOrthFuseMax; ++i) acc[i] = 0;
        for (int64_t q = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x; q < np;
             q += (int64_t)gridDim.x * kCgsBlock) {
            Pk<T> v[kOrthFuseMax];
#pragma unroll
            for (int i = 0; i < kOrthFuseMax; ++i)
                if (i < k) v[i] = ld_pk(V + (int64_t)i * ldv, q, n);
            Pk<T> sv;
#pragma unroll
            for (int e = 0; e < Pk<T>::W; ++e) sv.e[e] = 0;
#pragma unroll
            for (int i = 0; i < kOrthFuseMax; ++i)
                if (i < k) {
                    const T h = hs[i];
#pragma unroll
                    for (int e = 0; e < Pk<T>::W; ++e) sv.e[e] += v[i].e[e] * h;
                }
            Pk<T> wp = ld_pk(w, q, n);
#pragma unroll
            for (int e = 0; e < Pk<T>::W; ++e) wp.e[e] -= sv.e[e];
            reinterpret_cast<Pk<T>*>(w)[q] = wp;
#pragma unroll
            for (int i = 0; i < kOrthFuseMax; ++i)
                if (i < k) acc[i] += pk_dot(v[i], wp);
        }
        static_assert(kOrthFuseMax == kDotGroup, "one group of pass-2 partials");
        block_partials<T, kDotGroup>(acc, k, lds, red2);
        return;
    }
    (void)orth_subtract<T>(n, k, V, ldv, hs, w);
    for (int i0 = 0; i0 < k; i0 += kDotGroup) {
        T acc[kDotGroup];
#pragma unroll
        for (int g = 0; g < kDotGroup; ++g) acc[g] = 0;
        for (int64_t q = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x; q < np;
             q += (int64_t)gridDim.x * kCgsBlock) {
            Pk<T> wp = ld_pk_raw(w, q);
            Pk<T> v[kDotGroup];
#pragma unroll
            for (int g = 0; g < kDotGroup; ++g)
                if (i0 + g < k) v[g] = ld_pk_raw(V + (int64_t)(i0 + g) * ldv, q);
            if ((q + 1) * Pk<T>::W > n) {
                pk_tail(wp, q, n);
#pragma unroll
                for (int g = 0; g < kDotGroup; ++g) pk_tail(v[g], q, n);
            }
#pragma unroll
            for (int g = 0; g < kDotGroup; ++g)
                if (i0 + g < k) acc[g] += pk_dot(v[g], wp);
        }
        block_partials<T, kDotGroup>(acc, min(kDotGroup, k - i0), lds, red2 + (int64_t)i0 * gridDim.x);
    }
}

// h2 = reduce(red2) (every block); block 0 stores h2 (FP64); w -= V h2;
// partials of ||w||^2 into red3[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(kCgsBlock) void k_orth_update(int64_t n, int k, const T* __restrict__ V, int64_t ldv,
                                                           const T* __restrict__ red2, unsigned G2,
                                                           double* __restrict__ h2, T* __restrict__ w,
                                                           T* __restrict__ red3) {
    extern __shared__ char smem[];
    T* hs = reinterpret_cast<T*>(smem);
    __shared__ T lds[kCgsWaves];
    block_reduce_partials<T>(red2, k, G2, hs);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += kCgsBlock) h2[i] = (double)hs[i];
    const T acc[1] = {orth_subtract<T>(n, k, V, ldv, hs, w)};
    block_partials<T, 1>(acc, 1, lds, red3);
}

// ||w||^2 = reduce(red3); Givens update (block 0); w *= 1/||w|| unless breakdown
template <typename T>
__global__ __launch_bounds__(kCgsBlock) void k_finish(int64_t n, T* __restrict__ w, const T* __restrict__ red3,
                                                      unsigned G3, GivensArgs ga) {
    __shared__ T tot[1];
    block_reduce_partials<T>(red3, 1, G3, tot);
    const double hn2 = (double)tot[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) givens_step(ga, hn2);
    const double hn = sqrt(hn2);
    const double wpre = sqrt(ga.h1[ga.j + 1]);
    if (!(hn > 1e-14 * wpre)) return;
    const T s = (T)(1.0 / hn);
    const int64_t np = n_packs<T>(n);
    const int64_t stride = (int64_t)gridDim.x * kCgsBlock;
    int64_t q = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x;
    // four packs per trip, loaded together
    for (; q + 3 * stride < np; q += 4 * stride) {
        Pk<T> wp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) wp[u] = ld_pk_raw(w, q + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if ((q + u * stride + 1) * Pk<T>::W > n) pk_tail(wp[u], q + u * stride, n);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int e = 0; e < Pk<T>::W; ++e) wp[u].e[e] *= s;
            reinterpret_cast<Pk<T>*>(w)[q + u * stride] = wp[u];
        }
    }
    for (; q < np; q += stride) {
        Pk<T> wp = ld_pk(w, q, n);
#pragma unroll
        for (int e = 0; e < Pk<T>::W; ++e) wp.e[e] *= s;
        reinterpret_cast<Pk<T>*>(w)[q] = wp;
    }
}

template <typename T>
void arnoldi_cgs2(int64_t n, int j, const T* V, int64_t ldv, T* w, double* h1, double* h2, const GivensArgs& ga,
                  double* red, hipStream_t st) {
    const int k = j + 1;
    const unsigned G = cgs_grid<T>(n);
    T* r1 = reinterpret_cast<T*>(red);
    T* r2 = r1 + (int64_t)(k + 1) * G;
    T* r3 = r2 + (int64_t)k * G;
    launch_span(k_multidot<T>, dim3(G, (k + 1 + kDotGroup - 1) / kDotGroup), dim3(kCgsBlock), 0, st, true, false,
                n, k, V, ldv, (const T*)w, r1);
    launch_span(k_orth_dot<T>, dim3(G), dim3(kCgsBlock), (k + 1) * sizeof(T), st, false, false, n, k, V, ldv,
                (const T*)r1, G, h1, w, r2);
    launch_span(k_orth_update<T>, dim3(G), dim3(kCgsBlock), k * sizeof(T), st, false, false, n, k, V, ldv,
                (const T*)r2, G, h2, w, r3);
    launch_span(k_finish<T>, dim3(G), dim3(kCgsBlock), 0, st, false, true, n, w, (const T*)r3, G, ga);
}

// Start of a GMRES cycle with the residual norm on the device: v /= nrm,
// g = [nrm, 0, ...].
template <typename T>
__global__ void k_start_cycle(int64_t n, T* __restrict__ v, const double* __restrict__ nrm, double* __restrict__ g,
                              int len) {
    const double s = nrm[0];
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < len; i += kBlock) g[i] = (i == 0) ? s : 0.0;
    const T f = (T)(1.0 / s);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        v[i] *= f;
}
template <typename T>
void start_cycle(int64_t n, T* v, const double* nrm, double* g, int len, hipStream_t st) {
    hipLaunchKernelGGL((k_start_cycle<T>), dim3(std::min<int64_t>(grid_for(n), 4096)), dim3(kBlock), 0, st, n, v, nrm,
                       g, len);
}

__global__ void k_init_g(double* g, int len, double beta) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = (i == 0) ? beta : 0.0;
}
void init_g(double* g, int len, double beta, hipStream_t st) {
    hipLaunchKernelGGL(k_init_g, dim3(1), dim3(kBlock), 0, st, g, len, beta);
}

__global__ void k_backsolve(int k, int ld, const double* H, const double* g, double* y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int c = i + 1; c < k; ++c) s -= H[(int64_t)c * ld + i] * y[c];
        y[i] = s / H[(int64_t)i * ld + i];
    }
}
void backsolve(int k, int ldh, const double* H, const double* g, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, st, k, ldh, H, g, y);
}

// x (+)= V y over the first k basis vectors: 16-byte packs of V per thread,
// eight vectors' packs loaded before they are used, each element's sum in FP64
// in the order of the basis.
constexpr int kCombineUnroll = 8;
template <typename T, typename TX>
__global__ __launch_bounds__(kBlock) void k_combine(int64_t n, int k, const T* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ y, TX* __restrict__ x, int acc) {
    constexpr int W = Pk<T>::W;
    __shared__ double ys[256];
    const int64_t np = n_packs<T>(n);
    for (int64_t q0 = (int64_t)blockIdx.x * kBlock; q0 < np; q0 += (int64_t)gridDim.x * kBlock) {
        const int64_t q = q0 + threadIdx.x;
        double s[W];
#pragma unroll
        for (int e = 0; e < W; ++e) s[e] = 0.0;
        for (int c0 = 0; c0 < k; c0 += 256) {
            const int cnt = min(256, k - c0);
            __syncthreads();
            if ((int)threadIdx.x < cnt) ys[threadIdx.x] = y[c0 + threadIdx.x];
            __syncthreads();
            if (q < np) {
                int i = 0;
                for (; i + kCombineUnroll <= cnt; i += kCombineUnroll) {
                    Pk<T> v[kCombineUnroll];
#pragma unroll
                    for (int u = 0; u < kCombineUnroll; ++u) v[u] = ld_pk_raw(V + (int64_t)(c0 + i + u) * ldv, q);
                    if ((q + 1) * W > n) {
#pragma unroll
                        for (int u = 0; u < kCombineUnroll; ++u) pk_tail(v[u], q, n);
                    }
#pragma unroll
                    for (int u = 0; u < kCombineUnroll; ++u)
#pragma unroll
                        for (int e = 0; e < W; ++e) s[e] += (double)v[u].e[e] * ys[i + u];
                }
                for (; i < cnt; ++i) {
                    const Pk<T> v = ld_pk(V + (int64_t)(c0 + i) * ldv, q, n);
#pragma unroll
                    for (int e = 0; e < W; ++e) s[e] += (double)v.e[e] * ys[i];
                }
            }
        }
        if (q < np) {
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int64_t t = q * W + e;
                if (t < n) x[t] = acc ? (TX)((double)x[t] + s[e]) : (TX)s[e];
            }
        }
    }
}
template <typename T, typename TX>
void combine(int64_t n, int k, const T* V, int64_t ldv, const double* y, TX* x, bool accumulate, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((n_packs<T>(n) + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL((k_combine<T, TX>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0, st, n,
                       k, V, ldv, y, x, accumulate ? 1 : 0);
}

// ||x||: partials, then a one-block finalisation
template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm2_part(int64_t n, const T* x, T* red) {
    __shared__ T lds[4];
    T acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kBlock)
        acc += x[t] * x[t];
    T s = block_sum(acc, lds);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm2_fin(const T* red, unsigned G, double* out, double* hout) {
    __shared__ T tot[1];
    block_reduce_partials<T>(red, 1, G, tot);
    if (threadIdx.x == 0) {
        out[0] = sqrt((double)tot[0]);
        if (hout) hout[0] = out[0];
    }
}
template <typename T>
void norm2(int64_t n, const T* x, double* out, double* red, hipStream_t st, double* hout) {
    const unsigned G = orth_grid(n);
    hipLaunchKernelGGL((k_norm2_part<T>), dim3(G), dim3(kBlock), 0, st, n, x, reinterpret_cast<T*>(red));
    hipLaunchKernelGGL((k_norm2_fin<T>), dim3(1), dim3(kBlock), 0, st, reinterpret_cast<const T*>(red), G, out,
                       hout);
}

template <typename T>
__global__ void k_scale_by(int64_t n, const T* x, const double* s, int inverse, T* y) {
    const double sv = inverse ? 1.0 / s[0] : s[0];
    const T f = (T)sv;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = x[i] * f;
}
template <typename T>
void scale_by(int64_t n, const T* x, const double* s, bool inverse, T* y, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_by<T>), dim3(std::min<int64_t>(grid_for(n), 4096)), dim3(kBlock), 0, st, n, x, s,
                       inverse ? 1 : 0, y);
}

// ---------------------------------------------------------------------------
// V-cycle pieces
// ---------------------------------------------------------------------------

// Chebyshev step coefficients live in device memory: coef[0] = 1/theta (first
// step: c1 = 0, c2 = 1/theta); step s >= 1: c1 = coef[2s-1], c2 = coef[2s].
template <typename T>
__device__ inline void cheb_coef(const T* coef, int s, T& c1, T& c2) {
    c1 = s == 0 ? T(0) : coef[2 * s - 1];
    c2 = s == 0 ? coef[0] : coef[2 * s];
}

template <typename T>
__global__ void k_cheb_first(int64_t n, const T* b, const T* dinv, const T* coef, T* x, T* d) {
    const T c2 = coef[0];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const T di = c2 * dinv[i] * b[i];
        d[i] = di;
        x[i] = di;
    }
}
template <typename T>
void cheb_first(int64_t n, const T* b, const T* dinv, const T* coef, T* x, T* d, hipStream_t st) {
    hipLaunchKernelGGL((k_cheb_first<T>), dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n, b,
                       dinv, coef, x, d);
}

// Fused residual + Chebyshev update: r = b - M x; d = c1 d + c2 dinv r; xout = x + d,
// where x = xin, or x = xin + P ec (prolongation of the coarse correction ec
// through the aggregate map) when agg != nullptr.
template <typename T, int BS, int W, int U>
__global__ __launch_bounds__(kBlock) void k_cheb_step(BlockOp<T> M, const T* __restrict__ xin, T* __restrict__ xout,
                                                      T* __restrict__ d, const T* __restrict__ b,
                                                      const T* __restrict__ dinv, const T* __restrict__ coef,
                                                      int step, const int32_t* __restrict__ agg,
                                                      const T* __restrict__ ec) {
    const int64_t tid = (M.xcd ? xcd_block() : (int64_t)blockIdx.x) * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < M.n;
    // The epilogue's own-row operands are loaded before the row loop, so their
    // latency overlaps the gathers instead of following the reduction: the
    // aggregate of the row first (its coarse correction is one more load),
    // then the row bounds and the rest, with no arithmetic on loaded values
    // before the loop.
    const bool out_lane = valid && lane < BS;
    const int64_t i = (int64_t)BS * row + lane;
    int ag = 0, kb = 0, ke = 0;
    if (out_lane && agg) ag = agg[row];
    if (valid) {
        if (M.ell) {
            kb = row * M.ell;
            ke = kb + M.ell;
        } else {
            kb = M.rp[row];
            ke = M.rp[row + 1];
        }
    }
    T xi = 0, eci = 0, ex = 0, bi = 0, dvi = 0, dprev = 0;
    if (out_lane) {
        xi = xin[i];
        if (M.dextra) ex = M.dextra[i];
        bi = b[i];
        dvi = dinv[i];
        if (step != 0) dprev = d[i];
        if (agg) eci = ec[(int64_t)BS * ag + lane];
    }
    T acc[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) acc[r] = 0;
    // the column source (16-bit offsets from the row, or 32-bit columns) is
    // chosen once, outside the walk, so that a trip's loads issue together
    auto walk = [&](auto column) {
        for (int k0 = kb + lane; k0 < ke; k0 += U * W) {
            int kk[U];
            bool on[U];
            trip_blocks<U>(k0, ke, W, kk, on);
            int j[U];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = column(kk[u]);
            T v[U][BS * BS];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < BS; ++r)
#pragma unroll
                    for (int c = 0; c < BS; ++c) v[u][r * BS + c] = M.v[r * M.rs + c * M.cs + kk[u]];
            T xj[U][BS];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < BS; ++c) xj[u][c] = xin[(int64_t)BS * j[u] + c];
            if (agg) {
                int J[U];
#pragma unroll
                for (int u = 0; u < U; ++u) J[u] = agg[j[u]];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int c = 0; c < BS; ++c) xj[u][c] += ec[(int64_t)BS * J[u] + c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < BS; ++r)
#pragma unroll
                    for (int c = 0; c < BS; ++c) acc[r] += v[u][r * BS + c] * (on[u] ? xj[u][c] : T(0));
        }
    };
    if (M.dcol)
        walk([&](int k) { return row + (int)M.dcol[k]; });
    else
        walk([&](int k) { return M.col[k]; });
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < BS; ++r) acc[r] += __shfl_xor(acc[r], off, W);
    if (!out_lane) return;
    if (agg) xi += eci;
    T s = acc[0];
#pragma unroll
    for (int r = 1; r < BS; ++r)
        if (lane == r) s = acc[r];
    if (M.dextra) s += ex * xi;
    T c1, c2;
    cheb_coef(coef, step, c1, c2);
    const T ri = bi - s;
    T di = c2 * dvi * ri;
    if (step != 0) di += c1 * dprev;
    d[i] = di;
    xout[i] = xi + di;
}

template <typename T, int BS>
void cheb_step_w(const BlockOp<T>& M, const T* xin, T* xout, T* d, const T* b, const T* dinv, const T* coef, int step,
                 const int32_t* agg, const T* ec, hipStream_t st) {
    switch (M.lanes) {
        case 64:
            launch_timed(k_cheb_step<T, BS, 64, 1>, dim3(grid_for((int64_t)M.n * 64)), dim3(kBlock), st, M, xin,
                         xout, d, b, dinv, coef, step, agg, ec);
            break;
        case 8:
            if (M.unroll == 4)
                launch_timed(k_cheb_step<T, BS, 8, 4>, dim3(grid_for((int64_t)M.n * 8)), dim3(kBlock), st, M, xin,
                             xout, d, b, dinv, coef, step, agg, ec);
            else
                launch_timed(k_cheb_step<T, BS, 8, 2>, dim3(grid_for((int64_t)M.n * 8)), dim3(kBlock), st, M, xin,
                             xout, d, b, dinv, coef, step, agg, ec);
            break;
        case 32:
            launch_timed(k_cheb_step<T, BS, 32, 1>, dim3(grid_for((int64_t)M.n * 32)), dim3(kBlock), st, M, xin,
                         xout, d, b, dinv, coef, step, agg, ec);
            break;
        default:
            launch_timed(k_cheb_step<T, BS, 16, 1>, dim3(grid_for((int64_t)M.n * 16)), dim3(kBlock), st, M, xin,
                         xout, d, b, dinv, coef, step, agg, ec);
    }
}

template <typename T>
void cheb_step(int bs, const BlockOp<T>& M, const T* xin, T* xout, T* d, const T* b, const T* dinv, const T* coef,
               int step, const int32_t* agg, const T* ec, hipStream_t st) {
    if (M.ell && !M.dcol) throw std::runtime_error("cheb_step: fixed-width rows need their column offsets");
    if (bs == 3)
        cheb_step_w<T, 3>(M, xin, xout, d, b, dinv, coef, step, agg, ec, st);
    else
        cheb_step_w<T, 1>(M, xin, xout, d, b, dinv, coef, step, agg, ec, st);
}

// Factored application of S_hat = D - C diag(A)^{-1} B on the finest pressure
// level, two passes over the node-block value planes (V: the 16 planes, B in
// planes 4r+3, C in planes 12+c, D in plane 15), instead of one pass over the
// explicit distance-2 pattern of S_hat (several times more gathers):
//   pass 1: t4[4i..4i+2] = dinvA .* (B xx), t4[4i+3] = xx_i
//   pass 2: s = D xx - C t, then the Chebyshev update with residual b - s
//           (coef != nullptr), else y = alpha s + beta z
// where xx = x, or x + P ec (prolongated coarse correction) when agg != nullptr.
// Pass 2 gathers one 4-wide record per block (the three t values and xx of
// the column node), so the aggregate map is read by pass 1 only.  Both passes
// walk their rows U blocks per lane per trip as the block SpMV does.
template <typename T>
struct Vec4 {
    T a, b, c, d;
};
__device__ inline Vec4<float> load4(const float* p) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    return {q.x, q.y, q.z, q.w};
}
__device__ inline Vec4<double> load4(const double* p) {
    const double2 q0 = reinterpret_cast<const double2*>(p)[0];
    const double2 q1 = reinterpret_cast<const double2*>(p)[1];
    return {q0.x, q0.y, q1.x, q1.y};
}

template <typename T, int W, bool AGG>
__global__ __launch_bounds__(kBlock) void k_sfact_bt(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int16_t* __restrict__ dcol, int ell,
                                                     const T* __restrict__ V,
                                                     int64_t nnzb, const T* __restrict__ dinvA,
                                                     const T* __restrict__ x, const int32_t* __restrict__ agg,
                                                     const T* __restrict__ ec, T* __restrict__ t4, int xcd) {
    constexpr int U = W < 16 ? 16 / W : 1;
    const int64_t tid = (xcd ? xcd_block() : (int64_t)blockIdx.x) * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < n;
    int kb = 0, ke = 0;
    if (valid) {
        if (ell) {
            kb = row * ell;
            ke = kb + ell;
        } else {
            kb = rp[row];
            ke = rp[row + 1];
        }
    }
    // own-row operands, loaded ahead of the row loop: diag(A)^{-1} on lanes
    // 0-2, the row's xx on lane 3
    T dai = 0, xo = 0, eco = 0;
    if (valid && lane < 3) dai = dinvA[3 * (int64_t)row + lane];
    if (valid && lane == 3) {
        xo = x[row];
        if (AGG) eco = ec[agg[row]];
    }
    T acc[3] = {0, 0, 0};
    // the column source (16-bit offsets from the row, or 32-bit columns) is
    // chosen once, outside the walk, so that a trip's loads issue together
    auto walk = [&](auto column) {
        for (int k0 = kb + lane; k0 < ke; k0 += U * W) {
            int kk[U];
            bool on[U];
            trip_blocks<U>(k0, ke, W, kk, on);
            int j[U];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = column(kk[u]);
            T v[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < 3; ++r) v[u][r] = V[(4 * r + 3) * nnzb + kk[u]];
            T xj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xj[u] = x[j[u]];
            if (AGG) {
                int J[U];
#pragma unroll
                for (int u = 0; u < U; ++u) J[u] = agg[j[u]];
#pragma unroll
                for (int u = 0; u < U; ++u) xj[u] += ec[J[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < 3; ++r) acc[r] += v[u][r] * (on[u] ? xj[u] : T(0));
        }
    };
    if (dcol)
        walk([&](int k) { return row + (int)dcol[k]; });
    else
        walk([&](int k) { return col[k]; });
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] += __shfl_xor(acc[r], off, W);
    if (!valid || lane > 3) return;
    T out;
    if (lane == 3) {
        out = xo;
        if (AGG) out += eco;
    } else {
        out = dai * (lane == 0 ? acc[0] : (lane == 1 ? acc[1] : acc[2]));
    }
    t4[4 * (int64_t)row + lane] = out;
}

template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_sfact_dc(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int16_t* __restrict__ dcol, int ell,
                                                     const T* __restrict__ V,
                                                     int64_t nnzb, const T* __restrict__ t4, T* __restrict__ y,
                                                     T alpha, const T* __restrict__ z, T beta,
                                                     const T* __restrict__ b, const T* __restrict__ dinv,
                                                     const T* __restrict__ coef, int step, T* __restrict__ d,
                                                     int xcd) {
    constexpr int U = W < 16 ? 16 / W : 1;
    const int64_t tid = (xcd ? xcd_block() : (int64_t)blockIdx.x) * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < n;
    // own-row epilogue operands, loaded ahead of the row loop
    const bool smooth_lane = valid && lane == 0 && coef;
    int kb = 0, ke = 0;
    if (valid) {
        if (ell) {
            kb = row * ell;
            ke = kb + ell;
        } else {
            kb = rp[row];
            ke = rp[row + 1];
        }
    }
    T zi = 0, xi = 0, bi = 0, dvi = 0, dprev = 0;
    if (valid && lane == 0 && !coef && z) zi = z[row];
    if (smooth_lane) {
        xi = t4[4 * (int64_t)row + 3];
        bi = b[row];
        dvi = dinv[row];
        if (step != 0) dprev = d[row];
    }
    T acc = 0;
    // the column source (16-bit offsets from the row, or 32-bit columns) is
    // chosen once, outside the walk, so that a trip's loads issue together
    auto walk = [&](auto column) {
        for (int k0 = kb + lane; k0 < ke; k0 += U * W) {
            int kk[U];
            bool on[U];
            trip_blocks<U>(k0, ke, W, kk, on);
            int j[U];
#pragma unroll
            for (int u = 0; u < U; ++u) j[u] = column(kk[u]);
            T vd[U], vc[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                vd[u] = V[15 * nnzb + kk[u]];
#pragma unroll
                for (int c = 0; c < 3; ++c) vc[u][c] = V[(12 + c) * nnzb + kk[u]];
            }
            Vec4<T> q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) q[u] = load4(t4 + 4 * (int64_t)j[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!on[u]) q[u] = Vec4<T>{0, 0, 0, 0};
                acc += vd[u] * q[u].d;
                acc -= vc[u][0] * q[u].a;
                acc -= vc[u][1] * q[u].b;
                acc -= vc[u][2] * q[u].c;
            }
        }
    };
    if (dcol)
        walk([&](int k) { return row + (int)dcol[k]; });
    else
        walk([&](int k) { return col[k]; });
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, W);
    if (!valid || lane != 0) return;
    if (!coef) {
        T out = alpha * acc;
        if (z) out += beta * zi;
        y[row] = out;
        return;
    }
    T c1, c2;
    cheb_coef(coef, step, c1, c2);
    T di = c2 * dvi * (bi - acc);
    if (step != 0) di += c1 * dprev;
    d[row] = di;
    y[row] = xi + di;
}

template <typename T>
void shat_factored(int n, const int32_t* rp, const int32_t* col, const int16_t* dcol, int ell, const T* V,
                   int64_t nnzb, const T* dinvA, const T* x, const int32_t* agg, const T* ec, T* t, T* y, T alpha,
                   const T* z, T beta, const T* b, const T* dinv, const T* coef, int step, T* d, int xcd, int lanes,
                   hipStream_t st) {
    if (n <= 0) return;
    if (ell && !dcol) throw std::runtime_error("shat_factored: fixed-width rows need their column offsets");
    auto run = [&](auto w) {
        constexpr int W = decltype(w)::value;
        const dim3 grid(grid_for((int64_t)n * W));
        if (agg)
            launch_span(k_sfact_bt<T, W, true>, grid, dim3(kBlock), 0, st, true, false, n, rp, col, dcol, ell, V,
                        nnzb, dinvA, x, agg, ec, t, xcd);
        else
            launch_span(k_sfact_bt<T, W, false>, grid, dim3(kBlock), 0, st, true, false, n, rp, col, dcol, ell, V,
                        nnzb, dinvA, x, agg, ec, t, xcd);
        launch_span(k_sfact_dc<T, W>, grid, dim3(kBlock), 0, st, false, true, n, rp, col, dcol, ell, V, nnzb,
                    (const T*)t, y, alpha, z, beta, b, dinv, coef, step, d, xcd);
    };
    if (lanes == 4) run(std::integral_constant<int, 4>{});
    else if (lanes == 8) run(std::integral_constant<int, 8>{});
    else run(std::integral_constant<int, 16>{});
}

// Restriction bc = P^T r of a precomputed residual; when xc != nullptr also
// the first Chebyshev step of the coarse level from a zero guess:
// xc = dc = c2c dinvc bc.
template <typename T>
__global__ void k_restrict_first(int nc, int bs, const int32_t* __restrict__ aptr,
                                 const int32_t* __restrict__ anodes, const T* __restrict__ r, T* __restrict__ bc,
                                 T* __restrict__ xc, T* __restrict__ dc, const T* __restrict__ dinvc,
                                 const T* __restrict__ coefc, const T* __restrict__ scale) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nc * bs) return;
    const int I = (int)(t / bs), c = (int)(t % bs);
    T s = 0;
    for (int q = aptr[I]; q < aptr[I + 1]; ++q) s += r[(int64_t)bs * anodes[q] + c];
    if (scale) s *= scale[0];
    bc[t] = s;
    if (xc) {
        const T di = coefc[0] * dinvc[t] * s;
        xc[t] = di;
        dc[t] = di;
    }
}

template <typename T>
void restrict_first(int nc, int bs, const int32_t* aptr, const int32_t* anodes, const T* r, T* bc, T* xc, T* dc,
                    const T* dinvc, const T* coefc, const T* scale, hipStream_t st) {
    hipLaunchKernelGGL((k_restrict_first<T>), dim3(grid_for((int64_t)nc * bs)), dim3(kBlock), 0, st, nc, bs, aptr,
                       anodes, r, bc, xc, dc, dinvc, coefc, scale);
}

// Residual fused with the restriction, for the coarser levels: one wavefront
// per aggregate I, 16 lanes per fine row of I (aggregates of two pairwise
// matchings hold at most 4 nodes; larger ones loop), so the rows are summed
// in parallel:
// bc = P^T (b - M x), then the coarse first Chebyshev step as in
// k_restrict_first.  Saves the launch of a separate residual kernel where the
// level is too small to be bandwidth-bound.
constexpr int kAggMax = 4;
constexpr int kRowLanes = 64 / kAggMax;

template <typename T, int BS>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(BlockOp<T> M, const T* __restrict__ x,
                                                           const T* __restrict__ b, int nc,
                                                           const int32_t* __restrict__ aptr,
                                                           const int32_t* __restrict__ anodes, T* __restrict__ bc,
                                                           T* __restrict__ xc, T* __restrict__ dc,
                                                           const T* __restrict__ dinvc, const T* __restrict__ coefc,
                                                           const T* __restrict__ scale) {
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int I = (int)(tid >> 6);
    const int lane = threadIdx.x & 63;
    const int sub = lane / kRowLanes, l = lane % kRowLanes;
    const bool valid = I < nc;
    const int64_t t = (int64_t)BS * I + lane;
    const T fc = (valid && lane < BS && xc) ? coefc[0] * dinvc[t] : T(0);  // loaded ahead of the loops
    const T sc = scale ? scale[0] : T(1);
    // acc = sum over the aggregate of (M x + dextra x - b): the negated residual
    T acc[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) acc[r] = 0;
    if (valid) {
        const int q1 = aptr[I + 1];
        for (int q = aptr[I] + sub; q < q1; q += kAggMax) {
            const int row = anodes[q];
            const int k1 = M.rp[row + 1];
            // U blocks per lane per trip, every load of the trip issued before
            // the first sum; a block past the row end loads the trip's first
            // again and adds nothing, so the sums are those of one block at a
            // time.  Scalar rows take four (measured 36.3 -> 32.5 us on the
            // 4e6-node contraction-expansion's level-1 S_hat); 3x3 blocks one,
            // as four would hold 116 registers (172 -> 249 us on level 1 of A)
            constexpr int U = BS == 1 ? 4 : 1;
            for (int k0 = M.rp[row] + l; k0 < k1; k0 += U * kRowLanes) {
                int kk[U];
                bool on[U];
                trip_blocks<U>(k0, k1, kRowLanes, kk, on);
                int j[U];
#pragma unroll
                for (int u = 0; u < U; ++u) j[u] = M.col[kk[u]];
                T v[U][BS * BS];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < BS; ++r)
#pragma unroll
                        for (int c = 0; c < BS; ++c) v[u][r * BS + c] = M.v[r * M.rs + c * M.cs + kk[u]];
                T xj[U][BS];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int c = 0; c < BS; ++c) xj[u][c] = x[(int64_t)BS * j[u] + c];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (on[u]) {
#pragma unroll
                        for (int r = 0; r < BS; ++r)
#pragma unroll
                            for (int c = 0; c < BS; ++c) acc[r] += v[u][r * BS + c] * xj[u][c];
                    }
            }
            if (l < BS) {
                const int64_t i = (int64_t)BS * row + l;
                T t = -b[i];
                if (M.dextra) t += M.dextra[i] * x[i];
#pragma unroll
                for (int r = 0; r < BS; ++r)
                    if (l == r) acc[r] += t;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < BS; ++r) acc[r] += __shfl_xor(acc[r], off, 64);
    if (!valid || lane >= BS) return;
    T s = -acc[0];
#pragma unroll
    for (int r = 1; r < BS; ++r)
        if (lane == r) s = -acc[r];
    s *= sc;
    bc[t] = s;
    if (xc) {
        const T di = fc * s;
        xc[t] = di;
        dc[t] = di;
    }
}

template <typename T>
void resid_restrict(int bs, const BlockOp<T>& M, const T* x, const T* b, int nc, const int32_t* aptr,
                    const int32_t* anodes, T* bc, T* xc, T* dc, const T* dinvc, const T* coefc, const T* scale,
                    hipStream_t st) {
    if (nc <= 0) return;
    if (M.ell) throw std::runtime_error("resid_restrict: walks the node-graph row layout only");
    const dim3 grid(grid_for((int64_t)nc * 64));
    if (bs == 3)
        hipLaunchKernelGGL((k_resid_restrict<T, 3>), grid, dim3(kBlock), 0, st, M, x, b, nc, aptr, anodes, bc, xc, dc,
                           dinvc, coefc, scale);
    else
        hipLaunchKernelGGL((k_resid_restrict<T, 1>), grid, dim3(kBlock), 0, st, M, x, b, nc, aptr, anodes, bc, xc, dc,
                           dinvc, coefc, scale);
}

template <typename T>
__global__ void k_restrict(int nc, int bs, const int32_t* aptr, const int32_t* anodes, const T* r, T* bc) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nc * bs) return;
    const int I = (int)(t / bs), c = (int)(t % bs);
    T s = 0;
    for (int q = aptr[I]; q < aptr[I + 1]; ++q) s += r[(int64_t)bs * anodes[q] + c];
    bc[t] = s;
}
template <typename T>
void restrict_agg(int nc, int bs, const int32_t* aptr, const int32_t* anodes, const T* r, T* bc, hipStream_t st) {
    hipLaunchKernelGGL((k_restrict<T>), dim3(grid_for((int64_t)nc * bs)), dim3(kBlock), 0, st, nc, bs, aptr, anodes,
                       r, bc);
}

// x += P ec, one thread per vector entry (node i, component c): the x loads and stores
// and the aggregate-map loads of a wavefront are contiguous
template <typename T, int BS>
__global__ __launch_bounds__(kBlock) void k_prolong(int64_t nv, const int32_t* __restrict__ agg,
                                                    const T* __restrict__ ec, T* __restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nv) return;
    const int64_t i = t / BS;
    const int c = (int)(t - i * BS);
    x[t] += ec[(int64_t)BS * agg[i] + c];
}
template <typename T>
void prolong_add(int n, int bs, const int32_t* agg, const T* ec, T* x, hipStream_t st) {
    const int64_t nv = (int64_t)n * bs;
    if (bs == 3)
        hipLaunchKernelGGL((k_prolong<T, 3>), dim3(grid_for(nv)), dim3(kBlock), 0, st, nv, agg, ec, x);
    else
        hipLaunchKernelGGL((k_prolong<T, 1>), dim3(grid_for(nv)), dim3(kBlock), 0, st, nv, agg, ec, x);
}

// x = Minv b (FP64 arithmetic), one wavefront per row
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const double* Minv, const T* b, T* x) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (row >= n) return;
    double s = 0.0;
    for (int c = l; c < n; c += 64) s += Minv[(int64_t)row * n + c] * (double)b[c];
    s = wave_sum(s);
    if (l == 0) x[row] = (T)s;
}
template <typename T>
void dense_gemv(int n, const double* Minv, const T* b, T* x, hipStream_t st) {
    hipLaunchKernelGGL((k_dense_gemv<T>), dim3((n + 3) / 4), dim3(kBlock), 0, st, n, Minv, b, x);
}

// ---------------------------------------------------------------------------
// Set-up numerics (FP64)
// ---------------------------------------------------------------------------

// Coarse value q of every plane (r < np_r, c < np_c) = sum of the listed fine
// values; on the coarse diagonal also the fine extra diagonal of the aggregate.
__global__ void k_galerkin(int64_t nq, int np_r, int np_c, const int32_t* gptr, const int32_t* gidx,
                           const double* vf, int64_t frs, int64_t fcs, double* vc, int64_t crs, int64_t ccs,
                           const int32_t* qrow, const int32_t* ccol, const double* dextra, const int32_t* aptr,
                           const int32_t* anodes) {
    // one thread per (plane, coarse value): the planes of a value are
    // independent sums, so they run side by side (the coarsest levels have few
    // values, each gathered from many fine ones)
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nq * np_r * np_c) return;
    const int plane = (int)(t / nq);
    const int64_t q = t % nq;
    const int r = plane / np_c, c = plane % np_c;
    const int t0 = gptr[q], t1 = gptr[q + 1];
    double s = 0.0;
    const double* p = vf + r * frs + c * fcs;
    for (int k = t0; k < t1; ++k) s += p[gidx[k]];
    if (dextra && r == c && qrow[q] == ccol[q]) {
        const int I = qrow[q];
        for (int a = aptr[I]; a < aptr[I + 1]; ++a) s += dextra[(int64_t)np_r * anodes[a] + r];
    }
    vc[r * crs + c * ccs + q] = s;
}
void galerkin(int64_t nq, int np_r, int np_c, const int32_t* gptr, const int32_t* gidx, const double* vf,
              int64_t frs, int64_t fcs, double* vc, int64_t crs, int64_t ccs, const int32_t* qrow,
              const int32_t* ccol, const double* dextra, const int32_t* aptr, const int32_t* anodes,
              hipStream_t st) {
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_galerkin, dim3(grid_for(nq * np_r * np_c)), dim3(kBlock), 0, st, nq, np_r, np_c, gptr,
                       gidx, vf, frs, fcs, vc, crs, ccs, qrow, ccol, dextra, aptr, anodes);
}

__global__ void k_block_dinv(int n, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs,
                             int64_t cs, const double* dextra, double* dinv, double* diag) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * bs) return;
    const int i = (int)(t / bs), r = (int)(t % bs);
    const int k = lower_bound_dev(col, rp[i], rp[i + 1], i);
    double d = v[r * rs + r * cs + k];
    if (dextra) d += dextra[t];
    if (diag) diag[t] = d;
    dinv[t] = 1.0 / d;
}
void block_dinv(int n, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs, int64_t cs,
                const double* dextra, double* dinv, double* diag, hipStream_t st) {
    hipLaunchKernelGGL(k_block_dinv, dim3(grid_for((int64_t)n * bs)), dim3(kBlock), 0, st, n, bs, rp, col, v, rs,
                       cs, dextra, dinv, diag);
}

// S_hat_ij = D_ij - sum_{k in N(i)} sum_c C_{i,k,c} B_{k,j,c} / diag(A)_{3k+c}
//
// 16 lanes per row i.  The row's S_hat columns and accumulators sit in LDS;
// lane t first loads neighbour k_t = col[r0 + t] (its row range, C_{i,k,:} and
// diag(A)^{-1}_k) and seeds the entry j = k_t with D_ij.  Then, for the
// neighbours in column order, the lanes take the blocks (k, j) of row k, find
// j among the row's S_hat columns (binary search in LDS) and subtract the
// three products.  The lanes of one step hold distinct j and the steps follow
// the row's column order, so every entry sees the same operations in the
// same order as a loop over k per entry; each step costs one round of
// coalesced loads of row k instead of a binary search in global memory per
// entry and neighbour.  Rows with more than kShatLds S_hat entries or more
// than kShatW neighbours take that per-entry loop.
constexpr int kShatW = 16;
constexpr int kShatLds = 128;
constexpr int kShatRows = kBlock / kShatW;

__device__ inline int lds_lower_bound(const int32_t* a, int n, int key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_shat(int n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const double* __restrict__ V,
                                                 int64_t nnzb, const double* __restrict__ dinvA,
                                                 const int32_t* __restrict__ srp, const int32_t* __restrict__ scol,
                                                 double* __restrict__ shat) {
    __shared__ int32_t lcol[kShatRows][kShatLds];
    __shared__ double lacc[kShatRows][kShatLds];
    const int g = threadIdx.x / kShatW, lane = threadIdx.x % kShatW;
    const int row = blockIdx.x * kShatRows + g;
    // whole 16-lane groups leave together; no barrier spans groups
    if (row >= n) return;
    const int r0 = rp[row], r1 = rp[row + 1], nq = r1 - r0;
    const int s0 = srp[row], ns = srp[row + 1] - s0;
    if (ns > kShatLds || nq > kShatW) {
        for (int e = s0 + lane; e < s0 + ns; e += kShatW) {
            const int j = scol[e];
            double s = 0.0;
            const int pd = lower_bound_dev(col, r0, r1, j);
            if (pd < r1 && col[pd] == j) s = V[15 * nnzb + pd];
            for (int q = r0; q < r1; ++q) {
                const int k = col[q];
                const int k0 = rp[k], k1 = rp[k + 1];
                const int p2 = lower_bound_dev(col, k0, k1, j);
                if (p2 < k1 && col[p2] == j) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        s -= V[(12 + c) * nnzb + q] * V[(4 * c + 3) * nnzb + p2] * dinvA[3 * (int64_t)k + c];
                }
            }
            shat[e] = s;
        }
        return;
    }
    int32_t* lc = lcol[g];
    double* la = lacc[g];
    for (int e = lane; e < ns; e += kShatW) {
        lc[e] = scol[s0 + e];
        la[e] = 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    int k0 = 0, k1 = 0;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    if (lane < nq) {
        const int q = r0 + lane;
        const int k = col[q];
        k0 = rp[k];
        k1 = rp[k + 1];
        c0 = V[12 * nnzb + q];
        c1 = V[13 * nnzb + q];
        c2 = V[14 * nnzb + q];
        d0 = dinvA[3 * (int64_t)k];
        d1 = dinvA[3 * (int64_t)k + 1];
        d2 = dinvA[3 * (int64_t)k + 2];
        const double dij = V[15 * nnzb + q];
        const int e = lds_lower_bound(lc, ns, k);
        if (e < ns && lc[e] == k) la[e] = dij;
    }
    __builtin_amdgcn_wave_barrier();
    for (int t = 0; t < nq; ++t) {
        const int kb = __shfl(k0, t, kShatW), ke = __shfl(k1, t, kShatW);
        const double C0 = __shfl(c0, t, kShatW), C1 = __shfl(c1, t, kShatW), C2 = __shfl(c2, t, kShatW);
        const double D0 = __shfl(d0, t, kShatW), D1 = __shfl(d1, t, kShatW), D2 = __shfl(d2, t, kShatW);
        for (int p2 = kb + lane; p2 < ke; p2 += kShatW) {
            const int j = col[p2];
            const double b0 = V[3 * nnzb + p2], b1 = V[7 * nnzb + p2], b2 = V[11 * nnzb + p2];
            const int e = lds_lower_bound(lc, ns, j);
            if (e < ns && lc[e] == j) {
                double s = la[e];
                s -= C0 * b0 * D0;
                s -= C1 * b1 * D1;
                s -= C2 * b2 * D2;
                la[e] = s;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    for (int e = lane; e < ns; e += kShatW) shat[s0 + e] = la[e];
}
void shat_numeric(int n, const int32_t* rp, const int32_t* col, const double* V, int64_t nnzb, const double* dinvA,
                  const int32_t* srp, const int32_t* scol, double* shat, hipStream_t st) {
    hipLaunchKernelGGL(k_shat, dim3((n + kShatRows - 1) / kShatRows), dim3(kBlock), 0, st, n, rp, col, V, nnzb,
                       dinvA, srp, scol, shat);
}

// Dense copy of a block-sparse matrix into the left half of work [n][2n]
// (right half: identity) for the Gauss-Jordan inverse.
__global__ void k_dense_from_csr(int nb, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs,
                                 int64_t cs, const double* dextra, double* work) {
    const int n = nb * bs;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * 2 * n) return;
    const int r = (int)(t / (2 * n)), c = (int)(t % (2 * n));
    double val = 0.0;
    if (c >= n) {
        val = (c - n == r) ? 1.0 : 0.0;
    } else {
        const int I = r / bs, rr = r % bs, J = c / bs, cc = c % bs;
        const int k = lower_bound_dev(col, rp[I], rp[I + 1], J);
        if (k < rp[I + 1] && col[k] == J) val = v[rr * rs + cc * cs + k];
        if (dextra && r == c) val += dextra[r];
    }
    work[t] = val;
}
void dense_from_csr(int nb, int bs, const int32_t* rp, const int32_t* col, const double* v, int64_t rs, int64_t cs,
                    const double* dextra, double* work, hipStream_t st) {
    const int64_t n = (int64_t)nb * bs;
    hipLaunchKernelGGL(k_dense_from_csr, dim3(grid_for(n * 2 * n)), dim3(kBlock), 0, st, nb, bs, rp, col, v, rs, cs,
                       dextra, work);
}

// Gauss-Jordan with partial pivoting on [M | I] (n x 2n), one launch per
// pivot step spread over many workgroups (one wavefront per row): each step
// reads the rows from one half of the work buffer and writes them to the
// other, so no workgroup overwrites a row that another still reads.  Two
// independent matrices share every launch (the coarsest levels of both
// hierarchies).  work: [2][n][2n], the input in the first half.
constexpr int kGjRows = kBlock / 64;

struct GjStep {
    int n[2];
    const double* src[2];
    double* dst[2];
    int blocks0;   // workgroups of matrix 0; the rest belong to matrix 1
};

__global__ __launch_bounds__(kBlock) void k_gj_step(GjStep a, int k) {
    const int m = (int)blockIdx.x < a.blocks0 ? 0 : 1;
    const int n = a.n[m];
    const int b = m == 0 ? (int)blockIdx.x : (int)blockIdx.x - a.blocks0;
    const double* src = a.src[m];
    double* dst = a.dst[m];
    const int64_t n2 = 2 * (int64_t)n;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = b * kGjRows + w;
    if (k >= n) {  // this matrix is finished: carry its rows over
        if (r < n)
            for (int64_t c = l; c < n2; c += 64) dst[r * n2 + c] = src[r * n2 + c];
        return;
    }
    // pivot: the largest |M_rk| over r >= k, the smallest row on ties
    __shared__ double sval[kBlock];
    __shared__ int sidx[kBlock];
    double best = -1.0;
    int bi = k;
    for (int q = k + (int)threadIdx.x; q < n; q += kBlock) {
        const double v = fabs(src[q * n2 + k]);
        if (v > best) {
            best = v;
            bi = q;
        }
    }
    sval[threadIdx.x] = best;
    sidx[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = sval[threadIdx.x + s];
            const int oi = sidx[threadIdx.x + s];
            if (o > sval[threadIdx.x] || (o == sval[threadIdx.x] && oi < sidx[threadIdx.x])) {
                sval[threadIdx.x] = o;
                sidx[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = sidx[0];
    if (r >= n) return;
    const double inv_p = 1.0 / src[p * n2 + k];
    const double* prow = src + p * n2;
    double* drow = dst + r * n2;
    if (r == k) {
        for (int64_t c = l; c < n2; c += 64) drow[c] = prow[c] * inv_p;
    } else {
        // after exchanging rows k and p, row r holds the old row sr
        const double* srow = src + (r == p ? k : r) * n2;
        const double f = srow[k];
        for (int64_t c = l; c < n2; c += 64) drow[c] = srow[c] - f * (prow[c] * inv_p);
    }
}

__global__ void k_gj_extract(int n0, const double* w0, double* inv0, int n1, const double* w1, double* inv1) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s0 = (int64_t)n0 * n0;
    if (t < s0) {
        inv0[t] = w0[(t / n0) * 2 * n0 + n0 + t % n0];
    } else if (t < s0 + (int64_t)n1 * n1) {
        const int64_t u = t - s0;
        inv1[u] = w1[(u / n1) * 2 * n1 + n1 + u % n1];
    }
}

// Blocked form: one launch per panel of kGjPanel pivot steps.  Each workgroup
// owns kGjSlab columns of [M | I] (all rows) and keeps, redundantly, a copy of
// the panel's columns: it repeats the panel's pivot choices and multipliers on
// that copy (the same arithmetic in every workgroup) and applies them to its
// columns in LDS.  Element by element the operations are those of k_gj_step,
// so the result is the same.  LDS: n (kGjPanel + kGjSlab + 1) doubles.
constexpr int kGjPanel = 8, kGjSlab = 8;
constexpr int kGjPanelMaxN = 448;

struct GjPanel {
    int n[2];
    const double* src[2];
    double* dst[2];
    int blocks0;   // workgroups of matrix 0; the rest belong to matrix 1
};

__global__ __launch_bounds__(kBlock) void k_gj_panel(GjPanel a, int k0) {
    extern __shared__ double lds[];
    __shared__ double sval[kBlock / 64];
    __shared__ int sidx[kBlock / 64];
    __shared__ double prow[kGjPanel + kGjSlab];  // scaled pivot row (old row p)
    __shared__ double rowk[kGjPanel + kGjSlab];  // old row k
    const int m = (int)blockIdx.x < a.blocks0 ? 0 : 1;
    const int n = a.n[m];
    const int b = m == 0 ? (int)blockIdx.x : (int)blockIdx.x - a.blocks0;
    const double* src = a.src[m];
    double* dst = a.dst[m];
    const int64_t n2 = 2 * (int64_t)n;
    const int c0 = b * kGjSlab;
    const int nc = (int)min((int64_t)kGjSlab, n2 - c0);
    const int P = min(kGjPanel, n - k0);   // pivot steps of this matrix in the panel (<= 0: carry over)
    double* pan = lds;                     // [n][kGjPanel]
    double* sl = pan + n * kGjPanel;       // [n][kGjSlab]
    double* f = sl + n * kGjSlab;          // [n] multipliers
    const int tid = threadIdx.x;
    for (int e = tid; e < n * kGjSlab; e += kBlock) {
        const int r = e / kGjSlab, c = e % kGjSlab;
        sl[e] = c < nc ? src[r * n2 + c0 + c] : 0.0;
    }
    for (int e = tid; e < n * kGjPanel; e += kBlock) {
        const int r = e / kGjPanel, t = e % kGjPanel;
        pan[e] = t < P ? src[r * n2 + k0 + t] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < P; ++t) {
        const int k = k0 + t;
        double best = -1.0;
        int bi = k;
        for (int q = k + tid; q < n; q += kBlock) {
            const double v = fabs(pan[q * kGjPanel + t]);
            if (v > best) {
                best = v;
                bi = q;
            }
        }
        // pivot: the largest |value|, the smallest row among equal ones (a total
        // order, so the wavefront butterflies and the 4-way merge find the
        // same row as any reduction order)
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (o > best || (o == best && oi < bi)) {
                best = o;
                bi = oi;
            }
        }
        if ((tid & 63) == 0) {
            sval[tid >> 6] = best;
            sidx[tid >> 6] = bi;
        }
        __syncthreads();
        double pb = sval[0];
        int p = sidx[0];
        for (int w = 1; w < kBlock / 64; ++w)
            if (sval[w] > pb || (sval[w] == pb && sidx[w] < p)) {
                pb = sval[w];
                p = sidx[w];
            }
        const double inv_p = 1.0 / pan[p * kGjPanel + t];
        if (tid < kGjPanel) {
            prow[tid] = pan[p * kGjPanel + tid] * inv_p;
            rowk[tid] = pan[k * kGjPanel + tid];
        } else if (tid < kGjPanel + kGjSlab) {
            prow[tid] = sl[p * kGjSlab + tid - kGjPanel] * inv_p;
            rowk[tid] = sl[k * kGjSlab + tid - kGjPanel];
        }
        // after exchanging rows k and p, row r holds the old row (r == p ? k : r)
        for (int r = tid; r < n; r += kBlock) f[r] = pan[(r == p ? k : r) * kGjPanel + t];
        __syncthreads();
        for (int e = tid; e < n * kGjPanel; e += kBlock) {
            const int r = e / kGjPanel, c = e % kGjPanel;
            if (r == k) pan[e] = prow[c];
            else pan[e] = (r == p ? rowk[c] : pan[e]) - f[r] * prow[c];
        }
        for (int e = tid; e < n * kGjSlab; e += kBlock) {
            const int r = e / kGjSlab, c = e % kGjSlab;
            if (r == k) sl[e] = prow[kGjPanel + c];
            else sl[e] = (r == p ? rowk[kGjPanel + c] : sl[e]) - f[r] * prow[kGjPanel + c];
        }
        __syncthreads();
    }
    for (int e = tid; e < n * kGjSlab; e += kBlock) {
        const int r = e / kGjSlab, c = e % kGjSlab;
        if (c < nc) dst[r * n2 + c0 + c] = sl[e];
    }
}

void gauss_jordan_inverse2(int n0, double* work0, double* inv0, int n1, double* work1, double* inv1,
                           hipStream_t st) {
    const int steps = std::max(n0, n1);
    if (std::max(n0, n1) <= kGjPanelMaxN) {
        const int panels = (std::max(n0, n1) + kGjPanel - 1) / kGjPanel;
        GjPanel a;
        a.n[0] = n0;
        a.n[1] = n1;
        a.blocks0 = (int)((2 * (int64_t)n0 + kGjSlab - 1) / kGjSlab);
        const int blocks = a.blocks0 + (int)((2 * (int64_t)n1 + kGjSlab - 1) / kGjSlab);
        const size_t lds = (size_t)std::max(n0, n1) * (kGjPanel + kGjSlab + 1) * sizeof(double);
        double* half0[2] = {work0, work0 + 2 * (int64_t)n0 * n0};
        double* half1[2] = {work1, work1 + 2 * (int64_t)n1 * n1};
        for (int i = 0; i < panels; ++i) {
            a.src[0] = half0[i & 1];
            a.dst[0] = half0[(i + 1) & 1];
            a.src[1] = half1[i & 1];
            a.dst[1] = half1[(i + 1) & 1];
            hipLaunchKernelGGL(k_gj_panel, dim3(blocks), dim3(kBlock), lds, st, a, i * kGjPanel);
        }
        const int64_t tot = (int64_t)n0 * n0 + (int64_t)n1 * n1;
        hipLaunchKernelGGL(k_gj_extract, dim3(grid_for(tot)), dim3(kBlock), 0, st, n0, half0[panels & 1], inv0, n1,
                           half1[panels & 1], inv1);
        return;
    }
    GjStep a;
    a.n[0] = n0;
    a.n[1] = n1;
    a.blocks0 = (n0 + kGjRows - 1) / kGjRows;
    const int blocks = a.blocks0 + (n1 + kGjRows - 1) / kGjRows;
    double* half0[2] = {work0, work0 + 2 * (int64_t)n0 * n0};
    double* half1[2] = {work1, work1 + 2 * (int64_t)n1 * n1};
    for (int k = 0; k < steps; ++k) {
        a.src[0] = half0[k & 1];
        a.dst[0] = half0[(k + 1) & 1];
        a.src[1] = half1[k & 1];
        a.dst[1] = half1[(k + 1) & 1];
        hipLaunchKernelGGL(k_gj_step, dim3(blocks), dim3(kBlock), 0, st, a, k);
    }
    const int64_t tot = (int64_t)n0 * n0 + (int64_t)n1 * n1;
    hipLaunchKernelGGL(k_gj_extract, dim3(grid_for(tot)), dim3(kBlock), 0, st, n0, half0[steps & 1], inv0, n1,
                       half1[steps & 1], inv1);
}

__global__ void k_power_start(int64_t n, double* x) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t h = ((uint64_t)i * 2654435761ull) & 0xffffffffull;
    x[i] = 0.5 + (double)h / 4294967296.0;
}
void power_start(int64_t n, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_power_start, dim3(grid_for(n)), dim3(kBlock), 0, st, n, x);
}

// Gershgorin bound of D^{-1} M: max over point rows of |dinv_r| sum_c |M_rc|
// (the extra diagonal added to the diagonal entry).  W lanes per block row as
// in the SpMV; per-block maxima into part[blockIdx.x], then a one-block
// maximum into out[0].
template <int BS, int W>
__global__ __launch_bounds__(kBlock) void k_gersh_part(BlockOp<double> M, const double* __restrict__ dinv,
                                                       double* __restrict__ part) {
    __shared__ double lds[kBlock / 64];
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int row = (int)(tid / W);
    const int lane = threadIdx.x % W;
    const bool valid = row < M.n;
    double acc[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) acc[r] = 0.0;
    if (valid) {
        const int k1 = M.rp[row + 1];
        for (int k = M.rp[row] + lane; k < k1; k += W) {
            const bool diag = M.col[k] == row;
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
                for (int c = 0; c < BS; ++c) {
                    double v = M.v[r * M.rs + c * M.cs + k];
                    if (diag && c == r && M.dextra) v += M.dextra[(int64_t)BS * row + r];
                    acc[r] += fabs(v);
                }
        }
    }
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < BS; ++r) acc[r] += __shfl_xor(acc[r], off, W);
    double mx = 0.0;
    if (valid && lane == 0)
#pragma unroll
        for (int r = 0; r < BS; ++r) mx = fmax(mx, acc[r] * fabs(dinv[(int64_t)BS * row + r]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, lds[w]);
        part[blockIdx.x] = m;
    }
}
__global__ void k_max_fin(const double* part, int G, double* out) {
    __shared__ double lds[kBlock / 64];
    double mx = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) mx = fmax(mx, part[b]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, lds[w]);
        out[0] = m;
    }
}
template <int BS, int W>
int gersh_launch(const BlockOp<double>& M, const double* dinv, double* part, hipStream_t st) {
    const int G = (int)grid_for((int64_t)M.n * W);
    hipLaunchKernelGGL((k_gersh_part<BS, W>), dim3(G), dim3(kBlock), 0, st, M, dinv, part);
    return G;
}
template <int BS>
int gersh_w(const BlockOp<double>& M, const double* dinv, double* part, hipStream_t st) {
    switch (M.lanes) {
        case 64: return gersh_launch<BS, 64>(M, dinv, part, st);
        case 32: return gersh_launch<BS, 32>(M, dinv, part, st);
        default: return gersh_launch<BS, 16>(M, dinv, part, st);
    }
}
// part: one partial per launched block (at most n*64/kBlock + 1 entries)
void gershgorin_bound(const BlockOp<double>& M, int bs, const double* dinv, double* part, double* out,
                      hipStream_t st) {
    if (M.n <= 0) return;
    const int G = bs == 3 ? gersh_w<3>(M, dinv, part, st) : gersh_w<1>(M, dinv, part, st);
    hipLaunchKernelGGL(k_max_fin, dim3(1), dim3(kBlock), 0, st, part, G, out);
}

// dK_{3 node + c} = sum_k c_k (a^k_{node,c})^2 over outlet slots (outlets are disjoint)
__global__ void k_rank_one_diag(int n_slots, const int32_t* onode, const int32_t* oid, const double* amsk,
                                const double* ck, double* dK) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n_slots * 3) return;
    const int sl = (int)(t / 3), c = (int)(t % 3);
    const double a = amsk[t];
    dK[3 * (int64_t)onode[sl] + c] = ck[oid[sl]] * a * a;
}
void rank_one_diag(int n_slots, const int32_t* onode, const int32_t* oid, const double* amsk, const double* ck,
                   double* dK, hipStream_t st) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_rank_one_diag, dim3(grid_for((int64_t)n_slots * 3)), dim3(kBlock), 0, st, n_slots, onode,
                       oid, amsk, ck, dK);
}

// Transposed system: plane (r,c) of block (i,j) = plane (c,r) of block (j,i)
__global__ void k_transpose_values(int64_t nnzb, const int32_t* tmap, const double* V, double* Vt) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnzb) return;
    const int64_t kt = tmap[k];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) Vt[(4 * r + c) * nnzb + k] = V[(4 * c + r) * nnzb + kt];
}
void transpose_values(int64_t nnzb, const int32_t* tmap, const double* V, double* Vt, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_values, dim3(grid_for(nnzb)), dim3(kBlock), 0, st, nnzb, tmap, V, Vt);
}

__global__ void k_export_aos(int64_t nnzb, const double* V, double* dst) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnzb) return;
#pragma unroll
    for (int p = 0; p < 16; ++p) dst[16 * k + p] = V[p * nnzb + k];
}
void export_aos(int64_t nnzb, const double* V, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_export_aos, dim3(grid_for(nnzb)), dim3(kBlock), 0, st, nnzb, V, dst);
}

__global__ void k_newton_update(int64_t n, double gdt, const double* dx, double* y, double* ydot) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double d = dx[i];
        y[i] += gdt * d;
        ydot[i] += d;
    }
}
void newton_update(int64_t n, double gdt, const double* dx, double* y, double* ydot, hipStream_t st) {
    hipLaunchKernelGGL(k_newton_update, dim3(std::min<int64_t>(grid_for(n), 65535)), dim3(kBlock), 0, st, n, gdt, dx,
                       y, ydot);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
#define NS_INST(T)                                                                                                   \
    template void spmv<T>(int, int, const BlockOp<T>&, const T*, T*, T, const T*, T, const T*, const RankOne<T>*,   \
                          hipStream_t, const FirstStep<T>*);                                                         \
    template void spmv_full<T>(int, const int32_t*, const int32_t*, const T*, int64_t, const T*, T*, T, const T*, T, \
                               const RankOne<T>*, hipStream_t, int, const int16_t*);                                 \
    template void outlet_dot<T>(int, const int32_t*, const int32_t*, const T*, const T*, const T*, T*, hipStream_t);  \
    template void axpby<T>(int64_t, T, const T*, T, const T*, T*, hipStream_t);                                      \
    template void fill<T>(int64_t, T, T*, hipStream_t);                                                              \
    template void mul<T>(int64_t, const T*, const T*, T*, hipStream_t);                                              \
    template void arnoldi_cgs2<T>(int64_t, int, const T*, int64_t, T*, double*, double*, const GivensArgs&, double*,  \
                                  hipStream_t);                                                                      \
    template void norm2<T>(int64_t, const T*, double*, double*, hipStream_t, double*);                               \
    template void scale_by<T>(int64_t, const T*, const double*, bool, T*, hipStream_t);                             \
    template void start_cycle<T>(int64_t, T*, const double*, double*, int, hipStream_t);                             \
    template void cheb_first<T>(int64_t, const T*, const T*, const T*, T*, T*, hipStream_t);                         \
    template void cheb_step<T>(int, const BlockOp<T>&, const T*, T*, T*, const T*, const T*, const T*, int,           \
                               const int32_t*, const T*, hipStream_t);                                               \
    template void restrict_first<T>(int, int, const int32_t*, const int32_t*, const T*, T*, T*, T*, const T*,         \
                                    const T*, const T*, hipStream_t);                                                 \
    template void restrict_agg<T>(int, int, const int32_t*, const int32_t*, const T*, T*, hipStream_t);              \
    template void shat_factored<T>(int, const int32_t*, const int32_t*, const int16_t*, int, const T*, int64_t,      \
                                   const T*, const T*, const int32_t*, const T*, T*, T*, T, const T*, T, const T*,   \
                                   const T*, const T*, int, T*, int, int, hipStream_t);                              \
    template void resid_restrict<T>(int, const BlockOp<T>&, const T*, const T*, int, const int32_t*, const int32_t*, \
                                    T*, T*, T*, const T*, const T*, const T*, hipStream_t);                          \
    template void prolong_add<T>(int, int, const int32_t*, const T*, T*, hipStream_t);                               \
    template void dense_gemv<T>(int, const double*, const T*, T*, hipStream_t);

NS_INST(double)
NS_INST(float)
template void convert<double, float>(int64_t, const double*, float*, hipStream_t);
template void convert<float, double>(int64_t, const float*, double*, hipStream_t);
template void convert<double, double>(int64_t, const double*, double*, hipStream_t);
template void convert<float, float>(int64_t, const float*, float*, hipStream_t);
template void combine<double, double>(int64_t, int, const double*, int64_t, const double*, double*, bool,
                                      hipStream_t);
template void combine<float, float>(int64_t, int, const float*, int64_t, const double*, float*, bool, hipStream_t);
template void combine<float, double>(int64_t, int, const float*, int64_t, const double*, double*, bool,
                                     hipStream_t);

}  // namespace ns
