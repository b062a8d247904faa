// Exclusive prefix sums for the CSR offsets of crossing records, child slots of
// split nodes and leaf / internal-node numbering.  Three passes: per-block
// totals, a single-block scan of the totals, per-block scan plus carry-in.
#include "common.h"

namespace hg {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ inline int64_t load_val(const T *in, int64_t i, int64_t n)
{
    return i < n ? int64_t(in[i]) : 0;
}

// Inclusive scan across one 64-lane wavefront.
__device__ inline int64_t wave_incl_scan(int64_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan across the block; returns the block total in *total.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t wave_tot[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; w++) {
        int64_t t = wave_tot[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const T *in, int64_t n, int64_t *tile_sum)
{
    const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) s += load_val(in, base + j, n);
    int64_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One block scans the per-tile totals in place (exclusive) and stores the
// grand total at tile_sum[n_tiles].
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tile_sums(int64_t *tile_sum, int64_t n_tiles)
{
    int64_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += SCAN_THREADS) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < n_tiles ? tile_sum[i] : 0;
        int64_t total;
        int64_t ex = block_excl_scan(v, &total);
        if (i < n_tiles) tile_sum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tile_sum[n_tiles] = carry;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_tile_scan(const T *in, int64_t n, const int64_t *tile_sum, int64_t n_tiles, int64_t *out)
{
    const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        v[j] = load_val(in, base + j, n);
        s += v[j];
    }
    int64_t total;
    int64_t run = tile_sum[blockIdx.x] + block_excl_scan(s, &total);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tile_sum[n_tiles];
}

// Inputs of at most one tile: one block does everything.
template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_one_tile(const T *in, int64_t n, int64_t *out)
{
    const int64_t base = int64_t(threadIdx.x) * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        v[j] = load_val(in, base + j, n);
        s += v[j];
    }
    int64_t total;
    int64_t run = block_excl_scan(s, &total);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) out[n] = total;
}

template <typename T>
int scan_impl(const T *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s)
{
    if (n < 0) return HG_E_INVAL;
    if (n <= SCAN_TILE) {
        k_scan_one_tile<T><<<1, SCAN_THREADS, 0, s>>>(in, n, out);
        HG_CHECK(hipGetLastError());
        return HG_OK;
    }
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles > 0x7fffffff) return HG_E_LIMIT;
    k_tile_sums<T><<<dim3(unsigned(tiles)), dim3(SCAN_THREADS), 0, s>>>(in, n, tmp);
    HG_CHECK(hipGetLastError());
    k_scan_tile_sums<<<1, SCAN_THREADS, 0, s>>>(tmp, tiles);
    HG_CHECK(hipGetLastError());
    k_tile_scan<T><<<dim3(unsigned(tiles)), dim3(SCAN_THREADS), 0, s>>>(in, n, tmp, tiles, out);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

}  // namespace

size_t scan_tmp_elems(int64_t n)
{
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return size_t(tiles < 1 ? 1 : tiles) + 1;
}

int scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s)
{
    return scan_impl<int32_t>(in, out, n, tmp, s);
}

int scan_u8_to_i64(const uint8_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s)
{
    return scan_impl<uint8_t>(in, out, n, tmp, s);
}

}  // namespace hg
