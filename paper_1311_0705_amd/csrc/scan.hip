// Exclusive prefix sums for the CSR offsets of crossing records, child slots of
// split nodes and leaf / internal-node numbering.  Per-block totals, a scan of
// the totals, per-block scans plus carry-in (the device-count scan folds the
// middle step into the last).
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

// ---- element count on the device ---------------------------------------------
// A fixed grid of DSCAN_BLOCKS blocks; block b scans the contiguous range
// [b*per, (b+1)*per) with per = ceil(n / DSCAN_BLOCKS) rounded up to a tile.
constexpr int DSCAN_BLOCKS = 256;

__device__ inline int64_t dscan_per(int64_t n)
{
    const int64_t per = (n + DSCAN_BLOCKS - 1) / DSCAN_BLOCKS;
    return (per + SCAN_TILE - 1) / SCAN_TILE * SCAN_TILE;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_dscan_sums(const T *in, const int64_t *n_dev, int64_t *bsum)
{
    const int64_t n = *n_dev;
    const int64_t per = dscan_per(n);
    const int64_t b0 = int64_t(blockIdx.x) * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    int64_t s = 0;
    for (int64_t base = b0 + int64_t(threadIdx.x) * SCAN_ITEMS; base < b1; base += SCAN_TILE) {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) s += load_val(in, base + j, b1);
    }
    int64_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Each block scans the DSCAN_BLOCKS block totals itself for its carry-in (no
// separate pass over them); block 0 stores the grand total at out[n].
template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_dscan_apply(const T *in, const int64_t *n_dev, const int64_t *bsum, int64_t *out)
{
    static_assert(DSCAN_BLOCKS == SCAN_THREADS, "one block total per thread");
    __shared__ int64_t s_carry;
    const int64_t n = *n_dev;
    const int64_t per = dscan_per(n);
    const int64_t b0 = int64_t(blockIdx.x) * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    int64_t grand;
    const int64_t ex = block_excl_scan(bsum[threadIdx.x], &grand);
    if (int(threadIdx.x) == int(blockIdx.x)) s_carry = ex;
    __syncthreads();
    int64_t carry = s_carry;
    for (int64_t tile = b0; tile < b1; tile += SCAN_TILE) {
        const int64_t base = tile + int64_t(threadIdx.x) * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS];
        int64_t s = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) {
            v[j] = load_val(in, base + j, b1);
            s += v[j];
        }
        int64_t total;
        int64_t run = carry + block_excl_scan(s, &total);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) {
            if (base + j < b1) out[base + j] = run;
            run += v[j];
        }
        carry += total;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = grand;
}

// ---- per-chunk segmented scan of the batched walk's counts --------------------
__global__ void __launch_bounds__(SCAN_THREADS)
    k_chunk_sums(const BatchChunk *__restrict__ chunks, const WalkArgs *__restrict__ args,
                 int64_t *csum)
{
    const BatchChunk c = chunks[blockIdx.x];
    const int32_t *cnt = args[c.grid].count;
    int64_t s = 0;
    for (int64_t base = c.start + int64_t(threadIdx.x) * SCAN_ITEMS; base < c.end; base += SCAN_TILE) {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) s += load_val(cnt, base + j, c.end);
    }
    int64_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

// cex = exclusive scan of the chunk sums over the whole table; a chunk's base
// within its grid is cex[c] - cex[head].
__global__ void __launch_bounds__(SCAN_THREADS)
    k_chunk_apply(const BatchChunk *__restrict__ chunks, const WalkArgs *__restrict__ args,
                  const int64_t *cex)
{
    const BatchChunk c = chunks[blockIdx.x];
    const WalkArgs &A = args[c.grid];
    const int32_t *cnt = A.count;
    int64_t *out = const_cast<int64_t *>(A.offsets);
    int64_t carry = cex[blockIdx.x] - cex[c.head];
    for (int64_t tile = c.start; tile < c.end; tile += SCAN_TILE) {
        const int64_t base = tile + int64_t(threadIdx.x) * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS];
        int64_t s = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) {
            v[j] = load_val(cnt, base + j, c.end);
            s += v[j];
        }
        int64_t total;
        int64_t run = carry + block_excl_scan(s, &total);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; j++) {
            if (base + j < c.end) out[base + j] = run;
            run += v[j];
        }
        carry += total;
    }
    if (c.end == A.n && threadIdx.x == 0) out[A.n] = carry;
}

__global__ void k_chunk_empty(const WalkArgs *__restrict__ args, int ng)
{
    const int g = int(blockIdx.x) * SCAN_THREADS + threadIdx.x;
    if (g < ng && args[g].n == 0) const_cast<int64_t *>(args[g].offsets)[0] = 0;
}

}  // namespace

size_t scan_dev_tmp_elems() { return size_t(DSCAN_BLOCKS) + 1; }

int scan_u8_to_i64_dev(const uint8_t *in, int64_t *out, const int64_t *n_dev, int64_t *tmp,
                       hipStream_t s)
{
    k_dscan_sums<uint8_t><<<DSCAN_BLOCKS, SCAN_THREADS, 0, s>>>(in, n_dev, tmp);
    HG_CHECK(hipGetLastError());
    k_dscan_apply<uint8_t><<<DSCAN_BLOCKS, SCAN_THREADS, 0, s>>>(in, n_dev, tmp, out);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

size_t scan_chunks_tmp_elems(int n_chunks)
{
    return 2 * (size_t(n_chunks) + 1) + scan_tmp_elems(n_chunks);
}

int scan_chunks(const BatchChunk *chunks, int n_chunks, const WalkArgs *args, int ng, int64_t *tmp,
                hipStream_t s)
{
    if (ng > 0) {
        k_chunk_empty<<<unsigned((ng + SCAN_THREADS - 1) / SCAN_THREADS), SCAN_THREADS, 0, s>>>(args, ng);
        HG_CHECK(hipGetLastError());
    }
    if (n_chunks <= 0) return HG_OK;
    int64_t *csum = tmp;
    int64_t *cex = tmp + (n_chunks + 1);
    int64_t *stmp = tmp + 2 * (size_t(n_chunks) + 1);
    k_chunk_sums<<<unsigned(n_chunks), SCAN_THREADS, 0, s>>>(chunks, args, csum);
    HG_CHECK(hipGetLastError());
    int rc = scan_impl<int64_t>(csum, cex, n_chunks, stmp, s);
    if (rc) return rc;
    k_chunk_apply<<<unsigned(n_chunks), SCAN_THREADS, 0, s>>>(chunks, args, cex);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

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
