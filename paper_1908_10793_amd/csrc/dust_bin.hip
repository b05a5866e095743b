// Stable counting sort of particles by cell (or tile-major cell) key: an
// LSD radix sort with 8-bit digits over as many passes as the key range
// needs.  Each pass: per-block digit histograms, one exclusive scan over
// (digit, block), and a scatter in which every block ranks its elements
// stably (wave ballots for lanes, LDS counters across waves and chunks).
// Deterministic: no atomics decide an order.
#include "dust_device.h"
#include "dust_launch.h"
#include "dust_particle.h"

namespace dust {

static constexpr int BIN_THREADS = 256;
static constexpr int BIN_ITEMS = 16;
static constexpr int BIN_TILE = BIN_THREADS * BIN_ITEMS;  // elements per block

__global__ void k_make_keys(const int32_t* cell, int64_t n, const Box* boxes, int nbox,
                            uint32_t nbins, int key_mode, TileShape ts, uint32_t* key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t c = cell[i];
  uint32_t k = nbins;
  if (c >= 0 && c < (int64_t)nbins) {
    if (key_mode == DUST_BIN_TILE) {
      int b = find_box(boxes, nbox, c);
      k = tile_key(boxes[b], c - boxes[b].cell_base, ts);
    } else {
      k = (uint32_t)c;
    }
  }
  key[i] = k;
}

__global__ void __launch_bounds__(BIN_THREADS) k_digit_hist(const uint32_t* key, int64_t n,
                                                            int shift, uint32_t* hist,
                                                            int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * BIN_TILE;
  for (int c = 0; c < BIN_ITEMS; ++c) {
    int64_t e = base + c * BIN_THREADS + threadIdx.x;
    if (e < n) atomicAdd(&h[(key[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// One radix pass of one block of BIN_TILE elements: the block's elements
// are first placed in LDS in stable digit order (wave ballots rank lanes with
// equal digits, LDS counters carry the ranks across waves and chunks), then
// written out run by run, so that consecutive threads write consecutive
// addresses of a digit's output range.  val_in = nullptr: values are the
// element indices (first pass).
__global__ void __launch_bounds__(BIN_THREADS) k_digit_scatter(const uint32_t* __restrict__ key_in,
                                                               const uint32_t* __restrict__ val_in,
                                                               int64_t n, int shift,
                                                               const uint32_t* __restrict__ offs,
                                                               int nblocks, uint32_t* key_out,
                                                               uint32_t* val_out) {
  __shared__ uint32_t s_key[BIN_TILE], s_val[BIN_TILE];
  __shared__ uint32_t lstart[256], running[256], gstart[256];
  __shared__ uint32_t cnt[BIN_THREADS / 64][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * BIN_TILE;
  const int nloc = (int)(n - base < BIN_TILE ? n - base : BIN_TILE);
  uint32_t k[BIN_ITEMS], v[BIN_ITEMS];
#pragma unroll
  for (int c = 0; c < BIN_ITEMS; ++c) {
    const int l = c * BIN_THREADS + t;
    const bool valid = l < nloc;
    k[c] = valid ? key_in[base + l] : 0u;
    v[c] = valid ? (val_in ? val_in[base + l] : (uint32_t)(base + l)) : 0u;
  }
  // block histogram of the digit, then its exclusive scan
  running[t] = 0;
  for (int w = 0; w < BIN_THREADS / 64; ++w) cnt[w][t] = 0;
  gstart[t] = offs[(int64_t)t * nblocks + blockIdx.x];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < BIN_ITEMS; ++c)
    if (c * BIN_THREADS + t < nloc) atomicAdd(&running[(k[c] >> shift) & 255u], 1u);
  __syncthreads();
  const uint32_t mine = running[t];
  lstart[t] = mine;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t x = t >= off ? lstart[t - off] : 0u;
    __syncthreads();
    lstart[t] += x;
    __syncthreads();
  }
  lstart[t] -= mine;
  running[t] = lstart[t];
  __syncthreads();
  // stable placement in LDS, chunk by chunk
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int c = 0; c < BIN_ITEMS; ++c) {
    const bool valid = c * BIN_THREADS + t < nloc;
    const uint32_t d = (k[c] >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
    for (int bt = 0; bt < 8; ++bt) {
      const unsigned long long m = __ballot((d >> bt) & 1u);
      peers &= ((d >> bt) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) cnt[wv][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wv; ++w) pos += cnt[w][d];
      s_key[pos] = k[c];
      s_val[pos] = v[c];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < BIN_THREADS / 64; ++w) {
      add += cnt[w][t];
      cnt[w][t] = 0;
    }
    running[t] += add;
    __syncthreads();
  }
  // write out run by run
  for (int p = t; p < nloc; p += BIN_THREADS) {
    const uint32_t kk = s_key[p];
    const uint32_t d = (kk >> shift) & 255u;
    const uint32_t o = gstart[d] + (uint32_t)p - lstart[d];
    key_out[o] = kk;
    val_out[o] = s_val[p];
  }
}

// Exclusive scan of uint32 in place, three-phase with recursion.
static constexpr int SCAN_THREADS = 256;
static constexpr int SCAN_ITEMS = 8;
static constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_block(uint32_t* a, int64_t n,
                                                             uint32_t* block_sums) {
  __shared__ uint32_t s[SCAN_THREADS];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS], tot = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    uint32_t x = v[k];
    v[k] = tot;
    tot += x;
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    uint32_t x = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t excl = s[threadIdx.x] - tot;
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) a[base + k] = v[k] + excl;
  if (threadIdx.x == SCAN_THREADS - 1 && block_sums) block_sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(uint32_t* a, int64_t n, const uint32_t* block_offs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += block_offs[i / SCAN_TILE];
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t bin_blocks(int64_t n) { return ceil_div(n, BIN_TILE); }

size_t bin_scan_tmp_words(int64_t m) {
  size_t words = 0;
  while (m > SCAN_TILE) {
    m = ceil_div(m, SCAN_TILE);
    words += (size_t)m;
  }
  return words + 1;
}

static void scan_exclusive(uint32_t* a, int64_t m, uint32_t* tmp, hipStream_t st) {
  if (m <= 0) return;
  if (m <= SCAN_TILE) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(SCAN_THREADS), 0, st, a, m, (uint32_t*)nullptr);
    return;
  }
  int64_t nb = ceil_div(m, SCAN_TILE);
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, a, m, tmp);
  scan_exclusive(tmp, nb, tmp + nb, st);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, a, m, tmp);
}

__global__ void k_bin_starts(const uint32_t* key, int64_t n, uint32_t nbins, int64_t* start) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t k = key[i];
  int64_t kp = i == 0 ? -1 : (int64_t)key[i - 1];
  for (int64_t b = kp + 1; b <= k && b <= (int64_t)nbins; ++b) start[b] = i;
  if (i == n - 1)
    for (int64_t b = k + 1; b <= (int64_t)nbins; ++b) start[b] = n;
}

__global__ void k_fill_i64(int64_t* a, int64_t n, int64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_copy_perm(const uint32_t* v, int64_t n, int32_t* perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = (int32_t)v[i];
}

int launch_bin(const int32_t* cell, int64_t n, const Box* boxes_dev, int nbox, int64_t nbins,
               int key_mode, TileShape tile, BinWork& w, int32_t* perm_out,
               int64_t* bin_start_out, bool keys_ready, hipStream_t st) {
  if (n == 0) {
    if (bin_start_out)
      hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)ceil_div(nbins + 1, 256)), dim3(256), 0, st,
                         bin_start_out, nbins + 1, (int64_t)0);
    return 0;
  }
  if (!keys_ready)
    hipLaunchKernelGGL(k_make_keys, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, cell, n,
                       boxes_dev, nbox, (uint32_t)nbins, key_mode, tile, w.key[0]);
  int bits = 1;
  while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)nbins) ++bits;
  int npass = (bits + 7) / 8;
  int nblocks = (int)ceil_div(n, BIN_TILE);
  int cur = 0;
  for (int p = 0; p < npass; ++p) {
    int shift = 8 * p;
    hipLaunchKernelGGL(k_digit_hist, dim3(nblocks), dim3(BIN_THREADS), 0, st, w.key[cur], n, shift,
                       w.hist, nblocks);
    scan_exclusive(w.hist, (int64_t)256 * nblocks, w.scan_tmp, st);
    hipLaunchKernelGGL(k_digit_scatter, dim3(nblocks), dim3(BIN_THREADS), 0, st, w.key[cur],
                       p == 0 ? (const uint32_t*)nullptr : (const uint32_t*)w.val[cur], n, shift,
                       w.hist, nblocks, w.key[1 - cur], w.val[1 - cur]);
    cur = 1 - cur;
  }
  if (perm_out)
    hipLaunchKernelGGL(k_copy_perm, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, w.val[cur], n,
                       perm_out);
  if (bin_start_out)
    hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, w.key[cur], n,
                       (uint32_t)nbins, bin_start_out);
  return cur;
}

template <int BYTES> struct Blob { unsigned char b[BYTES]; };

template <typename T>
__global__ void k_permute(const T* in, T* out, const uint32_t* perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

void launch_permute(const void* in, void* out, const uint32_t* perm, int64_t n, int bytes,
                    hipStream_t st) {
  if (n == 0) return;
  unsigned g = (unsigned)ceil_div(n, 256);
  if (bytes == 1)
    hipLaunchKernelGGL(k_permute<uint8_t>, dim3(g), dim3(256), 0, st, (const uint8_t*)in,
                       (uint8_t*)out, perm, n);
  else if (bytes == 4)
    hipLaunchKernelGGL(k_permute<uint32_t>, dim3(g), dim3(256), 0, st, (const uint32_t*)in,
                       (uint32_t*)out, perm, n);
  else
    hipLaunchKernelGGL(k_permute<uint64_t>, dim3(g), dim3(256), 0, st, (const uint64_t*)in,
                       (uint64_t*)out, perm, n);
}

}  // namespace dust
